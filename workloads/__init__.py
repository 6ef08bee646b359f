"""Seeded synthetic inputs with the shapes of the paper's problem classes.

This module only discretises PDEs and draws random numbers.  It holds none of
the root-node method's arithmetic (no strength, aggregation, pattern,
tentative operator or energy minimisation), so both the CPU oracle and the HIP
path can take their inputs from here without sharing any of the method.

Problem classes (the paper's own meshes are not available; these are stand-ins
of the same class, stencil and size):

* ``poisson5``      -- 5-point finite-difference Laplacian, Dirichlet nodes
                       eliminated (the 2D model problem of the background
                       section).
* ``q1_aniso``      -- bilinear (Q1) finite elements for the rotated anisotropic
                       diffusion operator -div(Q^T D Q grad u), D = diag(1, eps),
                       of the totally-anisotropic-diffusion experiment.
* ``upwind_cd``     -- first-order upwind finite differences for
                       b.grad u - eps Laplace u (a non-symmetric stand-in for the
                       recirculating-flow / transport experiments).
* ``q1_elasticity`` -- Q1 plane-strain linear elasticity with one side clamped
                       (the elasticity experiment's equation), node-blocked.
* ``laplace1d``     -- the 8-node 1D Laplacian of the worked SA example.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "BSR", "stencil_grid", "poisson5", "laplace1d", "q1_stencil",
    "q1_aniso", "upwind_cd", "q1_elasticity", "rbm", "ones",
    "aniso_batch_params", "aniso_batch", "loss_weights", "config", "laplace27", "ring_graph",
]


@dataclass
class CSR:
    """Compressed sparse row matrix: int32 indices (sorted, unique), fp64 values."""
    n_rows: int
    n_cols: int
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n_rows, self.n_cols))
        for i in range(self.n_rows):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            d[i, self.colind[s:e]] += self.vals[s:e]
        return d


@dataclass
class BSR:
    """Node-blocked sparse row matrix with m x m blocks (row-major inside a block).

    Row I / column J of the block structure are nodes; scalar DOF of node I and
    component c is m*I + c.
    """
    n_nodes: int
    m: int
    rowptr: np.ndarray
    colind: np.ndarray
    vals: np.ndarray  # [nnzb, m, m]

    @property
    def nnzb(self) -> int:
        return int(self.rowptr[-1])

    def to_csr(self) -> CSR:
        """Scalar CSR with the same stored entries (explicit zeros kept)."""
        m, nn = self.m, self.n_nodes
        nb = np.diff(self.rowptr).astype(np.int64)
        # scalar row m*I+c holds, for each block (I,J) in order, m entries m*J+c'
        rows_len = np.repeat(nb * m, m)
        rowptr = np.zeros(nn * m + 1, dtype=np.int64)
        np.cumsum(rows_len, out=rowptr[1:])
        colind = np.empty(rowptr[-1], dtype=np.int32)
        vals = np.empty(rowptr[-1])
        # vectorised fill: for block b in row I, scalar row m*I+c, offset
        blk_row = np.repeat(np.arange(nn), nb)
        blk_pos = np.arange(self.nnzb) - self.rowptr[blk_row]
        for c in range(m):
            base = rowptr[m * blk_row + c] + blk_pos * m
            for cc in range(m):
                colind[base + cc] = m * self.colind + cc
                vals[base + cc] = self.vals[:, c, cc]
        return CSR(nn * m, nn * m, rowptr.astype(np.int32), colind, vals)


def _csr_from_offsets(nx: int, ny: int, offsets, values) -> CSR:
    """Constant stencil on an nx-by-ny node grid (node = j*nx + i).

    Every stencil offset that stays inside the grid is stored (structural
    entries, even when the value is 0); neighbours outside the grid are
    Dirichlet nodes that have been eliminated.
    """
    offsets = list(offsets)
    order = sorted(range(len(offsets)), key=lambda q: (offsets[q][1], offsets[q][0]))
    offsets = [offsets[q] for q in order]
    values = np.asarray([values[q] for q in order], dtype=np.float64)
    n = nx * ny
    ii, jj = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ii = ii.ravel()
    jj = jj.ravel()
    cols = np.empty((n, len(offsets)), dtype=np.int64)
    valid = np.empty((n, len(offsets)), dtype=bool)
    for q, (dx, dy) in enumerate(offsets):
        i2, j2 = ii + dx, jj + dy
        valid[:, q] = (i2 >= 0) & (i2 < nx) & (j2 >= 0) & (j2 < ny)
        cols[:, q] = j2 * nx + i2
    counts = valid.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    colind = cols[valid].astype(np.int32)
    vals = np.broadcast_to(values, (n, len(offsets)))[valid].copy()
    return CSR(n, n, rowptr.astype(np.int32), colind, vals)


def stencil_grid(nx: int, ny: int, stencil: dict) -> CSR:
    """CSR for ``stencil`` ({(dx, dy): value}) on an nx-by-ny grid."""
    offs = list(stencil.keys())
    return _csr_from_offsets(nx, ny, offs, [stencil[o] for o in offs])


def poisson5(nx: int, ny: int | None = None) -> CSR:
    """Unscaled 5-point Laplacian [-1; -1 4 -1; -1] (integer entries)."""
    ny = nx if ny is None else ny
    return stencil_grid(nx, ny, {(0, 0): 4.0, (-1, 0): -1.0, (1, 0): -1.0,
                                 (0, -1): -1.0, (0, 1): -1.0})


def laplace27(nx: int) -> CSR:
    """27-point 3D Laplacian on an nx^3 grid: 26 on the diagonal, -1 to every
    neighbour of the 3x3x3 box (Dirichlet nodes eliminated)."""
    n = nx ** 3
    idx = np.arange(n)
    x, y, z = idx % nx, (idx // nx) % nx, idx // (nx * nx)
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                ok = (x + dx >= 0) & (x + dx < nx) & (y + dy >= 0) & (y + dy < nx) & (z + dz >= 0) & (z + dz < nx)
                r = idx[ok]
                rows.append(r)
                cols.append(r + dx + nx * dy + nx * nx * dz)
                vals.append(np.full(r.size, 26.0 if (dx, dy, dz) == (0, 0, 0) else -1.0))
    rows, cols, vals = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.add.at(rowptr, rows + 1, 1)
    return CSR(n, n, np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def ring_graph(n: int, offsets=(1, 4100, 9001, 13007)) -> CSR:
    """Graph Laplacian of a circulant graph: node i joined to i +- o (mod n) for
    each offset o, weight -1, diagonal = degree + 1 (symmetric positive
    definite).  Neighbours far apart in the numbering give an irregular
    column structure (no short runs of neighbour rows)."""
    idx = np.arange(n)
    rows, cols = [idx], [idx]
    for o in offsets:
        for s in (o, -o):
            rows.append(idx)
            cols.append((idx + s) % n)
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    key = np.unique(rows.astype(np.int64) * n + cols)
    rows, cols = (key // n).astype(np.int64), (key % n).astype(np.int64)
    vals = np.where(rows == cols, 0.0, -1.0)
    deg = np.bincount(rows, weights=(rows != cols).astype(np.float64), minlength=n)
    vals[rows == cols] = deg + 1.0
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    return CSR(n, n, np.cumsum(rowptr).astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def laplace1d(n: int = 8) -> CSR:
    """1D Laplacian tridiag(-1, 2, -1) on n nodes."""
    return stencil_grid(n, 1, {(0, 0): 2.0, (-1, 0): -1.0, (1, 0): -1.0})


# --- bilinear finite elements -------------------------------------------------
_GP = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
_CORNERS = ((0, 0), (1, 0), (1, 1), (0, 1))


def _q1_grads(xi: float, eta: float) -> np.ndarray:
    """Gradients of the four bilinear shape functions on the unit square."""
    g = np.empty((4, 2))
    for a, (cx, cy) in enumerate(_CORNERS):
        sx = xi if cx else 1.0 - xi
        sy = eta if cy else 1.0 - eta
        dsx = 1.0 if cx else -1.0
        dsy = 1.0 if cy else -1.0
        g[a, 0] = dsx * sy
        g[a, 1] = sx * dsy
    return g


def q1_element_diffusion(K: np.ndarray) -> np.ndarray:
    """4x4 element matrix of int grad(phi_a)^T K grad(phi_b) on a unit square.

    2x2 Gauss quadrature is exact here.  In 2D the matrix does not depend on
    the element size h.
    """
    Ke = np.zeros((4, 4))
    for xi in _GP:
        for eta in _GP:
            g = _q1_grads(xi, eta)
            Ke += 0.25 * g @ K @ g.T
    return Ke


def q1_stencil(eps: float, psi: float) -> dict:
    """Interior 9-point stencil of Q1 for -div(Q^T D Q grad u), D = diag(1, eps)."""
    c, s = math.cos(psi), math.sin(psi)
    Q = np.array([[c, -s], [s, c]])
    D = np.diag([1.0, eps])
    Ke = q1_element_diffusion(Q.T @ D @ Q)
    st = {}
    for a, pa in enumerate(_CORNERS):
        for b, pb in enumerate(_CORNERS):
            off = (pb[0] - pa[0], pb[1] - pa[1])
            st[off] = st.get(off, 0.0) + Ke[a, b]
    return st


def q1_aniso(nx: int, eps: float = 1e-3, psi: float = math.pi / 8, ny: int | None = None) -> CSR:
    """Q1 rotated anisotropic diffusion on nx*ny interior nodes of a uniform mesh."""
    ny = nx if ny is None else ny
    return stencil_grid(nx, ny, q1_stencil(eps, psi))


def upwind_cd(nx: int, eps: float = 1e-4, angle: float = 3 * math.pi / 16) -> CSR:
    """First-order upwind FD for b.grad u - eps Laplace u, times h^2, h = 1/(nx+1).

    b = (cos angle, sin angle) has positive components, so the upwind
    differences are backward differences in x and y.
    """
    h = 1.0 / (nx + 1)
    b1, b2 = math.cos(angle), math.sin(angle)
    st = {(0, 0): 4 * eps + h * (b1 + b2),
          (-1, 0): -(eps + h * b1), (0, -1): -(eps + h * b2),
          (1, 0): -eps, (0, 1): -eps}
    return stencil_grid(nx, nx, st)


def _q1_element_elasticity(lam: float, mu: float) -> np.ndarray:
    """8x8 plane-strain Q1 element stiffness (DOF 2*a + comp) on a unit square."""
    C = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0], [0.0, 0.0, mu]])
    Ke = np.zeros((8, 8))
    for xi in _GP:
        for eta in _GP:
            g = _q1_grads(xi, eta)
            Bm = np.zeros((3, 8))
            Bm[0, 0::2] = g[:, 0]
            Bm[1, 1::2] = g[:, 1]
            Bm[2, 0::2] = g[:, 1]
            Bm[2, 1::2] = g[:, 0]
            Ke += 0.25 * Bm.T @ C @ Bm
    return Ke


def q1_elasticity(nx: int, ny: int | None = None, E: float = 1.0, nu: float = 0.3):
    """Q1 plane-strain elasticity, node-blocked 2x2.

    Mesh nodes sit at (i*h, j*h), i = 0..nx, j = 0..ny-1, h = 1/nx.  The west
    column i = 0 is clamped and eliminated; all other sides are traction free.
    Free node (i, j) has index j*nx + (i-1).  Returns (BSR, coords[n_nodes, 2]).
    """
    ny = nx if ny is None else ny
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    Ke = _q1_element_elasticity(lam, mu)
    ei, ej = np.meshgrid(np.arange(nx), np.arange(ny - 1), indexing="xy")
    ei, ej = ei.ravel(), ej.ravel()
    nn = nx * ny
    rows, cols, blocks = [], [], []
    for a, (ax, ay) in enumerate(_CORNERS):
        for b, (bx, by) in enumerate(_CORNERS):
            ia, ja = ei + ax, ej + ay
            ib, jb = ei + bx, ej + by
            ok = (ia >= 1) & (ib >= 1)
            rows.append((ja * nx + ia - 1)[ok])
            cols.append((jb * nx + ib - 1)[ok])
            blocks.append(np.broadcast_to(Ke[2 * a:2 * a + 2, 2 * b:2 * b + 2], (int(ok.sum()), 2, 2)))
    r = np.concatenate(rows).astype(np.int64)
    c = np.concatenate(cols).astype(np.int64)
    v = np.concatenate(blocks)
    key = r * nn + c
    uk, inv = np.unique(key, return_inverse=True)
    vb = np.zeros((uk.size, 2, 2))
    np.add.at(vb, inv, v)
    br = (uk // nn).astype(np.int64)
    bc = (uk % nn).astype(np.int32)
    rowptr = np.zeros(nn + 1, dtype=np.int64)
    np.cumsum(np.bincount(br, minlength=nn), out=rowptr[1:])
    h = 1.0 / nx
    jj, ii = np.divmod(np.arange(nn), nx)
    coords = np.stack([(ii + 1) * h, jj * h], axis=1)
    return BSR(nn, 2, rowptr.astype(np.int32), bc, vb), coords


def rbm(coords: np.ndarray) -> np.ndarray:
    """2D rigid-body modes [t_x, t_y, r], r = (-y, x), interleaved DOF 2*node+comp."""
    nn = coords.shape[0]
    B = np.zeros((2 * nn, 3))
    B[0::2, 0] = 1.0
    B[1::2, 1] = 1.0
    B[0::2, 2] = -coords[:, 1]
    B[1::2, 2] = coords[:, 0]
    return B


def ones(n: int) -> np.ndarray:
    """The constant candidate, shape (n, 1)."""
    return np.ones((n, 1))


# --- batched anisotropic problems ---------------------------------------------
def aniso_batch_params(batch: int = 16, seed: int = 0):
    """(eps_b, psi_b): eps = 10^U(-3, 0), psi = U(0, pi), drawn in that order per b."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(batch):
        e = 10.0 ** rng.uniform(-3.0, 0.0)
        p = rng.uniform(0.0, math.pi)
        out.append((e, p))
    return out, rng


def aniso_batch(nx: int, batch: int = 16, seed: int = 0):
    """Batch of Q1 anisotropic problems sharing one 9-point structure.

    Returns (structure CSR of problem 0, values [batch, nnz], params, rng); the
    rng continues the same stream so loss weights can be drawn from it.
    """
    params, rng = aniso_batch_params(batch, seed)
    mats = [q1_aniso(nx, e, p) for (e, p) in params]
    vals = np.stack([m.vals for m in mats])
    return mats[0], vals, params, rng


def loss_weights(rng: np.random.Generator, batch: int, nnz_n: int) -> np.ndarray:
    """W_b ~ N(0, 1) over the pattern entries, drawn after the problem parameters."""
    return rng.standard_normal((batch, nnz_n))


# --- named configurations ------------------------------------------------------
def config(name: str, scale: int | None = None):
    """Inputs of a named workload.

    Returns a dict with keys: A (CSR), Ab (BSR or None), B, Bhat (or None),
    m, theta, degree, iters, method, and for the batched case vals/W params.
    ``scale`` overrides the grid edge (small cases for tests).
    """
    if name == "poisson32":
        nx = scale or 32
        A = poisson5(nx)
        return dict(A=A, Ab=None, B=ones(A.n_rows), Bhat=None, m=1, theta=0.25,
                    degree=2, iters=4, method="cg")
    if name == "aniso512":
        nx = scale or 512
        A = q1_aniso(nx, 1e-3, math.pi / 8)
        return dict(A=A, Ab=None, B=ones(A.n_rows), Bhat=None, m=1, theta=0.1,
                    degree=2, iters=6, method="cg")
    if name == "upwind1024":
        nx = scale or 1024
        A = upwind_cd(nx)
        return dict(A=A, Ab=None, B=ones(A.n_rows), Bhat=ones(A.n_rows), m=1,
                    theta=0.0, degree=2, iters=8, method="gmres")
    if name == "elastic512":
        nx = scale or 512
        Ab, coords = q1_elasticity(nx)
        A = Ab.to_csr()
        return dict(A=A, Ab=Ab, B=rbm(coords), Bhat=None, m=2, theta=0.0,
                    degree=2, iters=6, method="cg")
    if name == "aniso_batch256":
        nx = scale or 256
        A0, vals, params, rng = aniso_batch(nx, 16, 0)
        return dict(A=A0, Ab=None, B=ones(A0.n_rows), Bhat=None, m=1, theta=0.0,
                    degree=2, iters=6, method="cg", batch_vals=vals,
                    params=params, rng=rng)
    raise KeyError(name)
