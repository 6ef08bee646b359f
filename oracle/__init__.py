"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg use it; the product path never does.  Every function follows
the paper step by step (see oracle.c for the passage each one follows).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

ORC_OK, ORC_ECAP, ORC_ESINGULAR, ORC_EBREAKDOWN, ORC_ENONFINITE, ORC_EINVAL = 0, -1, -2, -3, -4, -5

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        i, d, vp = C.c_int, C.c_double, C.c_void_p
        L.orc_set_threads.argtypes = [i]
        L.orc_threads.restype = i
        L.orc_strength.argtypes = [i, _i32p, _i32p, _f64p, i, d, _i32p, _i32p, i]
        L.orc_aggregate.argtypes = [i, _i32p, _i32p, _i32p, _i32p]
        L.orc_pattern_nodes.argtypes = [i, _i32p, _i32p, _i32p, i, i, _i32p, _i32p, i]
        L.orc_pattern_dofs.argtypes = [i, i, _i32p, _i32p, _i32p, _i32p, i, _i32p, _i32p, i, _u8p]
        L.orc_tentative.argtypes = [i, i, _i32p, _i32p, _u8p, _i32p, _i32p, i, _f64p, i, _f64p, _f64p, C.POINTER(C.c_int)]
        L.orc_gram_pinv.argtypes = [i, _f64p, _f64p]
        L.orc_gram_rows.argtypes = [i, _i32p, _i32p, _u8p, _f64p, i, _f64p]
        L.orc_project.argtypes = [i, _i32p, _i32p, _u8p, _f64p, i, _f64p, _f64p]
        L.orc_masked_product.argtypes = [i, i, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p, _f64p]
        L.orc_emin_cg.argtypes = [i, i, _i32p, _i32p, _f64p, _i32p, _i32p, _u8p, _f64p, i, _f64p, i, _f64p,
                                  _f64p, _f64p, _f64p, C.POINTER(C.c_int)]
        L.orc_emin_gmres.argtypes = [i, i, _i32p, _i32p, _f64p, _i32p, _i32p, _u8p, _f64p, i, _f64p, i, _f64p,
                                     _f64p, C.POINTER(C.c_int)]
        L.orc_emin_cg_jvp.argtypes = [i, i, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p, _u8p, _f64p, i, _f64p, i,
                                      _f64p, _f64p]
        L.orc_transpose.argtypes = [i, i, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
        L.orc_energy.argtypes = [i, i, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
        L.orc_energy.restype = d
        L.orc_constraint_residual.argtypes = [i, _i32p, _i32p, _f64p, _f64p, _f64p, i]
        L.orc_constraint_residual.restype = d
        L.orc_enforce.argtypes = [i, _i32p, _i32p, _u8p, _f64p, i, _f64p, _f64p]
        L.orc_filter.argtypes = [i, i, _i32p, _i32p, _f64p, vp, _i32p, i, d, _u8p]
        L.orc_compact.argtypes = [i, _i32p, _i32p, vp, _u8p, _i32p, _i32p, vp]
        L.orc_strength_values.argtypes = [i, _i32p, _i32p, _f64p, i, d, _i32p, _i32p, _f64p]
        L.orc_smooth_candidates.argtypes = [i, _i32p, _i32p, _f64p, _f64p, i, i, d]
        L.orc_emin_pcg.argtypes = L.orc_emin_cg.argtypes
        L.orc_emin_cgnr.argtypes = L.orc_emin_cg.argtypes
        L.orc_spgemm.argtypes = [i, i, i, _i32p, _i32p, vp, _i32p, _i32p, vp, _i32p, _i32p, vp, C.c_long]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n: int) -> None:
    """Threads of the oracle's row and entry loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def threads() -> int:
    return int(lib().orc_threads())


def strength(Ap, Aj, Ax, m, theta):
    """Nodal strength graph (Sp, Sj), diagonal included, symmetrised."""
    Ap, Aj, Ax = _i32(Ap), _i32(Aj), _f64(Ax)
    n = Ap.size - 1
    nn = n // m
    cap = 2 * int(Ap[-1]) + nn
    Sp = np.zeros(nn + 1, np.int32)
    Sj = np.zeros(max(cap, 1), np.int32)
    rc = lib().orc_strength(n, Ap, Aj, Ax, m, float(theta), Sp, Sj, cap)
    if rc < 0:
        raise OracleError(rc, "strength")
    return Sp, Sj[:rc].copy()


def aggregate(Sp, Sj):
    """Greedy root-node aggregation: (agg[nn], roots[n_agg])."""
    Sp, Sj = _i32(Sp), _i32(Sj)
    nn = Sp.size - 1
    agg = np.zeros(nn, np.int32)
    roots = np.zeros(max(nn, 1), np.int32)
    na = lib().orc_aggregate(nn, Sp, Sj, agg, roots)
    return agg, roots[:na].copy()


def pattern_nodes(Sp, Sj, agg, n_agg, d):
    Sp, Sj, agg = _i32(Sp), _i32(Sj), _i32(agg)
    nn = Sp.size - 1
    cap = max(nn, 1)
    while True:
        Np = np.zeros(nn + 1, np.int32)
        Nj = np.zeros(cap, np.int32)
        rc = lib().orc_pattern_nodes(nn, Sp, Sj, agg, int(n_agg), int(d), Np, Nj, cap)
        if rc == ORC_ECAP:
            cap *= 4
            continue
        if rc < 0:
            raise OracleError(rc, "pattern_nodes")
        return Np, Nj[:rc].copy()


def pattern_dofs(Npn, Njn, agg, roots, m):
    Npn, Njn, agg, roots = _i32(Npn), _i32(Njn), _i32(agg), _i32(roots)
    nn = Npn.size - 1
    cap = max(int(Npn[-1]) * m * m + nn * m, 1)
    Np = np.zeros(nn * m + 1, np.int32)
    Nj = np.zeros(cap, np.int32)
    is_root = np.zeros(nn * m, np.uint8)
    rc = lib().orc_pattern_dofs(nn, m, Npn, Njn, agg, roots, int(roots.size), Np, Nj, cap, is_root)
    if rc < 0:
        raise OracleError(rc, "pattern_dofs")
    return Np, Nj[:rc].copy(), is_root


def tentative(Np, Nj, is_root, agg, roots, m, B):
    """(T on N, Bc [m*n_agg, nB], rank-deficient row count)."""
    Np, Nj, agg, roots = _i32(Np), _i32(Nj), _i32(agg), _i32(roots)
    B = _f64(B)
    n, nB = B.shape
    T = np.zeros(int(Np[-1]))
    Bc = np.zeros((m * roots.size, nB))
    rd = C.c_int(0)
    rc = lib().orc_tentative(n, m, Np, Nj, np.ascontiguousarray(is_root, np.uint8), agg, roots,
                             int(roots.size), B, nB, T, Bc, C.byref(rd))
    if rc < 0:
        raise OracleError(rc, "tentative")
    return T, Bc, rd.value


def gram_pinv(G):
    G = _f64(G)
    nB = G.shape[0]
    Gp = np.zeros_like(G)
    fb = lib().orc_gram_pinv(nB, G.ravel().copy(), Gp.ravel())
    return Gp, bool(fb)


def gram_rows(Np, Nj, is_root, Bc, nB):
    n = Np.size - 1
    Gp = np.zeros(max(n * nB * nB, 1))
    bad = lib().orc_gram_rows(n, _i32(Np), _i32(Nj), np.ascontiguousarray(is_root, np.uint8),
                              _f64(Bc).ravel() if nB else np.zeros(1), nB, Gp)
    return Gp, bad


def project(Np, Nj, is_root, Bc, nB, X):
    """Pi = Pi_B o M applied to a copy of X."""
    Gp, _ = gram_rows(Np, Nj, is_root, Bc, nB)
    X = _f64(X).copy()
    lib().orc_project(Np.size - 1, _i32(Np), _i32(Nj), np.ascontiguousarray(is_root, np.uint8),
                      _f64(Bc).ravel() if nB else np.zeros(1), nB, Gp, X)
    return X


def masked_product(Ap, Aj, Ax, Np, Nj, nc, X):
    n = Np.size - 1
    Z = np.zeros(int(Np[-1]))
    lib().orc_masked_product(n, int(nc), _i32(Ap), _i32(Aj), _f64(Ax), _i32(Np), _i32(Nj), _f64(X), Z)
    return Z


def emin_cg(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K, variant="cg"):
    """K CG steps (variant "cg", Jacobi-preconditioned "pcg", or the normal
    equations "cgnr"); returns (P, info) with gamma/delta/alpha histories."""
    fn = {"cg": lib().orc_emin_cg, "pcg": lib().orc_emin_pcg, "cgnr": lib().orc_emin_cgnr}[variant]
    n = Np.size - 1
    P = np.zeros(int(Np[-1]))
    gam = np.zeros(K + 1)
    dl = np.zeros(max(K, 1))
    al = np.zeros(max(K, 1))
    it = C.c_int(0)
    rc = fn(n, int(nc), _i32(Ap), _i32(Aj), _f64(Ax), _i32(Np), _i32(Nj),
                           np.ascontiguousarray(is_root, np.uint8),
                           _f64(Bc).ravel() if nB else np.zeros(1), nB, _f64(T), int(K), P,
                           gam, dl, al, C.byref(it))
    return P, dict(status=rc, iters=it.value, gamma=gam, delta=dl[:K], alpha=al[:K])


def emin_cg_jvp(Ap, Aj, Ax, dAx, Np, Nj, is_root, nc, Bc, nB, T, K):
    n = Np.size - 1
    P = np.zeros(int(Np[-1]))
    dP = np.zeros(int(Np[-1]))
    rc = lib().orc_emin_cg_jvp(n, int(nc), _i32(Ap), _i32(Aj), _f64(Ax), _f64(dAx), _i32(Np), _i32(Nj),
                               np.ascontiguousarray(is_root, np.uint8),
                               _f64(Bc).ravel() if nB else np.zeros(1), nB, _f64(T), int(K), P, dP)
    if rc < 0:
        raise OracleError(rc, "emin_cg_jvp")
    return P, dP


def emin_gmres(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K):
    n = Np.size - 1
    P = np.zeros(int(Np[-1]))
    res = np.zeros(K + 1)
    it = C.c_int(0)
    rc = lib().orc_emin_gmres(n, int(nc), _i32(Ap), _i32(Aj), _f64(Ax), _i32(Np), _i32(Nj),
                              np.ascontiguousarray(is_root, np.uint8),
                              _f64(Bc).ravel() if nB else np.zeros(1), nB, _f64(T), int(K), P,
                              res, C.byref(it))
    return P, dict(status=rc, iters=it.value, resid=res)


def transpose(Ap, Aj, Ax, n_cols=None):
    Ap, Aj, Ax = _i32(Ap), _i32(Aj), _f64(Ax)
    nr = Ap.size - 1
    nc = nr if n_cols is None else n_cols
    Tp = np.zeros(nc + 1, np.int32)
    Tj = np.zeros(max(int(Ap[-1]), 1), np.int32)
    Tx = np.zeros(max(int(Ap[-1]), 1))
    lib().orc_transpose(nr, nc, Ap, Aj, Ax, Tp, Tj, Tx)
    return Tp, Tj[:Ap[-1]].copy(), Tx[:Ap[-1]].copy()


def energy(Ap, Aj, Ax, Np, Nj, nc, P):
    return lib().orc_energy(Np.size - 1, int(nc), _i32(Ap), _i32(Aj), _f64(Ax), _i32(Np), _i32(Nj), _f64(P))


def constraint_residual(Np, Nj, P, Bc, B):
    B = _f64(B)
    return lib().orc_constraint_residual(Np.size - 1, _i32(Np), _i32(Nj), _f64(P), _f64(Bc).ravel(),
                                         B.ravel(), B.shape[1])


def setup(A, B, m=1, theta=0.0, degree=2, agg=None, roots=None):
    """Strength -> aggregation -> pattern -> tentative for a CSR-like A.

    Returns a dict with S, agg, roots, nodal and DOF pattern, is_root, T, Bc.
    """
    Sp, Sj = strength(A.rowptr, A.colind, A.vals, m, theta)
    if agg is None:
        agg, roots = aggregate(Sp, Sj)
    Npn, Njn = pattern_nodes(Sp, Sj, agg, roots.size, degree)
    Np, Nj, is_root = pattern_dofs(Npn, Njn, agg, roots, m)
    T, Bc, rd = tentative(Np, Nj, is_root, agg, roots, m, B)
    return dict(Sp=Sp, Sj=Sj, agg=agg, roots=roots, Npn=Npn, Njn=Njn, Np=Np, Nj=Nj,
                is_root=is_root, T=T, Bc=Bc, nc=m * roots.size, rank_def=rd)


def enforce(Np, Nj, is_root, Bc, B, V):
    """Eq. Tproj on every F row of a copy of V: (values, rank-deficient rows)."""
    B = _f64(B)
    V = _f64(V).copy()
    rc = lib().orc_enforce(Np.size - 1, _i32(Np), _i32(Nj), np.ascontiguousarray(is_root, np.uint8),
                           _f64(Bc).ravel(), B.shape[1], B.ravel(), V)
    if rc < 0:
        raise OracleError(rc, "enforce")
    return V, rc


def filter_keep(Np, Nj, G, agg, m=1, k=0, theta=0.0, is_root=None):
    """Alg. filter on node blocks: the keep mask of every stored entry."""
    Np, Nj = _i32(Np), _i32(Nj)
    keep = np.zeros(max(int(Np[-1]), 1), np.uint8)
    ir = None if is_root is None else np.ascontiguousarray(is_root, np.uint8)
    rc = lib().orc_filter(Np.size - 1, int(m), Np, Nj, _f64(G), None if ir is None else ir.ctypes.data,
                          _i32(agg), int(k), float(theta), keep)
    if rc < 0:
        raise OracleError(rc, "filter")
    return keep[:int(Np[-1])].astype(bool)


def compact(Np, Nj, keep, V=None):
    """(Np2, Nj2, V2) of the kept entries."""
    Np, Nj = _i32(Np), _i32(Nj)
    kp = np.ascontiguousarray(keep, np.uint8)
    Np2 = np.zeros(Np.size, np.int32)
    Nj2 = np.zeros(max(int(kp.sum()), 1), np.int32)
    V2 = np.zeros(max(int(kp.sum()), 1)) if V is not None else None
    Vin = None if V is None else _f64(V)
    w = lib().orc_compact(Np.size - 1, Np, Nj, None if Vin is None else Vin.ctypes.data, kp, Np2, Nj2,
                          None if V2 is None else V2.ctypes.data)
    return Np2, Nj2[:w].copy(), (V2[:w].copy() if V2 is not None else None)


def postfilter(Ap, Aj, Ax, Np, Nj, is_root, agg, m, nc, Bc, B, P, k=0, theta=0.0, method="cg", iters=1):
    """The post-filter lines of Alg. root_node_setup (Sec. 3.7): filter P,
    enforce P Bc = B with Eq. Tproj, then `iters` more energy-minimisation
    steps from the enforced P on the filtered pattern.  Returns
    (Np2, Nj2, P_filtered_enforced, P_final, info)."""
    keep = filter_keep(Np, Nj, P, agg, m, k, theta, is_root)
    Np2, Nj2, Pf = compact(Np, Nj, keep, P)
    Pe, rd = enforce(Np2, Nj2, is_root, Bc, B, Pf)
    nB = _f64(B).shape[1]
    fn = emin_cg if method == "cg" else emin_gmres
    Pn, info = fn(Ap, Aj, Ax, Np2, Nj2, is_root, nc, Bc, nB, Pe, iters)
    info["rank_def"] = rd
    return Np2, Nj2, Pe, Pn, info


def spgemm(Xp, Xj, Xx, Yp, Yj, Yx, cols):
    """C = X Y (CSR): (Cp, Cj, Cx); Xx or Yx None gives the structure only."""
    Xp, Xj, Yp, Yj = _i32(Xp), _i32(Xj), _i32(Yp), _i32(Yj)
    rows = Xp.size - 1
    xv = None if Xx is None else _f64(Xx)
    yv = None if Yx is None else _f64(Yx)
    cap = 1024
    while True:
        Cp = np.zeros(rows + 1, np.int32)
        Cj = np.zeros(cap, np.int32)
        Cx = np.zeros(cap)
        rc = lib().orc_spgemm(rows, Yp.size - 1, int(cols), Xp, Xj, None if xv is None else xv.ctypes.data, Yp, Yj,
                              None if yv is None else yv.ctypes.data, Cp, Cj,
                              Cx.ctypes.data if (xv is not None and yv is not None) else None, cap)
        if rc == ORC_ECAP:
            cap *= 4
            continue
        if rc < 0:
            raise OracleError(rc, "spgemm")
        return Cp, Cj[:rc].copy(), (Cx[:rc].copy() if (xv is not None and yv is not None) else None)


def galerkin(Ap, Aj, Ax, Pp, Pj, Px, nc, RTp=None, RTj=None, RTx=None):
    """The coarse operator of Sec. 3.8, A_c = R (A P), with R = P^T for a
    symmetric A, or R = (R^T)^T from the given R^T (n x nc, CSR)."""
    n = Pp.size - 1
    APp, APj, APx = spgemm(Ap, Aj, Ax, Pp, Pj, Px, nc)
    if RTp is None:
        RTp, RTj, RTx = Pp, Pj, Px
    Rp, Rj, Rx = transpose(RTp, RTj, RTx, n_cols=nc)
    return spgemm(Rp, Rj, Rx, APp, APj, APx, nc)


def strength_values(Ap, Aj, Ax, m, theta, Sp, Sj):
    """Eq. soc values of the node graph S (Sp, Sj) from orc_strength."""
    Sx = np.zeros(max(int(Sp[-1]), 1))
    rc = lib().orc_strength_values(_i32(Ap).size - 1, _i32(Ap), _i32(Aj), _f64(Ax), int(m), float(theta), _i32(Sp),
                                   _i32(Sj), Sx)
    if rc < 0:
        raise OracleError(rc, "strength_values")
    return Sx[:int(Sp[-1])].copy()


def pattern_values(Sp, Sj, Sx, agg, n_agg, d):
    """N = S^d C with values (Sec. 3.4 with the normalised S of Eq. soc): X_0 = C,
    X_{t+1} = S X_t as sparse products.  Returns (Np, Nj, Nx) on node rows."""
    nn = _i32(Sp).size - 1
    Xp, Xj, Xx = np.arange(nn + 1, dtype=np.int32), _i32(agg).copy(), np.ones(nn)
    for _ in range(d):
        Xp, Xj, Xx = spgemm(Sp, Sj, Sx, Xp, Xj, Xx, n_agg)
    return Xp, Xj, Xx


def prefilter_setup(A, B, m, theta, degree, k=0, theta_f=0.0, agg=None, roots=None):
    """The lines of Alg. root_node_setup up to inject with the pre-filter
    (Sec. 3.5): strength, aggregation, N = S^d C with Eq. soc values, filter
    of N (node rows, own aggregate as the diagonal), unamalgamate, root rows,
    tentative.  Returns the dict of setup() plus the nodal valued pattern."""
    Sp, Sj = strength(A.rowptr, A.colind, A.vals, m, theta)
    if agg is None:
        agg, roots = aggregate(Sp, Sj)
    Sx = strength_values(A.rowptr, A.colind, A.vals, m, theta, Sp, Sj)
    Vp, Vj, Vx = pattern_values(Sp, Sj, Sx, agg, roots.size, degree)
    keep = filter_keep(Vp, Vj, Vx, agg, 1, k, theta_f)
    Npn, Njn, _ = compact(Vp, Vj, keep, Vx)
    Np, Nj, is_root = pattern_dofs(Npn, Njn, agg, roots, m)
    T, Bc, rd = tentative(Np, Nj, is_root, agg, roots, m, B)
    return dict(Sp=Sp, Sj=Sj, Sx=Sx, agg=agg, roots=roots, Vp=Vp, Vj=Vj, Vx=Vx, Npn=Npn, Njn=Njn, Np=Np, Nj=Nj,
                is_root=is_root, T=T, Bc=Bc, nc=m * roots.size, rank_def=rd)


def smooth_candidates(Ap, Aj, Ax, B, sweeps, omega):
    """`sweeps` damped Jacobi sweeps on A B = 0 applied to a copy of B."""
    B = _f64(B).copy()
    if B.ndim == 1:
        B = B[:, None].copy()
    rc = lib().orc_smooth_candidates(_i32(Ap).size - 1, _i32(Ap), _i32(Aj), _f64(Ax), B, B.shape[1], int(sweeps),
                                     float(omega))
    if rc < 0:
        raise OracleError(rc, "smooth_candidates")
    return B


def emin_pcg(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K):
    return emin_cg(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K, variant="pcg")


def emin_cgnr(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K):
    return emin_cg(Ap, Aj, Ax, Np, Nj, is_root, nc, Bc, nB, T, K, variant="cgnr")


def hierarchy(A, B, m=1, theta=0.0, degree=2, iters=4, method="cg", max_levels=10, min_coarse=64):
    """Alg. root_node_setup applied level by level, each coarse operator the
    Galerkin product of the level above (Sec. 3.8): strength, aggregation,
    pattern, tentative T, energy minimisation of P (CG; or GMRES for P and for
    R^T on A^T with T-hat = T, the left candidates equal to B), A_c = R A P,
    and the coarse candidates Bc as the next level's B.  Level 0 may be
    node-blocked (m = 2, A given as its scalar CSR); the coarse levels are
    scalar (their DOFs are m per aggregate).  Stops after max_levels levels,
    at a level of at most min_coarse rows, or where a level would not
    coarsen.  Returns the list of levels: dicts with A, B, m and, above the
    coarsest, the single-level set-up, P and RT (None for CG)."""
    levels = []
    Al, ml = A, m
    Bl = _f64(B).reshape(A.n_rows, -1)
    while True:
        lev = dict(A=Al, B=Bl, m=ml)
        levels.append(lev)
        if len(levels) >= max_levels or Al.n_rows <= min_coarse:
            break
        st = setup(Al, Bl, ml, theta, degree)
        nc, nB = st["nc"], Bl.shape[1]
        if nc == 0 or nc >= Al.n_rows:
            break
        args = (st["Np"], st["Nj"], st["is_root"], nc, st["Bc"], nB, st["T"], iters)
        RT = None
        if method == "cg":
            P, info = emin_cg(Al.rowptr, Al.colind, Al.vals, *args)
            if info["status"] != 0:
                raise OracleError(info["status"], "hierarchy: CG")
        else:
            P, _ = emin_gmres(Al.rowptr, Al.colind, Al.vals, *args)
            Tp, Tj, Tx = transpose(Al.rowptr, Al.colind, Al.vals)
            RT, _ = emin_gmres(Tp, Tj, Tx, *args)
        rt = () if RT is None else (st["Np"], st["Nj"], RT)
        Acp, Acj, Acx = galerkin(Al.rowptr, Al.colind, Al.vals, st["Np"], st["Nj"], P, nc, *rt)
        lev.update(setup=st, P=P, RT=RT)
        Al = type(Al)(nc, nc, Acp, Acj, Acx)
        Bl = _f64(st["Bc"]).reshape(nc, nB)
        ml = 1
    return levels


def operator_complexity(levels):
    """Sec. 2.4: the stored entries of every level's operator over those of
    the finest (scalar entries)."""
    return sum(lv["A"].nnz for lv in levels) / levels[0]["A"].nnz
