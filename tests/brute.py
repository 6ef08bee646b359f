"""Dense brute-force formulations used to pin the oracle on tiny problems.

These do not reuse the oracle's formulas: the energy is built as a dense
quadratic form on the vector of pattern entries, the constraint space as the
null space of an explicit constraint matrix (via SVD), and Krylov minimisers
and KKT solutions by dense linear algebra.
"""
from __future__ import annotations

import numpy as np


def entries(Np, Nj):
    """List of (row, col) of the pattern in CSR order."""
    rows = np.repeat(np.arange(Np.size - 1), np.diff(Np))
    return rows, np.asarray(Nj)


def energy_matrix(Ad, Np, Nj):
    """H with p^T H p = trace(P^T A P) for P supported on the pattern; also
    (H p)_e = (A P)_e for every pattern entry e."""
    r, c = entries(Np, Nj)
    same_col = c[:, None] == c[None, :]
    return np.where(same_col, Ad[np.ix_(r, r)], 0.0)


def constraint_matrix(Np, Nj, is_root, Bc):
    """Rows: one per root-row entry (value fixed) and one per (F row, candidate)."""
    r, c = entries(Np, Nj)
    E = r.size
    rows = []
    for e in range(E):
        if is_root[r[e]]:
            v = np.zeros(E)
            v[e] = 1.0
            rows.append(v)
    nB = 0 if Bc is None else Bc.shape[1]
    for i in range(Np.size - 1):
        if is_root[i]:
            continue
        for q in range(nB):
            v = np.zeros(E)
            s, t = Np[i], Np[i + 1]
            v[s:t] = Bc[Nj[s:t], q]
            rows.append(v)
    return np.array(rows).reshape(-1, E)


def null_basis(Cm, E):
    """Orthonormal basis (E x r) of the null space of Cm."""
    if Cm.shape[0] == 0:
        return np.eye(E)
    u, s, vt = np.linalg.svd(Cm)
    tol = max(Cm.shape) * np.finfo(float).eps * (s[0] if s.size else 0.0)
    rank = int((s > tol).sum())
    return vt[rank:].T


def krylov_basis(M, g, k):
    """Orthonormal basis of span{g, M g, ..., M^{k-1} g} with full
    re-orthogonalisation (two passes)."""
    Q = []
    v = g.copy()
    for _ in range(k):
        for _ in range(2):
            for q in Q:
                v = v - (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= 1e-14 * np.linalg.norm(g):
            break
        v = v / nv
        Q.append(v)
        v = M @ v
    return np.array(Q).T


def cg_krylov_argmin(Ad, Np, Nj, is_root, Bc, t, K):
    """argmin of trace(P^T A P) over t + span of the first K Krylov vectors of
    the projected operator started from the projected negative gradient."""
    H = energy_matrix(Ad, Np, Nj)
    Nb = null_basis(constraint_matrix(Np, Nj, is_root, Bc), t.size)
    Hr = Nb.T @ H @ Nb
    g = -Nb.T @ (H @ t)
    Q = krylov_basis(Hr, g, K)
    y = np.linalg.solve(Q.T @ Hr @ Q, Q.T @ g)
    return t + Nb @ (Q @ y)


def kkt_solution(Ad, Np, Nj, is_root, Bc, t):
    """Exact constrained minimiser of trace(P^T A P) over t + null(C)."""
    H = energy_matrix(Ad, Np, Nj)
    Nb = null_basis(constraint_matrix(Np, Nj, is_root, Bc), t.size)
    Hr = Nb.T @ H @ Nb
    g = -Nb.T @ (H @ t)
    return t + Nb @ np.linalg.solve(Hr, g)


def gmres_krylov_argmin(Ad, Np, Nj, is_root, Bc, t, K):
    """argmin ||Pi(A P)||_F over t + Krylov space (dense least squares)."""
    H = energy_matrix(Ad, Np, Nj)
    Nb = null_basis(constraint_matrix(Np, Nj, is_root, Bc), t.size)
    M = Nb.T @ H @ Nb
    g = -Nb.T @ (H @ t)
    Q = krylov_basis(M, g, K)
    y, *_ = np.linalg.lstsq(M @ Q, g, rcond=None)
    return t + Nb @ (Q @ y)


def projected_residual_norm(Ad, Np, Nj, is_root, Bc, p):
    H = energy_matrix(Ad, Np, Nj)
    Nb = null_basis(constraint_matrix(Np, Nj, is_root, Bc), p.size)
    return np.linalg.norm(Nb.T @ (H @ p))


def dense_projector(Np, Nj, is_root, Bc):
    Nb = null_basis(constraint_matrix(Np, Nj, is_root, Bc), int(Np[-1]))
    return Nb @ Nb.T


def to_dense(Np, Nj, vals, n_cols):
    r, c = entries(Np, Nj)
    D = np.zeros((Np.size - 1, n_cols))
    D[r, c] = vals
    return D
