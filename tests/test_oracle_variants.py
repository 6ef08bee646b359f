"""Pins of the oracle's variants (CPU only): candidate smoothing (the smooth
line of Alg. root_node_setup, Sec. 3.1), Jacobi-preconditioned CG and CGNR
(Sec. 4.2, energy minimisation in the A*A norm).

Smoothing: sweeps worked out by hand, an exact null vector left unchanged,
the A-norm decreasing.  PCG and CGNR: the K-step iterate equals the argmin
over the (preconditioned) Krylov space computed by dense linear algebra
(tests/brute.py), the converged iterate equals the dense KKT solution, and
the energy identity E_k - E_(k+1) = gamma_k^2 / delta_k holds.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests import brute as BF
from tests import cases as CS


def _dense(A):
    return sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n_rows, A.n_cols)).toarray()


def test_two_jacobi_sweeps_by_hand():
    A = W.laplace1d(4)  # [-1 2 -1], Dirichlet ends eliminated
    B = O.smooth_candidates(A.rowptr, A.colind, A.vals, np.ones(4), 1, 2.0 / 3.0)
    # rows 0 and 3: (A 1) = 1, so 1 - (2/3)(1/2) = 2/3; rows 1, 2: (A 1) = 0
    assert np.allclose(B[:, 0], [2 / 3, 1, 1, 2 / 3], rtol=0, atol=1e-15)
    B = O.smooth_candidates(A.rowptr, A.colind, A.vals, np.ones(4), 2, 2.0 / 3.0)
    # row 0: A B = 2(2/3) - 1 = 1/3 -> 2/3 - (2/3)(1/6) = 5/9; row 1: -2/3 + 2 - 1 = 1/3 -> 8/9
    assert np.allclose(B[:, 0], [5 / 9, 8 / 9, 8 / 9, 5 / 9], rtol=0, atol=1e-15)


def test_null_vector_is_left_alone_and_energy_decreases():
    # graph Laplacian with zero row sums: B = 1 is an exact null vector
    n = 50
    L = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    L[0, n - 1] = L[n - 1, 0] = -1.0
    L = L.tocsr()
    L.sort_indices()
    B = O.smooth_candidates(L.indptr, L.indices, L.data, np.ones((n, 2)), 4, 0.7)
    assert np.array_equal(B, np.ones((n, 2)))
    A = W.q1_aniso(20)
    Ad = _dense(A)
    B0 = np.random.default_rng(1).standard_normal((A.n_rows, 3))
    e_prev = np.trace(B0.T @ Ad @ B0)
    for s in range(1, 5):
        B = O.smooth_candidates(A.rowptr, A.colind, A.vals, B0, s, 2.0 / 3.0)
        e = np.trace(B.T @ Ad @ B)
        assert e < e_prev
        e_prev = e


def _reduced(Ad, c, H=None):
    Np, Nj, t = c["Np"], c["Nj"], c["T"]
    H = BF.energy_matrix(Ad, Np, Nj) if H is None else H
    Nb = BF.null_basis(BF.constraint_matrix(Np, Nj, c["is_root"], c["Bc"]), t.size)
    return H, Nb


def _varied_poisson(nx=10, seed=4):
    """5-point Poisson plus a positive diagonal shift that varies by row (so
    the Jacobi preconditioner is not a scalar), with the oracle's set-up."""
    A = W.poisson5(nx)
    rng = np.random.default_rng(seed)
    vals = A.vals.copy()
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.rowptr))
    diag = rows == A.colind
    vals[diag] += rng.uniform(0.0, 4.0, A.n_rows)
    A = type(A)(A.n_rows, A.n_cols, A.rowptr, A.colind, vals)
    st = O.setup(A, W.ones(A.n_rows), 1, 0.0, 2)  # every neighbour strong
    return dict(A=A, B=W.ones(A.n_rows), **st)


def _small_upwind(nx=12):
    A = W.upwind_cd(nx)
    st = O.setup(A, W.ones(A.n_rows), 1, 0.0, 2)
    return dict(A=A, B=W.ones(A.n_rows), **st)


def _case(name):
    if name == "varied_poisson10":
        return _varied_poisson()
    if name == "upwind12":
        return _small_upwind()
    return CS.case(name)


@pytest.mark.parametrize("name,K", [("laplace1d_8", 2), ("varied_poisson10", 3), ("elastic7", 3)])
def test_pcg_equals_preconditioned_krylov_argmin(name, K):
    c = _case(name)
    A = c["A"]
    Ad = _dense(A)
    H, Nb = _reduced(Ad, c)
    r, _ = BF.entries(c["Np"], c["Nj"])
    dinv = 1.0 / np.diag(Ad)[r]          # Jacobi: each entry scaled by its row's 1/a_ii
    Hr = Nb.T @ H @ Nb
    Mr = Nb.T @ (dinv[:, None] * Nb)     # the preconditioner on the constraint space
    g = -Nb.T @ (H @ c["T"])
    Q = BF.krylov_basis(Mr @ Hr, Mr @ g, K)
    y = np.linalg.solve(Q.T @ Hr @ Q, Q.T @ g)
    ref = c["T"] + Nb @ (Q @ y)
    P, info = O.emin_pcg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                         c["B"].shape[1], c["T"], K)
    # (a tiny problem may converge before K steps: the argmin is then the solution)
    assert info["status"] == 0 and 1 <= info["iters"] <= K
    assert np.max(np.abs(P - ref)) <= 1e-10


def test_pcg_with_constant_diagonal_is_cg():
    c = CS.case("poisson32")  # every diagonal entry 4: the preconditioner is a scalar
    A = c["A"]
    args = (A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"], 1, c["T"], 4)
    Pc, _ = O.emin_cg(*args)
    Pp, ip = O.emin_pcg(*args)
    assert np.max(np.abs(Pc - Pp)) <= 1e-14
    assert np.allclose(ip["gamma"] * 4.0, O.emin_cg(*args)[1]["gamma"], rtol=1e-13, atol=0)


@pytest.mark.parametrize("variant", ["pcg", "cgnr"])
def test_energy_identity(variant):
    c = CS.case("aniso40")
    A = c["A"]
    K = 5
    Ps = []
    for k in range(K + 1):
        P, info = O.emin_cg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"], 1, c["T"],
                            k, variant=variant)
        Ps.append(P)
    As = sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n_rows, A.n_rows))
    if variant == "pcg":
        E = [O.energy(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["nc"], P) for P in Ps]
    else:  # ||A P||_F^2 with A P taken whole
        E = [float(sp.linalg.norm(As @ sp.csr_matrix((P, c["Nj"], c["Np"]), shape=(A.n_rows, c["nc"]))) ** 2)
             for P in Ps]
    g, d = info["gamma"], info["delta"]
    for k in range(K):
        assert E[k + 1] < E[k]
        assert abs((E[k] - E[k + 1]) - g[k] ** 2 / d[k]) <= 1e-9 * abs(E[k] - E[k + 1])


@pytest.mark.parametrize("name,K", [("upwind12", 3), ("laplace1d_8", 3), ("asym20", 4)])
def test_cgnr_equals_normal_krylov_argmin(name, K):
    c = _case(name)
    A = c["A"]
    Ad = _dense(A)
    AtA = Ad.T @ Ad
    P = BF.cg_krylov_argmin(AtA, c["Np"], c["Nj"], c["is_root"], c["Bc"], c["T"], K)
    got, info = O.emin_cgnr(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                            c["B"].shape[1], c["T"], K)
    assert info["status"] == 0
    assert np.max(np.abs(got - P)) <= 1e-9 * max(1.0, np.max(np.abs(P)))


@pytest.mark.parametrize("variant,name", [("pcg", "laplace1d_8"), ("pcg", "varied_poisson10"),
                                          ("cgnr", "upwind12"), ("cgnr", "asym20")])
def test_converged_variants_reach_the_kkt_solution(variant, name):
    c = _case(name)
    A = c["A"]
    Ad = _dense(A)
    M = Ad if variant == "pcg" else Ad.T @ Ad
    ref = BF.kkt_solution(M, c["Np"], c["Nj"], c["is_root"], c["Bc"], c["T"])
    P, info = O.emin_cg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                        c["B"].shape[1], c["T"], 400, variant=variant)
    assert info["status"] == 0
    assert np.max(np.abs(P - ref)) <= 1e-8
