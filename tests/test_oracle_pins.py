"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: values the
paper prints for its worked examples (tests/golden), closed forms, invariants,
special cases that reduce to a textbook result, library routines, and dense
brute force on tiny inputs (tests/brute.py).
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import oracle as O
import workloads as W
from tests import brute

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _sp(A):
    return sp.csr_matrix((A.vals, A.colind, A.rowptr), shape=(A.n_rows, A.n_cols))


def _setup(A, B, m=1, theta=0.0, d=2):
    return O.setup(A, B, m, theta, d)


# ----------------------------------------------------------------------------
# generators (input shapes the configurations name)
# ----------------------------------------------------------------------------
def test_generator_sizes():
    assert W.poisson5(32).nnz == 4992
    assert W.q1_aniso(50, 1.0, 0.0).nnz == 21904          # Sec. 2.3 example
    assert W.q1_aniso(256).nnz == 586756 == (3 * 256 - 2) ** 2
    assert W.upwind_cd(64).nnz == 5 * 64 * 64 - 4 * 64


def test_q1_stencil_properties():
    st = W.q1_stencil(1.0, 0.0)
    assert math.isclose(st[(0, 0)], 8.0 / 3.0, rel_tol=1e-14)
    for off, v in st.items():
        if off != (0, 0):
            assert math.isclose(v, -1.0 / 3.0, rel_tol=1e-14)
    for eps, psi in [(1e-3, math.pi / 8), (0.3, 2.0)]:
        assert abs(sum(W.q1_stencil(eps, psi).values())) < 1e-14


# ----------------------------------------------------------------------------
# strength (Sec. 3.2)
# ----------------------------------------------------------------------------
def test_strength_tie_kept_poisson():
    A = W.poisson5(8)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, 0.25)
    # |a_ij| = 0.25 sqrt(a_ii a_jj) exactly: every neighbour is kept
    assert np.array_equal(Sp, A.rowptr) and np.array_equal(Sj, A.colind)


def test_strength_aniso_keeps_six_of_eight():
    A = W.q1_aniso(9)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, 0.1)
    i = 4 * 9 + 4
    offs = {(int(j % 9) - 4, int(j // 9) - 4) for j in Sj[Sp[i]:Sp[i + 1]]}
    assert offs == {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (-1, 1), (1, -1)}


def test_strength_theta_zero_is_structure_and_symmetric():
    A = W.upwind_cd(7)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, 0.0)
    assert np.array_equal(Sp, A.rowptr) and np.array_equal(Sj, A.colind)
    # a non-symmetric strong set is symmetrised: drop one direction by hand
    M = _sp(A).tolil()
    M[3, 4] = 1e-9
    M = M.tocsr()
    M.sort_indices()
    Sp, Sj = O.strength(M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data, 1, 0.5)
    S = sp.csr_matrix((np.ones(Sj.size), Sj, Sp), shape=M.shape)
    assert (S != S.T).nnz == 0


def test_strength_amalgamates_blocks():
    Ab, _ = W.q1_elasticity(5)
    A = Ab.to_csr()
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 2, 0.0)
    assert np.array_equal(Sp, Ab.rowptr) and np.array_equal(Sj, Ab.colind)


def _csr_from_dense(M):
    r, c = np.nonzero(M)
    rowptr = np.concatenate([[0], np.cumsum(np.bincount(r, minlength=M.shape[0]))]).astype(np.int32)
    return rowptr, c.astype(np.int32), M[r, c].astype(np.float64)


def test_strength_amalgamation_hand_example():
    # Sec. 3.2, amalgamate step (reading R4: a node pair is strong when any DOF
    # entry of its 2x2 block is), with theta = 1/2 so every test is exact:
    # keep |a_ij| >= theta sqrt|a_ii a_jj|.  Nodes 0, 1, 2 hold DOFs (0,1),
    # (2,3), (4,5); DOF diagonals 4, 1, 4, 1, 4, 1.
    #   block (0,1): a_02 = -1.5 (2.25 < 4: weak), a_03 = -1 (1 >= 1: strong,
    #                a tie), a_12 = -0.5 (0.25 < 1: weak)       -> strong
    #   block (0,2): a_04 = -1.9 (3.61 < 4), a_05 = -0.9 (0.81 < 1),
    #                a_15 = -0.4 (0.16 < 0.25)                   -> weak
    #   block (1,2): a_24 = -0.5 (0.25 < 4: weak); a_35 = -0.5 (0.25 >= 0.25:
    #                strong) but a_53 = -0.4 (0.16 < 0.25: weak), so only the
    #                symmetrisation S u S^T puts (2,1) in S        -> strong
    # AND over the block, the (0,0) component alone, or no symmetrisation each
    # give a different graph.
    M = np.zeros((6, 6))
    np.fill_diagonal(M, [4, 1, 4, 1, 4, 1])
    M[0, 1] = M[1, 0] = -0.1
    for (i, j, v) in [(0, 2, -1.5), (0, 3, -1.0), (1, 2, -0.5), (0, 4, -1.9), (0, 5, -0.9), (1, 5, -0.4),
                      (2, 4, -0.5)]:
        M[i, j] = M[j, i] = v
    M[3, 5], M[5, 3] = -0.5, -0.4
    Ap, Aj, Ax = _csr_from_dense(M)
    Sp, Sj = O.strength(Ap, Aj, Ax, 2, 0.5)
    got = {(I, int(J)) for I in range(3) for J in Sj[Sp[I]:Sp[I + 1]]}
    assert got == {(0, 0), (0, 1), (1, 0), (1, 1), (1, 2), (2, 1), (2, 2)}


@pytest.mark.parametrize("theta", [0.1, 0.3])
def test_strength_amalgamation_brute_force(theta):
    # node-blocked elasticity at theta > 0, where the blocks mix strong and weak
    # DOF entries: the node graph is "any entry of the block strong", then
    # symmetrised, then the diagonal; written out here with dense boolean arrays
    Ab, _ = W.q1_elasticity(7)
    A = Ab.to_csr()
    Ad = A.to_dense()
    d = np.diag(Ad)
    strong = (Ad != 0) & (Ad * Ad >= theta * theta * np.abs(np.outer(d, d)))
    nn = A.n_rows // 2
    node = strong.reshape(nn, 2, nn, 2).any(axis=(1, 3))
    node = node | node.T | np.eye(nn, dtype=bool)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 2, theta)
    want_p = np.concatenate([[0], np.cumsum(node.sum(1))])
    assert np.array_equal(Sp, want_p)
    assert np.array_equal(Sj, np.nonzero(node)[1])
    # the case discriminates: requiring every stored entry of a block to be
    # strong drops blocks that the rule keeps
    stored = (Ad != 0).reshape(nn, 2, nn, 2).any(axis=(1, 3))
    every = ((strong | (Ad == 0)).reshape(nn, 2, nn, 2).all(axis=(1, 3))) & stored
    assert (node & ~(every | every.T | np.eye(nn, dtype=bool))).any()


# ----------------------------------------------------------------------------
# aggregation (Sec. 3.3) against the worked examples
# ----------------------------------------------------------------------------
def test_aggregation_worked_example_1d():
    g = json.load(open(os.path.join(GOLD, "e1_laplace1d.json")))
    A = W.laplace1d(g["n"])
    agg, roots = O.aggregate(*O.strength(A.rowptr, A.colind, A.vals, 1, 0.0))
    got = [sorted(np.flatnonzero(agg == a).tolist()) for a in range(roots.size)]
    assert got == g["aggregates"]
    assert roots.tolist() == g["roots"]


def test_aggregation_q1_50_example():
    g = json.load(open(os.path.join(GOLD, "e2_q1_laplace50.json")))
    A = W.q1_aniso(g["nx"], 1.0, 0.0)
    assert A.nnz == g["nnz_A"]
    agg, roots = O.aggregate(*O.strength(A.rowptr, A.colind, A.vals, 1, 0.0))
    assert roots.size == g["n_agg"]
    Cm = sp.csr_matrix((np.ones(A.n_rows), agg, np.arange(A.n_rows + 1)), shape=(A.n_rows, roots.size))
    As = _sp(A).copy()
    As.data[:] = 1.0
    Ac = (Cm.T @ As @ Cm)
    assert Ac.nnz == g["nnz_coarse_one_candidate"]
    assert 4 * Ac.nnz == g["nnz_coarse_two_candidates"]


@pytest.mark.parametrize("nx,expect", [(512, 171 ** 2), (256, 86 ** 2)])
def test_aggregation_nine_point_closed_form(nx, expect):
    # every neighbour strong on a 9-point grid: sweep 1 tiles it by 3x3 boxes
    A = W.stencil_grid(nx, nx, {(dx, dy): 1.0 for dx in (-1, 0, 1) for dy in (-1, 0, 1)})
    agg, roots = O.aggregate(*O.strength(A.rowptr, A.colind, A.vals, 1, 0.0))
    assert roots.size == expect
    assert np.array_equal(agg[roots], np.arange(roots.size))


def test_aggregation_partition_properties():
    A = W.q1_aniso(40)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, 0.1)
    agg, roots = O.aggregate(Sp, Sj)
    assert agg.min() == 0 and agg.max() == roots.size - 1
    assert np.array_equal(agg[roots], np.arange(roots.size))
    # each node is the root or strongly adjacent to a member of its aggregate
    for i in range(agg.size):
        nb = Sj[Sp[i]:Sp[i + 1]]
        assert i in roots or np.any((agg[nb] == agg[i]) & (nb != i))


# ----------------------------------------------------------------------------
# pattern S^d C (Sec. 3.4)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("d", [0, 1, 2, 3])
def test_pattern_is_distance_d_closure(d):
    A = W.q1_aniso(14)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, 0.1)
    agg, roots = O.aggregate(Sp, Sj)
    Np, Nj = O.pattern_nodes(Sp, Sj, agg, roots.size, d)
    S = sp.csr_matrix((np.ones(Sj.size), Sj, Sp), shape=(A.n_rows,) * 2)
    dist = shortest_path(S, unweighted=True)
    Sd = S.toarray()
    Cm = np.zeros((A.n_rows, roots.size))
    Cm[np.arange(A.n_rows), agg] = 1
    dense = np.linalg.matrix_power(Sd, d) @ Cm > 0
    for i in range(A.n_rows):
        bfs = sorted(set(agg[dist[i] <= d].tolist()))
        assert Nj[Np[i]:Np[i + 1]].tolist() == bfs
        assert np.flatnonzero(dense[i]).tolist() == bfs


def test_pattern_nine_point_average_41_over_9():
    nx = 33
    A = W.stencil_grid(nx, nx, {(dx, dy): 1.0 for dx in (-1, 0, 1) for dy in (-1, 0, 1)})
    st = _setup(A, W.ones(A.n_rows), 1, 0.0, 2)
    lens = np.diff(st["Np"]).reshape(nx, nx)
    tile = lens[9:18, 9:18]          # three whole interior 3x3 aggregate tiles
    assert tile.sum() * 9 == 41 * tile.size
    assert set(np.unique(tile).tolist()) == {1, 4, 6, 9} - {9}


def test_pattern_dofs_unamalgamate_and_roots():
    Ab, xy = W.q1_elasticity(5)
    A = Ab.to_csr()
    st = _setup(A, W.rbm(xy), 2, 0.0, 2)
    Np, Nj, Npn, Njn, agg, roots = st["Np"], st["Nj"], st["Npn"], st["Njn"], st["agg"], st["roots"]
    for i in range(A.n_rows):
        I = i // 2
        row = Nj[Np[i]:Np[i + 1]].tolist()
        if roots[agg[I]] == I:
            assert st["is_root"][i] == 1 and row == [2 * agg[I] + i % 2]
        else:
            assert row == sorted(2 * a + c for a in Njn[Npn[I]:Npn[I + 1]] for c in (0, 1))


# ----------------------------------------------------------------------------
# tentative T and Eq. (Tproj)
# ----------------------------------------------------------------------------
def test_tproj_worked_example_row():
    g = json.load(open(os.path.join(GOLD, "e1_laplace1d.json")))
    A = W.laplace1d(g["n"])
    B = np.stack([np.ones(g["n"]), np.array(g["x"])], axis=1)
    st = _setup(A, B, 1, 0.0, 1)
    r = g["tproj_row1_d1"]
    s, e = st["Np"][1], st["Np"][2]
    assert st["Nj"][s:e].tolist() == r["J"]
    assert np.allclose(st["T"][s:e], r["values"], rtol=0, atol=1e-15)


def test_tentative_constant_is_aggregation_matrix():
    A = W.poisson5(12)
    st = _setup(A, W.ones(A.n_rows), 1, 0.25, 2)
    r, c = brute.entries(st["Np"], st["Nj"])
    assert np.array_equal(st["T"], (c == st["agg"][r]).astype(float))


@pytest.mark.parametrize("case", ["poisson", "elastic", "twocand"])
def test_tentative_interpolates_candidates(case):
    if case == "poisson":
        A, B, m = W.poisson5(10), W.ones(100), 1
    elif case == "elastic":
        Ab, xy = W.q1_elasticity(7)
        A, B, m = Ab.to_csr(), W.rbm(xy), 2
    else:
        A = W.poisson5(10)
        x = np.arange(100) % 10 / 10.0
        B, m = np.stack([np.ones(100), x, (np.arange(100) // 10) / 10.0], 1), 1
    st = _setup(A, B, m, 0.0, 3 if case == "twocand" else 2)
    assert st["rank_def"] == 0
    assert O.constraint_residual(st["Np"], st["Nj"], st["T"], st["Bc"], B) < 1e-14
    roots_rows = np.flatnonzero(st["is_root"])
    assert np.all(st["T"][st["Np"][roots_rows]] == 1.0)
    assert np.all(np.diff(st["Np"])[roots_rows] == 1)


def test_tproj_rank_deficient_row_is_min_norm_least_squares():
    # a corner DOF row whose pattern reaches a single aggregate cannot carry
    # the rotation: Eq. (Tproj) then takes the minimum-norm least-squares update
    Ab, xy = W.q1_elasticity(6)
    A, B = Ab.to_csr(), W.rbm(xy)
    st = _setup(A, B, 2, 0.0, 2)
    assert st["rank_def"] == 2
    Np, Nj, Bc = st["Np"], st["Nj"], st["Bc"]
    for i in np.flatnonzero(st["is_root"] == 0):
        s, e = Np[i], Np[i + 1]
        BJ = Bc[Nj[s:e]]
        t0 = (Nj[s:e] // 2 == st["agg"][i // 2]) * (Nj[s:e] % 2 == i % 2)
        u, *_ = np.linalg.lstsq(BJ.T, B[i] - t0 @ BJ, rcond=None)
        assert np.allclose(st["T"][s:e], t0 + u, atol=1e-13)


# ----------------------------------------------------------------------------
# small kernels against library routines / dense projectors
# ----------------------------------------------------------------------------
def test_masked_product_matches_library_product():
    A = W.q1_aniso(12)
    st = _setup(A, W.ones(A.n_rows), 1, 0.1, 2)
    rng = np.random.default_rng(3)
    X = rng.standard_normal(st["Nj"].size)
    Z = O.masked_product(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["nc"], X)
    Xd = brute.to_dense(st["Np"], st["Nj"], X, st["nc"])
    Y = _sp(A) @ Xd
    r, c = brute.entries(st["Np"], st["Nj"])
    assert np.allclose(Z, Y[r, c], rtol=0, atol=1e-13)


def test_gram_pinv_matches_library():
    rng = np.random.default_rng(1)
    M = rng.standard_normal((3, 3))
    G = M @ M.T + 0.1 * np.eye(3)
    Gp, fb = O.gram_pinv(G)
    assert not fb and np.allclose(Gp, np.linalg.inv(G), rtol=1e-12, atol=0)
    v = rng.standard_normal((3, 2))
    G = v @ v.T                       # rank 2
    Gp, fb = O.gram_pinv(G)
    assert fb and np.allclose(Gp, np.linalg.pinv(G), atol=1e-10)


@pytest.mark.parametrize("case", ["ones", "rbm"])
def test_projection_is_orthogonal_projector(case):
    if case == "ones":
        A, B, m = W.poisson5(5), W.ones(25), 1
    else:
        Ab, xy = W.q1_elasticity(3)
        A, B, m = Ab.to_csr(), W.rbm(xy), 2
    st = _setup(A, B, m, 0.0, 1)
    rng = np.random.default_rng(0)
    X = rng.standard_normal(st["Nj"].size)
    Pd = brute.dense_projector(st["Np"], st["Nj"], st["is_root"], st["Bc"])
    got = O.project(st["Np"], st["Nj"], st["is_root"], st["Bc"], B.shape[1], X)
    assert np.allclose(got, Pd @ X, atol=1e-12)


def test_transpose_matches_library():
    A = W.upwind_cd(9)
    Tp, Tj, Tx = O.transpose(A.rowptr, A.colind, A.vals)
    At = _sp(A).T.tocsr()
    At.sort_indices()
    assert np.array_equal(Tp, At.indptr) and np.array_equal(Tj, At.indices)
    assert np.array_equal(Tx, At.data)


# ----------------------------------------------------------------------------
# CG energy minimisation (Sec. 3.6, Sec. 4.1)
# ----------------------------------------------------------------------------
def _cg(A, st, K, nB=None):
    nB = st["Bc"].shape[1] if nB is None else nB
    return O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"],
                     st["Bc"], nB, st["T"], K)


@pytest.mark.parametrize("case", ["poisson32", "aniso", "elastic"])
def test_cg_invariants(case):
    if case == "poisson32":
        c = W.config("poisson32")
        A, B, m, th = c["A"], c["B"], 1, c["theta"]
    elif case == "aniso":
        A, B, m, th = W.q1_aniso(40), W.ones(1600), 1, 0.1
    else:
        Ab, xy = W.q1_elasticity(10)
        A, B, m, th = Ab.to_csr(), W.rbm(xy), 2, 0.0
    st = _setup(A, B, m, th, 2)
    K = 6
    energies = []
    for k in range(K + 1):
        P, info = _cg(A, st, k)
        assert info["status"] == 0
        energies.append(O.energy(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["nc"], P))
        assert O.constraint_residual(st["Np"], st["Nj"], P, st["Bc"], B) < 1e-12
        roots_rows = np.flatnonzero(st["is_root"])
        assert np.all(P[st["Np"][roots_rows]] == 1.0)
    g, dl = info["gamma"], info["delta"]
    for k in range(K):
        drop = energies[k] - energies[k + 1]
        assert drop > 0
        assert math.isclose(drop, g[k] ** 2 / dl[k], rel_tol=1e-9, abs_tol=1e-12 * energies[0])


@pytest.mark.parametrize("case,K", [("1d", 3), ("2d", 4), ("elastic", 3)])
def test_cg_is_krylov_argmin(case, K):
    if case == "1d":
        A, B, m, th = W.laplace1d(16), W.ones(16), 1, 0.25
    elif case == "2d":
        A, B, m, th = W.poisson5(6), W.ones(36), 1, 0.25
    else:
        Ab, xy = W.q1_elasticity(4)
        A, B, m, th = Ab.to_csr(), W.rbm(xy), 2, 0.0
    st = _setup(A, B, m, th, 2)
    P, info = _cg(A, st, K)
    ref = brute.cg_krylov_argmin(A.to_dense(), st["Np"], st["Nj"], st["is_root"], st["Bc"], st["T"], K)
    assert np.max(np.abs(P - ref)) < 1e-10


@pytest.mark.parametrize("case", ["2d", "elastic"])
def test_cg_converges_to_kkt(case):
    if case == "2d":
        A, B, m = W.poisson5(5), W.ones(25), 1
    else:
        Ab, xy = W.q1_elasticity(4)
        A, B, m = Ab.to_csr(), W.rbm(xy), 2
    st = _setup(A, B, m, 0.25 if m == 1 else 0.0, 1 if m == 1 else 2)
    assert st["rank_def"] == 0
    ref = brute.kkt_solution(A.to_dense(), st["Np"], st["Nj"], st["is_root"], st["Bc"], st["T"])
    # the oracle stops by itself once <R,R> has dropped by 1e24 (past that
    # point CG would iterate on round-off)
    P, info = _cg(A, st, 400)
    assert 0 < info["iters"] < 400
    assert info["gamma"][info["iters"]] <= 1e-24 * info["gamma"][0]
    assert np.max(np.abs(P - ref)) < 1e-9


def test_cg_reaches_ideal_interpolation():
    # Lemma th:cg: with no candidate constraint and a full F pattern, energy
    # minimisation converges to P_ideal = [-A_ff^{-1} A_fc; I] (Eq. ideal).
    A = W.poisson5(5)
    n = A.n_rows
    st = _setup(A, W.ones(n), 1, 0.25, 1)
    roots, agg, nc = st["roots"], st["agg"], st["nc"]
    is_root = np.zeros(n, np.uint8)
    is_root[roots] = 1
    Np = [0]
    Nj = []
    for i in range(n):
        cols = [int(agg[i])] if is_root[i] else list(range(nc))
        Nj += cols
        Np.append(len(Nj))
    Np, Nj = np.array(Np, np.int32), np.array(Nj, np.int32)
    r, c = brute.entries(Np, Nj)
    T = (c == agg[r]).astype(float)
    st2 = dict(Np=Np, Nj=Nj, is_root=is_root, nc=nc, Bc=np.zeros((nc, 1)), T=T)
    P, info = _cg(A, st2, 500, nB=0)
    assert 0 < info["iters"] < 500
    Ad = A.to_dense()
    F = np.flatnonzero(is_root == 0)
    Cpts = roots                      # coarse column a injects at node roots[a]
    ideal = -np.linalg.solve(Ad[np.ix_(F, F)], Ad[np.ix_(F, Cpts)])
    Pd = brute.to_dense(Np, Nj, P, nc)
    assert np.max(np.abs(Pd[F] - ideal)) < 1e-10
    assert np.array_equal(Pd[Cpts], np.eye(nc))


def test_cg_candidates_in_range_of_P():
    # e_B = (I - P P^+) B vanishes when P Bc = B (Sec. 3.9)
    Ab, xy = W.q1_elasticity(7)
    A, B = Ab.to_csr(), W.rbm(xy)
    st = _setup(A, B, 2, 0.0, 2)
    assert st["rank_def"] == 0
    P, _ = _cg(A, st, 4)
    Pd = brute.to_dense(st["Np"], st["Nj"], P, st["nc"])
    eB = B - Pd @ (np.linalg.pinv(Pd) @ B)
    assert np.max(np.abs(eB)) < 1e-12


def test_cg_breakdown_on_indefinite_operator():
    A = W.poisson5(6)
    neg = W.CSR(A.n_rows, A.n_cols, A.rowptr, A.colind, -A.vals)
    st = _setup(A, W.ones(36), 1, 0.25, 2)
    _, info = O.emin_cg(neg.rowptr, neg.colind, neg.vals, st["Np"], st["Nj"], st["is_root"], st["nc"],
                        st["Bc"], 1, st["T"], 3)
    assert info["status"] == O.ORC_EBREAKDOWN


# ----------------------------------------------------------------------------
# GMRES energy minimisation (Sec. 3.6, Sec. 4.2)
# ----------------------------------------------------------------------------
def _gmres(A, st, K):
    return O.emin_gmres(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"],
                        st["Bc"], st["Bc"].shape[1], st["T"], K)


@pytest.mark.parametrize("K", [1, 3, 5])
def test_gmres_is_residual_argmin(K):
    A = W.upwind_cd(6, eps=1e-2)
    st = _setup(A, W.ones(36), 1, 0.0, 2)
    P, info = _gmres(A, st, K)
    Ad = A.to_dense()
    ref = brute.gmres_krylov_argmin(Ad, st["Np"], st["Nj"], st["is_root"], st["Bc"], st["T"], K)
    assert np.max(np.abs(P - ref)) < 1e-10
    res = [brute.projected_residual_norm(Ad, st["Np"], st["Nj"], st["is_root"], st["Bc"],
                                         _gmres(A, st, k)[0]) for k in range(K + 1)]
    assert all(res[k + 1] <= res[k] * (1 + 1e-12) for k in range(K))
    assert np.allclose(info["resid"][:K + 1], res, rtol=1e-9)


def test_gmres_on_spd_reaches_cg_limit():
    A = W.poisson5(5)
    st = _setup(A, W.ones(25), 1, 0.25, 1)
    ref = brute.kkt_solution(A.to_dense(), st["Np"], st["Nj"], st["is_root"], st["Bc"], st["T"])
    dim = brute.null_basis(brute.constraint_matrix(st["Np"], st["Nj"], st["is_root"], st["Bc"]),
                           st["T"].size).shape[1]
    # the oracle stops once its residual estimate has dropped by 1e12: later
    # basis vectors would be normalised round-off
    P, info = _gmres(A, st, dim)
    assert 0 < info["iters"] <= dim
    assert info["resid"][info["iters"]] <= 1e-12 * info["resid"][0]
    assert np.max(np.abs(P - ref)) < 1e-9


def test_restriction_on_transpose_keeps_left_candidates():
    A = W.upwind_cd(16)
    Bh = W.ones(A.n_rows) * 1.0
    st = _setup(A, W.ones(A.n_rows), 1, 0.0, 2)
    Tp, Tj, Tx = O.transpose(A.rowptr, A.colind, A.vals)
    That, Bch, _ = O.tentative(st["Np"], st["Nj"], st["is_root"], st["agg"], st["roots"], 1, Bh)
    RT, info = O.emin_gmres(Tp, Tj, Tx, st["Np"], st["Nj"], st["is_root"], st["nc"], Bch, 1, That, 8)
    assert info["status"] == 0
    assert O.constraint_residual(st["Np"], st["Nj"], RT, Bch, Bh) < 1e-12
    assert info["resid"][-1] < info["resid"][0]


# ----------------------------------------------------------------------------
# tangent-linear model against finite differences
# ----------------------------------------------------------------------------
def test_cg_jvp_matches_central_differences():
    A = W.q1_aniso(8, 0.05, 1.0)
    st = _setup(A, W.ones(64), 1, 0.0, 2)
    rng = np.random.default_rng(7)
    v = rng.standard_normal(A.nnz)
    K = 4
    P, dP = O.emin_cg_jvp(A.rowptr, A.colind, A.vals, v, st["Np"], st["Nj"], st["is_root"], st["nc"],
                          st["Bc"], 1, st["T"], K)
    h = 1e-6 * np.max(np.abs(A.vals))
    def run(x):
        return O.emin_cg(A.rowptr, A.colind, x, st["Np"], st["Nj"], st["is_root"], st["nc"],
                         st["Bc"], 1, st["T"], K)[0]
    fd = (run(A.vals + h * v) - run(A.vals - h * v)) / (2 * h)
    assert np.linalg.norm(fd - dP) <= 1e-6 * np.linalg.norm(dP)
    assert np.array_equal(P, run(A.vals))


# ----------------------------------------------------------------------------
# metrics: constraint residual (Eq. mode_constraint) and energy
# ----------------------------------------------------------------------------
def test_constraint_residual_hand_example():
    # three rows over two coarse columns, two candidates, Bc = [[1, 2], [1, 1]];
    # row 1 is a root row (the identity row of column 1).  The exact P below
    # satisfies P Bc = B; each perturbation's residual is worked out by hand.
    Np = np.array([0, 2, 3, 5], np.int32)
    Nj = np.array([0, 1, 1, 0, 1], np.int32)
    Bc = np.array([[1.0, 2.0], [1.0, 1.0]])
    P = np.array([0.5, 0.25, 1.0, 0.25, 0.5])
    B = np.array([[0.75, 1.25], [1.0, 1.0], [0.75, 1.0]])
    assert O.constraint_residual(Np, Nj, P, Bc, B) == 0.0
    # F row 0 loses 0.3 at column 1 -> deviations (-0.3, -0.3); the root row
    # drops from 1 to 0.3 -> deviations (-0.7, -0.7): only negative
    # deviations, the largest on a root row
    Q = P.copy()
    Q[1] -= 0.3
    Q[2] = 0.3
    assert math.isclose(O.constraint_residual(Np, Nj, Q, Bc, B), 0.7, rel_tol=0, abs_tol=1e-15)
    # row 2 gains 0.1 at column 0 -> deviations (0.1 * 1, 0.1 * 2): the second
    # candidate decides
    Q = P.copy()
    Q[3] += 0.1
    assert math.isclose(O.constraint_residual(Np, Nj, Q, Bc, B), 0.2, rel_tol=0, abs_tol=1e-15)


def test_energy_is_trace_of_galerkin_product():
    # E(P) = trace(P^T A P) over the pattern, against a dense evaluation
    A = W.q1_aniso(9, 0.1, 0.7)
    st = _setup(A, W.ones(A.n_rows), 1, 0.1, 2)
    rng = np.random.default_rng(3)
    P = rng.standard_normal(st["Nj"].size)
    Pd = brute.to_dense(st["Np"], st["Nj"], P, st["nc"])
    e = O.energy(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["nc"], P)
    assert math.isclose(e, float(np.trace(Pd.T @ A.to_dense() @ Pd)), rel_tol=1e-12)


# ----------------------------------------------------------------------------
# threads: the oracle's results do not depend on the number of threads
# ----------------------------------------------------------------------------
def test_results_identical_across_thread_counts():
    A = W.q1_aniso(96)
    st = _setup(A, W.ones(A.n_rows), 1, 0.1, 2)
    Au = W.upwind_cd(64)
    su = _setup(Au, W.ones(Au.n_rows), 1, 0.0, 2)
    n0 = O.threads()
    out = []
    try:
        for t in (1, 3, 8):
            O.set_threads(t)
            P, info = _cg(A, st, 6)
            Q, qinfo = _gmres(Au, su, 8)
            out.append((P, info["gamma"], Q, qinfo["resid"]))
    finally:
        O.set_threads(n0)
    for r in out[1:]:
        for a, b in zip(out[0], r):
            assert np.array_equal(a, b)
