"""Pins of the oracle's pre-filter path (Sec. 3.5, Eq. soc, Sec. 3.4 with
values), CPU only: strength values worked out by hand, the valued pattern
against numpy's dense product of the same matrices, its structure against the
boolean pattern (pinned by brute-force BFS elsewhere), and invariants of the
filtered set-up."""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests import cases as CS

# 3 x 3 non-symmetric operator: |a_01| = 2, |a_10| = 1, |a_12| = 0.5, |a_21| = 0.25
AP = np.array([0, 2, 5, 7])
AJ = np.array([0, 1, 0, 1, 2, 1, 2])
AX = np.array([4.0, -2.0, -1.0, 4.0, -0.5, -0.25, 4.0])


def test_strength_values_by_hand_theta0():
    Sp, Sj = O.strength(AP, AJ, AX, 1, 0.0)
    Sx = O.strength_values(AP, AJ, AX, 1, 0.0, Sp, Sj)
    # (0,1) = (1,0) = max(2, 1) = 2; (1,2) = (2,1) = max(0.5, 0.25) = 0.5;
    # rows divided by their largest off value: row 1 -> [1, 1, 0.25]
    assert Sj.tolist() == [0, 1, 0, 1, 2, 1, 2]
    assert Sx.tolist() == [1.0, 1.0, 1.0, 1.0, 0.25, 1.0, 1.0]


def test_strength_values_by_hand_theta03():
    # theta^2 |a_ii a_jj| = 1.44: only a_01 (4 >= 1.44) is strong; S u S^T
    # adds (1,0) with the value of the strong entry it mirrors
    Sp, Sj = O.strength(AP, AJ, AX, 1, 0.3)
    Sx = O.strength_values(AP, AJ, AX, 1, 0.3, Sp, Sj)
    assert Sp.tolist() == [0, 2, 4, 5] and Sj.tolist() == [0, 1, 0, 1, 2]
    assert Sx.tolist() == [1.0, 1.0, 1.0, 1.0, 1.0]


def _bsr_to_csr(blocks, nn):
    """Scalar CSR of a node-blocked operator given as {(I, J): 2x2 block}."""
    A = sp.lil_matrix((2 * nn, 2 * nn))
    for (I, J), b in blocks.items():
        A[2 * I:2 * I + 2, 2 * J:2 * J + 2] = np.asarray(b) + 1e-300  # keep explicit zeros stored
    A = A.tocsr()
    A.data[np.abs(A.data) < 1e-200] = 0.0
    A.sort_indices()
    return A


def test_amalgamated_value_is_the_largest_strong_entry_of_the_block():
    d = [[4.0, 0.0], [0.0, 4.0]]
    blocks = {(0, 0): d, (1, 1): d, (2, 2): d,
              (0, 1): [[-0.1, 0.0], [0.0, -1.0]], (1, 0): [[-0.1, 0.0], [0.0, -1.0]],
              (0, 2): [[-0.5, -0.5], [-0.5, -0.5]], (2, 0): [[-0.5, -0.5], [-0.5, -0.5]]}
    A = _bsr_to_csr(blocks, 3)
    Sp, Sj = O.strength(A.indptr, A.indices, A.data, 2, 0.0)
    Sx = O.strength_values(A.indptr, A.indices, A.data, 2, 0.0, Sp, Sj)
    # node row 0: block (0,1) largest 1.0, block (0,2) largest 0.5 -> [1, 1, 0.5]
    # (its (0,0) entry, 0.1, or its mean, 0.275, would rank the blocks the other way)
    assert Sj[Sp[0]:Sp[1]].tolist() == [0, 1, 2]
    assert Sx[Sp[0]:Sp[1]].tolist() == [1.0, 1.0, 0.5]
    # with theta = 0.1 the 0.1 entries are weak (0.01 < 0.01 * 16) while 1.0
    # and the 0.5 entries (0.25 >= 0.16) stay strong: same values
    Sp, Sj = O.strength(A.indptr, A.indices, A.data, 2, 0.1)
    Sx = O.strength_values(A.indptr, A.indices, A.data, 2, 0.1, Sp, Sj)
    assert Sx[Sp[0]:Sp[1]].tolist() == [1.0, 1.0, 0.5]
    # with theta = 0.2 the 0.5 entries are weak too (0.25 < 0.64): node 2
    # leaves row 0 and block (0,1) alone sets the scale
    Sp, Sj = O.strength(A.indptr, A.indices, A.data, 2, 0.2)
    Sx = O.strength_values(A.indptr, A.indices, A.data, 2, 0.2, Sp, Sj)
    assert Sj[Sp[0]:Sp[1]].tolist() == [0, 1] and Sx[Sp[0]:Sp[1]].tolist() == [1.0, 1.0]


@pytest.mark.parametrize("name,d", [("laplace1d_8", 2), ("poisson32", 2), ("aniso40", 2), ("elastic7", 2),
                                    ("upwind64", 3), ("poisson37", 1), ("aniso40", 0)])
def test_valued_pattern_equals_dense_product(name, d):
    c = CS.case(name)
    A, m = c["A"], c["m"]
    Sx = O.strength_values(A.rowptr, A.colind, A.vals, m, c["theta"], c["Sp"], c["Sj"])
    nn = c["Sp"].size - 1
    na = c["roots"].size
    Vp, Vj, Vx = O.pattern_values(c["Sp"], c["Sj"], Sx, c["agg"], na, d)
    S = sp.csr_matrix((Sx, c["Sj"], c["Sp"]), shape=(nn, nn)).toarray()
    Cm = np.zeros((nn, na))
    Cm[np.arange(nn), c["agg"]] = 1.0
    ref = np.linalg.matrix_power(S, d) @ Cm
    got = sp.csr_matrix((Vx, Vj, Vp), shape=(nn, na)).toarray()
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(np.max(np.abs(ref)), 1.0)
    # its structure is the boolean pattern N = S^d C
    Bp, Bj = O.pattern_nodes(c["Sp"], c["Sj"], c["agg"], na, d)
    assert np.array_equal(Vp, Bp) and np.array_equal(Vj, Bj)
    # S has non-negative values, unit diagonal and unit largest off entry
    assert np.all(Sx >= 0.0) and np.all(np.diag(S) == 1.0)


def test_prefilter_setup_invariants():
    c = CS.case("aniso40")
    A = c["A"]
    st = O.prefilter_setup(A, c["B"], 1, c["theta"], 2, theta_f=0.1, agg=c["agg"], roots=c["roots"])
    assert st["Nj"].size < c["Nj"].size
    for i in range(A.n_rows):
        r = set(c["Nj"][c["Np"][i]:c["Np"][i + 1]].tolist())
        r2 = st["Nj"][st["Np"][i]:st["Np"][i + 1]].tolist()
        assert set(r2) <= r and c["agg"][i] in r2
    assert np.array_equal(st["is_root"], c["is_root"])
    assert O.constraint_residual(st["Np"], st["Nj"], st["T"], st["Bc"], c["B"]) <= 1e-14
    # no filtering: the unfiltered set-up exactly
    st0 = O.prefilter_setup(A, c["B"], 1, c["theta"], 2, theta_f=0.0, agg=c["agg"], roots=c["roots"])
    assert np.array_equal(st0["Np"], c["Np"]) and np.array_equal(st0["Nj"], c["Nj"])
    assert np.array_equal(st0["T"], c["T"])


def test_prefilter_keeps_the_strong_direction():
    """Rotated anisotropy (eps = 1e-3, angle pi/8): the pre-filter keeps the
    aggregates reached along the strong E-W couplings and drops more of
    those reached only through the weak N-S ones (Sec. 3.5: larger values
    mean a stronger path)."""
    A = W.q1_aniso(40)
    st = O.prefilter_setup(A, W.ones(A.n_rows), 1, 0.1, 2, theta_f=0.3)
    st0 = O.prefilter_setup(A, W.ones(A.n_rows), 1, 0.1, 2, theta_f=0.0)
    assert st["Nj"].size < st0["Nj"].size
    nx = 40
    # own aggregate centre of a row vs the centres of its kept / dropped aggregates
    roots = st["roots"]
    dx_k, dy_k, dx_d, dy_d = [], [], [], []
    for i in range(nx * 10, nx * 30):
        if st["is_root"][i]:
            continue
        kept = set(st["Nj"][st["Np"][i]:st["Np"][i + 1]].tolist())
        for a in st0["Nj"][st0["Np"][i]:st0["Np"][i + 1]]:
            r = roots[a]
            dx, dy = abs(r % nx - i % nx), abs(r // nx - i // nx)
            (dx_k if a in kept else dx_d).append(dx)
            (dy_k if a in kept else dy_d).append(dy)
    assert np.mean(dy_d) > np.mean(dy_k)
