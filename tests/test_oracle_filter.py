"""Pins of the oracle's filter, compaction and enforce (Alg. filter, Sec. 3.5
and Sec. 3.7; Eq. Tproj), CPU only.

Each expected value below is worked out by hand from the definitions, or
comes from a library routine that solves the same problem (the minimum-norm
least-squares solution of numpy), or from an invariant the paper states.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS

ROW = dict(Np=np.array([0, 5]), Nj=np.array([0, 1, 2, 3, 4]))
# row of aggregate 1: own entry 0.5 at column 1; off magnitudes 0.4, 0.02, 0.1, 0.04
VALS = np.array([-0.4, 0.5, 0.02, 0.1, -0.04])


def test_theta_drops_below_theta_times_largest_off_entry_ties_kept():
    # largest off magnitude 0.4; 0.25 * 0.4 == 0.1 exactly, and 0.1 is kept
    keep = O.filter_keep(ROW["Np"], ROW["Nj"], VALS, [1], 1, 0, 0.25)
    assert keep.tolist() == [True, True, False, True, False]
    keep = O.filter_keep(ROW["Np"], ROW["Nj"], VALS, [1], 1, 0, 0.26)
    assert keep.tolist() == [True, True, False, False, False]


@pytest.mark.parametrize("k,want", [(1, [1, 1, 0, 0, 0]), (2, [1, 1, 0, 1, 0]), (3, [1, 1, 0, 1, 1]),
                                    (4, [1, 1, 1, 1, 1]), (9, [1, 1, 1, 1, 1])])
def test_k_keeps_the_k_largest_off_entries(k, want):
    keep = O.filter_keep(ROW["Np"], ROW["Nj"], VALS, [1], 1, k, 0.0)
    assert keep.astype(int).tolist() == want


def test_both_rules_together():
    # k = 3 keeps 0.4, 0.1, 0.04; theta = 0.2 then drops 0.04 (< 0.08)
    keep = O.filter_keep(ROW["Np"], ROW["Nj"], VALS, [1], 1, 3, 0.2)
    assert keep.astype(int).tolist() == [1, 1, 0, 1, 0]


def test_own_aggregate_entry_is_kept_and_not_an_off_entry():
    Np, Nj = np.array([0, 3]), np.array([0, 1, 2])
    G = np.array([0.001, 0.9, 0.5])  # own aggregate 0 holds the smallest value
    keep = O.filter_keep(Np, Nj, G, [0], 1, 0, 0.6)
    assert keep.tolist() == [True, True, False]
    # if the own entry counted as the row maximum, 0.9 would be the only off
    # entry and k = 1 would keep it; own excluded: k = 1 keeps 0.9, drops 0.5
    keep = O.filter_keep(Np, Nj, G, [0], 1, 1, 0.0)
    assert keep.tolist() == [True, True, False]


def test_root_rows_and_empty_rows_are_kept():
    Np = np.array([0, 3, 3, 5])
    Nj = np.array([0, 1, 2, 0, 1])
    G = np.array([1.0, 1e-9, 1e-9, 0.1, 0.9])
    keep = O.filter_keep(Np, Nj, G, [0, 0, 1], 1, 0, 0.5, is_root=np.array([1, 0, 0], np.uint8))
    # row 0 is a root row: kept whole; row 2 (aggregate 1): own 0.9, off 0.1 kept (only off entry)
    assert keep.tolist() == [True, True, True, True, True]


def test_node_blocks_use_the_largest_entry_of_the_block():
    # one node row (DOF rows 0, 1) of aggregate 0 with node entries at node
    # columns 0 (own), 1 and 2; DOF columns 2a, 2a+1 interleaved
    Np = np.array([0, 6, 12])
    Nj = np.array([0, 1, 2, 3, 4, 5] * 2)
    G = np.array([[0.7, 0.0, 0.0, 0.3, 0.05, 0.05],
                  [0.0, 0.7, 0.0, 0.0, 0.05, -0.05]]).ravel()
    # block 1 has a single large entry (0.3), block 2 four entries of 0.05:
    # largest off block 0.3, threshold 0.2 * 0.3 = 0.06 -> block 2 dropped
    keep = O.filter_keep(Np, Nj, G, [0], 2, 0, 0.2)
    assert keep.astype(int).tolist() == [1, 1, 1, 1, 0, 0] * 2
    # (a rule reading one entry per block, or the block mean, would instead
    # drop block 1, whose (0,0) entry and mean are below those of block 2)
    # with a lower threshold, 0.1 * 0.3 = 0.03, block 2 stays
    keep = O.filter_keep(Np, Nj, G, [0], 2, 0, 0.1)
    assert keep.astype(int).tolist() == [1] * 12


def test_compact_keeps_order_and_values():
    Np = np.array([0, 3, 5])
    Nj = np.array([0, 2, 3, 1, 4])
    V = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    Np2, Nj2, V2 = O.compact(Np, Nj, [True, False, True, False, True], V)
    assert Np2.tolist() == [0, 2, 3] and Nj2.tolist() == [0, 3, 4] and V2.tolist() == [1.0, 3.0, 5.0]


def test_enforce_single_candidate_by_hand():
    # B = 1, Bc = [1, 2]: t = [0.5, 0.1] has t Bc = 0.7; r = 0.3, G = 5,
    # u = 0.3 / 5 * [1, 2] = [0.06, 0.12]
    Np, Nj = np.array([0, 2]), np.array([0, 1])
    V, rd = O.enforce(Np, Nj, np.zeros(1, np.uint8), np.array([[1.0], [2.0]]), np.ones((1, 1)), [0.5, 0.1])
    assert rd == 0
    assert np.allclose(V, [0.56, 0.22], rtol=0, atol=1e-15)
    # unit Bc: the deficit is shared equally
    V, _ = O.enforce(Np, Nj, np.zeros(1, np.uint8), np.ones((2, 1)), np.ones((1, 1)), [0.6, 0.3])
    assert np.allclose(V, [0.65, 0.35], rtol=0, atol=1e-15)


def test_enforce_is_the_minimum_norm_least_squares_update():
    rng = np.random.default_rng(3)
    n, nc, nB = 6, 9, 3
    Np = np.array([0, 1, 6, 11, 15, 16, 22])
    Nj = np.concatenate([[4], [0, 2, 3, 5, 8], [1, 2, 4, 6, 7], [0, 3, 5, 8], [2], [0, 1, 3, 4, 6, 8]])
    is_root = np.array([1, 0, 0, 0, 1, 0], np.uint8)
    Bc = rng.standard_normal((nc, nB))
    B = rng.standard_normal((n, nB))
    V0 = rng.standard_normal(Np[-1])
    V, rd = O.enforce(Np, Nj, is_root, Bc, B, V0)
    assert rd == 0
    for i in range(n):
        s, e = Np[i], Np[i + 1]
        if is_root[i]:
            assert np.array_equal(V[s:e], V0[s:e])
            continue
        BJ = Bc[Nj[s:e]]
        r = B[i] - V0[s:e] @ BJ
        u = np.linalg.lstsq(BJ.T, r, rcond=None)[0]  # minimum-norm solution of BJ^T u = r
        assert np.allclose(V[s:e], V0[s:e] + u, rtol=0, atol=1e-13)
        assert np.allclose(V[s:e] @ BJ, B[i], rtol=0, atol=1e-13)


def test_postfilter_pipeline_invariants():
    """Sec. 3.7 on the 40 x 40 anisotropic case: the filtered pattern is a
    subset holding every own-aggregate entry, enforce restores P Bc = B, the
    extra CG step keeps it and lowers the energy, root rows stay identity."""
    c = CS.case("aniso40")
    A = c["A"]
    Np2, Nj2, Pe, Pn, info = O.postfilter(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["agg"], 1,
                                          c["nc"], c["Bc"], c["B"], c["P"], theta=0.1)
    assert info["status"] == 0 and info["iters"] == 1
    assert Nj2.size < c["Nj"].size
    for i in range(c["Np"].size - 1):
        row = set(c["Nj"][c["Np"][i]:c["Np"][i + 1]].tolist())
        row2 = Nj2[Np2[i]:Np2[i + 1]].tolist()
        assert set(row2) <= row and c["agg"][i] in row2
    assert O.constraint_residual(Np2, Nj2, Pe, c["Bc"], c["B"]) <= 1e-12
    assert O.constraint_residual(Np2, Nj2, Pn, c["Bc"], c["B"]) <= 1e-12
    e0 = O.energy(A.rowptr, A.colind, A.vals, Np2, Nj2, c["nc"], Pe)
    e1 = O.energy(A.rowptr, A.colind, A.vals, Np2, Nj2, c["nc"], Pn)
    assert e1 < e0
    roots = np.flatnonzero(c["is_root"])
    assert np.all(Pn[Np2[roots]] == 1.0) and np.all(np.diff(Np2)[roots] == 1)


def test_postfilter_without_dropping_changes_nothing():
    c = CS.case("poisson32")
    A = c["A"]
    Np2, Nj2, Pe, _, _ = O.postfilter(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["agg"], 1,
                                      c["nc"], c["Bc"], c["B"], c["P"], theta=0.0)
    assert np.array_equal(Np2, c["Np"]) and np.array_equal(Nj2, c["Nj"])
    assert np.max(np.abs(Pe - c["P"])) <= 1e-14


def test_postfilter_elasticity_three_candidates():
    """Node-blocked elasticity (m = 2, three rigid-body modes): the filter
    keeps whole node blocks and enforce restores all three constraints."""
    c = CS.case("elastic7")
    A = c["A"]
    Np2, Nj2, Pe, Pn, info = O.postfilter(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["agg"], 2,
                                          c["nc"], c["Bc"], c["B"], c["P"], theta=0.5)
    assert info["status"] == 0
    assert Nj2.size < c["Nj"].size
    rows = np.diff(Np2)
    assert np.all(rows % 2 == 0) or np.all(rows[c["is_root"] == 1] == 1)
    F = c["is_root"] == 0
    assert np.array_equal(rows[0::2][F[0::2]], rows[1::2][F[1::2]])
    assert O.constraint_residual(Np2, Nj2, Pe, c["Bc"], c["B"]) <= 1e-12
    assert O.constraint_residual(Np2, Nj2, Pn, c["Bc"], c["B"]) <= 1e-12
