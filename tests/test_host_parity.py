"""Host-side library code against the oracle, on the CPU (no GPU needed).

rn_aggregate_host (the library's greedy root-node aggregation, Sec. 3.3) runs
on the host; it feeds the set-up whenever the caller brings no aggregation,
so it is compared with the oracle's aggregation here, element by element.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _library_aggregate(Sp, Sj):
    import paper_1610_03154_amd as R
    return R.aggregate_host(Sp, Sj)


def _graphs():
    g1 = json.load(open(os.path.join(GOLD, "e1_laplace1d.json")))
    g2 = json.load(open(os.path.join(GOLD, "e2_q1_laplace50.json")))
    A1 = W.laplace1d(g1["n"])
    yield "e1", O.strength(A1.rowptr, A1.colind, A1.vals, 1, 0.0)
    A2 = W.q1_aniso(g2["nx"], 1.0, 0.0)
    yield "e2", O.strength(A2.rowptr, A2.colind, A2.vals, 1, 0.0)
    A = W.q1_aniso(512)
    yield "aniso512", O.strength(A.rowptr, A.colind, A.vals, 1, 0.1)
    Ab, _ = W.q1_elasticity(64)
    A = Ab.to_csr()
    yield "elastic64_theta0.3", O.strength(A.rowptr, A.colind, A.vals, 2, 0.3)
    A = W.upwind_cd(128)
    yield "upwind128", O.strength(A.rowptr, A.colind, A.vals, 1, 0.0)
    A = W.ring_graph(5000)
    yield "ring5000", O.strength(A.rowptr, A.colind, A.vals, 1, 0.0)


@pytest.mark.parametrize("name,S", list(_graphs()), ids=lambda x: x if isinstance(x, str) else "")
def test_aggregate_host_matches_oracle(name, S):
    Sp, Sj = S
    agg_o, roots_o = O.aggregate(Sp, Sj)
    agg_l, roots_l = _library_aggregate(Sp, Sj)
    assert np.array_equal(agg_l, agg_o)
    assert np.array_equal(roots_l, roots_o)


def test_aggregate_host_empty_and_isolated():
    # no nodes; and a graph of isolated nodes (each its own root)
    agg, roots = _library_aggregate(np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert agg.size == 0 and roots.size == 0
    n = 5
    Sp = np.arange(n + 1, dtype=np.int32)
    Sj = np.arange(n, dtype=np.int32)
    agg, roots = _library_aggregate(Sp, Sj)
    ao, ro = O.aggregate(Sp, Sj)
    assert np.array_equal(agg, ao) and np.array_equal(roots, ro) and roots.size == n


def test_aggregate_host_rejects_bad_graph():
    import paper_1610_03154_amd as R
    with pytest.raises(R.RnError):
        R.aggregate_host(np.array([0, 2], np.int32), np.array([0, 3], np.int32))
