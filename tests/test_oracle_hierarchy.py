"""Pins of the oracle's multilevel set-up (CPU only): Alg. root_node_setup
applied level by level with A_c = R A P (Sec. 3.8), and its operator
complexity (Sec. 2.4).

The levels are compositions of functions pinned elsewhere; here the
composition itself is pinned: the two-level example's coarse size and
nonzero count (Sec. 2.3, `tests/golden/`), every coarse operator equal to
the dense triple product of the level above, the coarse candidates carried
down (A_c Bc = P^T A B with P Bc = B), symmetry for symmetric A, the GMRES
branch with R = (R^T)^T, a node-blocked finest level, the stopping rules,
and the complexity as a hand count.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def dense(A):
    return A.to_dense()


def dense_p(Np, Nj, V, nc):
    n = Np.size - 1
    D = np.zeros((n, nc))
    for i in range(n):
        D[i, Nj[Np[i]:Np[i + 1]]] = V[Np[i]:Np[i + 1]]
    return D


def test_two_level_example():
    """Sec. 2.3: Q1 Laplacian on 50 x 50, every neighbour strong, B = 1,
    pattern C (degree 0) and no smoothing steps: 289 coarse DOFs and 2401
    stored entries in the coarse operator."""
    g = json.load(open(os.path.join(GOLD, "e2_q1_laplace50.json")))
    A = W.q1_aniso(g["nx"], 1.0, 0.0)
    lv = O.hierarchy(A, W.ones(A.n_rows), theta=0.0, degree=0, iters=0, max_levels=2, min_coarse=1)
    assert len(lv) == 2
    assert lv[1]["A"].n_rows == g["n_agg"]
    assert lv[1]["A"].nnz == g["nnz_coarse_one_candidate"]
    assert O.operator_complexity(lv) == pytest.approx((A.nnz + g["nnz_coarse_one_candidate"]) / A.nnz, rel=1e-15)


# (on the Galerkin operators of smoothed P no off-diagonal entry reaches
# theta = 0.25 of the diagonal, so the Poisson case coarsens by structure)
@pytest.mark.parametrize("name,theta,K", [("poisson", 0.0, 4), ("aniso", 0.1, 3)])
def test_coarse_operators_are_dense_triple_products(name, theta, K):
    A = W.poisson5(24) if name == "poisson" else W.q1_aniso(30)
    B = W.ones(A.n_rows)
    lv = O.hierarchy(A, B, theta=theta, degree=2, iters=K, max_levels=6, min_coarse=20)
    assert len(lv) >= 3
    sizes = [l["A"].n_rows for l in lv]
    assert all(a > b for a, b in zip(sizes, sizes[1:]))
    assert sizes[-1] <= 20 or len(lv) == 6
    for a, b in zip(lv, lv[1:]):
        st = a["setup"]
        Ad = dense(a["A"])
        Pd = dense_p(st["Np"], st["Nj"], a["P"], st["nc"])
        Ac = Pd.T @ Ad @ Pd
        got = dense(b["A"])
        assert np.max(np.abs(got - Ac)) <= 1e-12 * np.max(np.abs(Ac))
        # symmetric A: symmetric coarse operator (to the rounding of two sum orders)
        assert np.max(np.abs(got - got.T)) <= 1e-14 * np.max(np.abs(got))
        # the coarse candidates: P Bc = B, so A_c Bc = P^T A B
        Bc = b["B"]
        assert np.max(np.abs(Pd @ Bc - a["B"])) <= 1e-12
        lhs, rhs = got @ Bc, Pd.T @ (Ad @ a["B"])
        assert np.max(np.abs(lhs - rhs)) <= 1e-10 * max(1.0, np.max(np.abs(rhs)))


def test_gmres_branch_uses_R_from_RT():
    A = W.upwind_cd(24)
    lv = O.hierarchy(A, W.ones(A.n_rows), theta=0.0, degree=2, iters=4, method="gmres", max_levels=3,
                     min_coarse=10)
    assert len(lv) == 3
    for a, b in zip(lv, lv[1:]):
        st = a["setup"]
        Pd = dense_p(st["Np"], st["Nj"], a["P"], st["nc"])
        RTd = dense_p(st["Np"], st["Nj"], a["RT"], st["nc"])
        assert a["RT"] is not None and np.max(np.abs(RTd - Pd)) > 1e-6  # non-symmetric A: R != P^T
        Ac = RTd.T @ dense(a["A"]) @ Pd
        assert np.max(np.abs(dense(b["A"]) - Ac)) <= 1e-12 * np.max(np.abs(Ac))
        # the left candidates are kept too: R^T Bc = B
        assert np.max(np.abs(RTd @ b["B"] - a["B"])) <= 1e-12


def test_node_blocked_finest_level():
    """Elasticity (m = 2, three rigid-body modes): the coarse level is scalar
    with 2 DOFs per aggregate and carries the three coarse candidates."""
    c = CS.case("elastic7")
    A = c["A"]
    lv = O.hierarchy(A, c["B"], m=2, theta=0.0, degree=2, iters=3, max_levels=2, min_coarse=1)
    assert len(lv) == 2 and lv[1]["m"] == 1
    st = lv[0]["setup"]
    assert lv[1]["A"].n_rows == 2 * st["roots"].size and lv[1]["B"].shape == (2 * st["roots"].size, 3)
    Pd = dense_p(st["Np"], st["Nj"], lv[0]["P"], st["nc"])
    Ac = Pd.T @ dense(A) @ Pd
    assert np.max(np.abs(dense(lv[1]["A"]) - Ac)) <= 1e-12 * np.max(np.abs(Ac))


def test_stopping_rules_and_complexity():
    A = W.poisson5(16)
    B = W.ones(A.n_rows)
    one = O.hierarchy(A, B, max_levels=1)
    assert len(one) == 1 and "P" not in one[0]
    small = O.hierarchy(A, B, min_coarse=A.n_rows)  # already coarse enough
    assert len(small) == 1
    # at theta = 0.25 the Galerkin operator of the first level has no strong
    # off-diagonal entry: one aggregate per row, no coarsening, the set-up ends
    lv = O.hierarchy(A, B, theta=0.25, iters=2, max_levels=10, min_coarse=4)
    assert len(lv) == 2 and lv[1]["A"].n_rows > 4 and "setup" not in lv[1]
    st = O.setup(lv[1]["A"], lv[1]["B"], 1, 0.25, 2)
    assert st["nc"] == lv[1]["A"].n_rows
    lv = O.hierarchy(A, B, theta=0.0, iters=2, max_levels=10, min_coarse=4)
    assert lv[-1]["A"].n_rows <= 4
    nnz = [l["A"].nnz for l in lv]
    assert O.operator_complexity(lv) == pytest.approx(sum(nnz) / nnz[0], rel=1e-15)
