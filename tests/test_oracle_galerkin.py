"""Pins of the oracle's sparse product and Galerkin coarse operator (Sec. 3.8,
A_c = R A P), CPU only: against scipy's sparse product and numpy's dense
product (library routines computing the same products), the coarse-operator
size the paper prints for its two-level example, and identities of the
Galerkin product."""
import json
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
import workloads as W
from tests import cases as CS

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _csr(p, j, x, shape):
    return sp.csr_matrix((x, j, p), shape=shape)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_spgemm_equals_scipy(seed):
    X = sp.random(57, 40, 0.12, format="csr", random_state=seed)
    Y = sp.random(40, 33, 0.15, format="csr", random_state=seed + 10)
    Cp, Cj, Cx = O.spgemm(X.indptr, X.indices, X.data, Y.indptr, Y.indices, Y.data, 33)
    Z = (X @ Y).tocsr()
    Z.sort_indices()
    assert np.array_equal(Cp, Z.indptr) and np.array_equal(Cj, Z.indices)
    assert np.max(np.abs(Cx - Z.data)) <= 1e-15 * np.max(np.abs(Z.data))


def test_spgemm_structure_keeps_cancelled_entries():
    # x = [1, -1] times rows [1], [1] of Y: the sum is exactly 0 but the entry
    # is structurally present (the product's pattern is the boolean one)
    Cp, Cj, Cx = O.spgemm([0, 2], [0, 1], [1.0, -1.0], [0, 1, 2], [0, 0], [1.0, 1.0], 1)
    assert Cp.tolist() == [0, 1] and Cj.tolist() == [0] and Cx.tolist() == [0.0]
    Cp, Cj, _ = O.spgemm([0, 2, 2], [0, 1], None, [0, 1, 3], [2, 0, 2], None, 3)
    assert Cp.tolist() == [0, 2, 2] and Cj.tolist() == [0, 2]


@pytest.mark.parametrize("name", ["poisson32", "upwind64", "elastic7"])
def test_galerkin_equals_dense_product(name):
    c = CS.case(name)
    A = c["A"]
    n, nc = A.n_rows, c["nc"]
    Pd = _csr(c["Np"], c["Nj"], c["P"], (n, nc)).toarray()
    Ad = _csr(A.rowptr, A.colind, A.vals, (n, n)).toarray()
    if c.get("RT") is not None:
        Rd = _csr(c["Np"], c["Nj"], c["RT"], (n, nc)).toarray().T
        Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], nc, c["Np"], c["Nj"], c["RT"])
    else:
        Rd = Pd.T
        Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], nc)
    ref = Rd @ Ad @ Pd
    got = _csr(Cp, Cj, Cx, (nc, nc)).toarray()
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    # the structure is the boolean product's (a superset of the nonzeros)
    assert np.all((ref != 0) <= (got != 0) | (np.abs(ref) < 1e-14 * np.max(np.abs(ref))))


def test_two_level_example_coarse_size():
    """Sec. 2.3's example: Q1 Laplacian on 50 x 50, every neighbour strong,
    289 aggregates; the tentative operator with one candidate (B = 1, pattern
    C) gives a coarse operator with 2401 nonzeros."""
    g = json.load(open(os.path.join(GOLD, "e2_q1_laplace50.json")))
    A = W.q1_aniso(g["nx"], 1.0, 0.0)
    st = O.setup(A, W.ones(A.n_rows), 1, 0.0, 0)  # degree 0: the pattern of C itself
    assert st["roots"].size == g["n_agg"]
    assert np.all(st["T"] == 1.0)  # T = C for B = 1
    Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["T"], st["nc"])
    assert Cj.size == g["nnz_coarse_one_candidate"]


@pytest.mark.parametrize("name", ["aniso40", "elastic7", "twocand13"])
def test_galerkin_maps_coarse_candidates(name):
    """With P Bc = B, A_c Bc = P^T A P Bc = P^T (A B) (Eq. mode_constraint)."""
    c = CS.case(name)
    A = c["A"]
    n, nc = A.n_rows, c["nc"]
    Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], nc)
    Ac = _csr(Cp, Cj, Cx, (nc, nc))
    P = _csr(c["Np"], c["Nj"], c["P"], (n, nc))
    As = _csr(A.rowptr, A.colind, A.vals, (n, n))
    lhs = Ac @ c["Bc"]
    rhs = P.T @ (As @ c["B"])
    assert np.max(np.abs(lhs - rhs)) <= 1e-12 * max(np.max(np.abs(rhs)), np.max(np.abs(Ac.data)))
    # symmetric A, R = P^T: A_c is symmetric up to the order of its sums
    D = (Ac - Ac.T).tocsr()
    assert (np.max(np.abs(D.data)) if D.nnz else 0.0) <= 1e-13 * np.max(np.abs(Ac.data))
