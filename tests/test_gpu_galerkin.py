"""GPU parity of the general sparse product (rn_spgemm) and the Galerkin
coarse operator (rn_galerkin, Sec. 3.8: A_c = R A P) against the oracle,
through the C ABI.

Structures are integer results: bit-exact.  Values: both sides add the terms
of an entry in the order of the left operand's row, from 0, with rounded
products and sums, so they agree exactly; the stated bar is the FP64 one
(max |dA_c| / max |A_c| <= 1e-12) and the achieved difference is printed.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from tests import cases as CS
from tests.test_gpu_parity import dev, dev_matrix, host

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context()


@pytest.mark.parametrize("shape,dens,seed", [((57, 40, 33), (0.12, 0.15), 0), ((1000, 700, 900), (0.01, 0.02), 1),
                                             ((3000, 3000, 50), (0.003, 0.05), 2), ((5, 7, 3), (0.0, 0.5), 3)])
def test_spgemm_matches_oracle(R, ctx, shape, dens, seed):
    rows, inner, cols = shape
    X = sp.random(rows, inner, dens[0], format="csr", random_state=seed)
    Y = sp.random(inner, cols, dens[1], format="csr", random_state=seed + 7)
    X.sort_indices()
    Y.sort_indices()
    Cp, Cj, Cx = O.spgemm(X.indptr, X.indices, X.data, Y.indptr, Y.indices, Y.data, cols)
    i32 = lambda a: dev(np.asarray(a, np.int32))
    Gp, Gj, Gx = ctx.spgemm(i32(X.indptr), i32(X.indices), dev(X.data), i32(Y.indptr), i32(Y.indices), dev(Y.data),
                            cols)
    assert np.array_equal(host(Gp), Cp) and np.array_equal(host(Gj), Cj)
    d = float(np.max(np.abs(host(Gx) - Cx))) if Cx.size else 0.0
    print(f"{shape}: nnz(C) {Cj.size}, max |dC| {d:.1e}")
    assert d <= FP64_TOL * max(float(np.max(np.abs(Cx))) if Cx.size else 0.0, 1e-300)
    # structure only
    Sp, Sj, Sx = ctx.spgemm(i32(X.indptr), i32(X.indices), None, i32(Y.indptr), i32(Y.indices), None, cols)
    assert Sx is None and np.array_equal(host(Sp), Cp) and np.array_equal(host(Sj), Cj)


GAL_CASES = ["poisson32", "aniso40", "upwind64", "elastic7", "twocand13", "lap27_10", "aniso512", "upwind1024",
             "elastic512"]


@pytest.mark.parametrize("name", GAL_CASES)
def test_galerkin_matches_oracle(R, ctx, name):
    c = CS.case(name)
    A = c["A"]
    nc = c["nc"]
    has_rt = c.get("RT") is not None
    if has_rt:
        Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], nc, c["Np"], c["Nj"], c["RT"])
    else:
        Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], nc)
    Ad = dev_matrix(R, c)  # node-blocked for the elasticity cases
    Gp, Gj, Gx = ctx.galerkin(Ad, nc, dev(c["Np"]), dev(c["Nj"]), dev(c["P"]), dev(c["RT"]) if has_rt else None)
    assert np.array_equal(host(Gp), Cp) and np.array_equal(host(Gj), Cj)
    err = CS.rel_max(host(Gx), Cx)
    print(f"{name}: A_c {nc} x {nc}, nnz {Cj.size}, max|dA_c|/max|A_c| = {err:.1e}")
    assert err <= FP64_TOL


def test_galerkin_of_gpu_setup(R, ctx):
    """The full level on the GPU (set-up, then A_c from the GPU's own P)
    against the oracle's A_c from the oracle's P."""
    c = CS.case("aniso512")
    A = c["A"]
    Cp, Cj, Cx = O.galerkin(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["P"], c["nc"])
    s = ctx.setup_native(dev_matrix(R, c), dev(c["B"]), dev(c["agg"]), dev(c["roots"]), c["theta"], c["degree"],
                         c["iters"], R.RN_CG, R.RN_FP64)
    Gp, Gj, Gx = ctx.galerkin(dev_matrix(R, c), c["nc"], s.tensor("N_rowptr"), s.tensor("N_colind"), s.tensor("P"))
    assert np.array_equal(host(Gp), Cp) and np.array_equal(host(Gj), Cj)
    err = CS.rel_max(host(Gx), Cx)
    print(f"aniso512 from the GPU's P: max|dA_c|/max|A_c| = {err:.1e}")
    assert err <= FP64_TOL
    s.close()
