"""GPU multilevel set-up (rn_hierarchy_build; Alg. root_node_setup level by
level, A_c = R A P of Sec. 3.8) against the oracle, through the C ABI.

Every level is checked on its own inputs (the GPU's A_l and B_l): the host
aggregation on the oracle's strength graph bit for bit, the pattern bit for
bit, P (and R^T) at the FP64 bars, the next operator equal to the oracle's
Galerkin product of the GPU's P and the next candidates equal to Bc; the
level count follows the stopping rules, and the operator complexity (Sec.
2.4) is the count of the levels' entries.  Where strength keeps the whole
structure (theta = 0) the oracle's own hierarchy is compared end to end.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS
from tests.test_gpu_parity import FP64_TOL, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context()


def _problem(name):
    if name == "aniso64":
        A = W.q1_aniso(64)
        return A, None, W.ones(A.n_rows), 1, 0.1, 4, "cg"
    if name == "poisson48":
        A = W.poisson5(48)
        return A, None, W.ones(A.n_rows), 1, 0.0, 4, "cg"
    if name == "upwind48":
        A = W.upwind_cd(48)
        return A, None, W.ones(A.n_rows), 1, 0.0, 4, "gmres"
    if name == "elastic16":
        Ab, xy = W.q1_elasticity(16)
        return Ab.to_csr(), Ab, W.rbm(xy), 2, 0.0, 3, "cg"
    if name == "aniso512":
        A = W.q1_aniso(512)
        return A, None, W.ones(A.n_rows), 1, 0.1, 6, "cg"
    raise KeyError(name)


def _build(R, ctx, name, max_levels, min_coarse):
    A, Ab, B, m, theta, K, method = _problem(name)
    if m == 2:
        dA = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=Ab.n_nodes * 2, block_m=2)
    else:
        dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    meth = R.RN_CG if method == "cg" else R.RN_GMRES
    h = ctx.hierarchy(dA, dev(np.ascontiguousarray(B, np.float64)), max_levels=max_levels, min_coarse=min_coarse,
                      theta=theta, degree=2, iters=K, method=meth)
    return A, B, m, theta, K, method, h, dA


CASES = [("aniso64", 5, 20), ("poisson48", 6, 16), ("upwind48", 4, 16), ("elastic16", 4, 24), ("aniso512", 4, 500)]


@pytest.mark.parametrize("name,max_levels,min_coarse", CASES)
def test_levels_against_the_oracle(R, ctx, name, max_levels, min_coarse):
    A0, B0, m0, theta, K, method, h, _ = _build(R, ctx, name, max_levels, min_coarse)
    nl = h.n_levels
    levels = [h.level(l) for l in range(nl)]
    assert nl >= 2
    nnz_scalar = []
    for l, lv in enumerate(levels):
        m = lv["block_m"]
        assert m == (m0 if l == 0 else 1)
        if l == 0:
            A = A0
        else:
            A = W.CSR(lv["n"], lv["n"], host(lv["A_rowptr"]), host(lv["A_colind"]), host(lv["A_vals"]))
        B = host(lv["B"])
        nnz_scalar.append(A.nnz)
        last = l == nl - 1
        if l > 0:  # the operator and candidates handed down from the level above
            prev, pA = levels[l - 1], levels_A[-1]
            Np, Nj = host(prev["N_rowptr"]), host(prev["N_colind"])
            rt = () if prev["RT"] is None else (Np, Nj, host(prev["RT"]))
            Cp, Cj, Cx = O.galerkin(pA.rowptr, pA.colind, pA.vals, Np, Nj, host(prev["P"]), prev["n_cols"], *rt)
            assert np.array_equal(Cp, A.rowptr) and np.array_equal(Cj, A.colind)
            assert np.max(np.abs(Cx - A.vals)) <= 1e-14 * np.max(np.abs(Cx))
            assert np.array_equal(host(prev["Bc"]), B)
        levels_A = (levels_A if l > 0 else []) + [A]
        # the level's own set-up on its inputs
        Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, m, theta)
        agg, roots = O.aggregate(Sp, Sj)
        coarsens = roots.size > 0 and m * roots.size < A.n_rows
        if last:
            assert l == h.n_levels - 1
            assert l + 1 == max_levels or A.n_rows <= min_coarse or not coarsens
            assert "P" not in lv
            continue
        assert A.n_rows > min_coarse and coarsens
        assert np.array_equal(host(lv["agg"]), agg) and np.array_equal(host(lv["roots"]), roots)
        st = O.setup(A, B, m, theta, 2, agg=agg, roots=roots)
        assert np.array_equal(host(lv["N_rowptr"]), st["Np"]) and np.array_equal(host(lv["N_colind"]), st["Nj"])
        nB = B.shape[1]
        args = (st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], nB, st["T"], K)
        tol = CS.ELASTIC_FP64_TOL if (name.startswith("elastic") and l == 0) else FP64_TOL
        if method == "cg":
            P, info = O.emin_cg(A.rowptr, A.colind, A.vals, *args)
            assert info["status"] == 0
        else:
            P, _ = O.emin_gmres(A.rowptr, A.colind, A.vals, *args)
            Tp, Tj, Tx = O.transpose(A.rowptr, A.colind, A.vals)
            RT, _ = O.emin_gmres(Tp, Tj, Tx, *args)
            assert CS.rel_max(host(lv["RT"]), RT) <= tol
        err = CS.rel_max(host(lv["P"]), P)
        print(f"{name} level {l}: n {A.n_rows}, nnz {A.nnz}, aggregates {roots.size}, max|dP|/max|P| = {err:.2e}")
        assert err <= tol
        assert lv["stats"].status_code == 0
    ref = sum(nnz_scalar) / nnz_scalar[0]
    assert h.operator_complexity() == pytest.approx(ref, rel=1e-14)
    h.close()


def test_structure_strength_matches_the_oracle_hierarchy(R, ctx):
    """theta = 0 (strength is A's structure): the oracle's own hierarchy has
    the same level sizes and nonzeros and operators to round-off."""
    A0, B0, m0, theta, K, method, h, _ = _build(R, ctx, "poisson48", 6, 16)
    ref = O.hierarchy(A0, B0, m=1, theta=0.0, degree=2, iters=K, method="cg", max_levels=6, min_coarse=16)
    assert h.n_levels == len(ref)
    for l, r in enumerate(ref):
        lv = h.level(l)
        assert lv["n"] == r["A"].n_rows and lv["nnz_A"] == r["A"].nnz
        assert np.array_equal(host(lv["A_colind"]), r["A"].colind)
        vals = host(lv["A_vals"])
        assert np.max(np.abs(vals - r["A"].vals)) <= 1e-12 * np.max(np.abs(r["A"].vals))
    assert h.operator_complexity() == pytest.approx(O.operator_complexity(ref), rel=1e-14)
    h.close()


def test_argument_errors(R, ctx):
    A = W.poisson5(8)
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    B = dev(W.ones(A.n_rows))
    for kw in (dict(max_levels=0), dict(min_coarse=-1), dict(method=R.RN_PCG_JACOBI)):
        with pytest.raises(R.RnError) as e:
            ctx.hierarchy(dA, B, **kw)
        assert e.value.status == R._lib.RN_EINVAL
    Ab, xy = W.q1_elasticity(6)
    dAb = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=Ab.n_nodes * 2, block_m=2)
    with pytest.raises(R.RnError) as e:  # R^T on A^T needs a scalar CSR operator
        ctx.hierarchy(dAb, dev(W.rbm(xy)), method=R.RN_GMRES)
    assert e.value.status == R._lib.RN_EINVAL
    one = ctx.hierarchy(dA, B, max_levels=1)
    assert one.n_levels == 1 and "P" not in one.level(0)
    assert one.operator_complexity() == 1.0
    one.close()
