"""GPU parity of the variants against the oracle, through the C ABI:
candidate smoothing (rn_smooth_candidates: same sums in the same order, so
bit-exact), Jacobi-preconditioned CG (RN_PCG_JACOBI) and CGNR (RN_CGNR) at the
FP64 bars (1e-12; the node-blocked elasticity bar where its FP64 spread is
wider), with their Krylov histories."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS
from tests.test_gpu_parity import dev, dev_matrix, host, run_path

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12


def tol(name):
    return CS.ELASTIC_FP64_TOL if name.startswith("elastic") else FP64_TOL


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


@pytest.fixture(scope="module")
def ctx(R):
    return R.Context()


@pytest.mark.parametrize("name,nB,sweeps", [("poisson32", 1, 4), ("aniso40", 2, 4), ("elastic7", 3, 3),
                                            ("upwind64", 1, 5), ("aniso512", 2, 4), ("elastic512", 3, 4)])
def test_smooth_candidates_bit_exact(R, ctx, name, nB, sweeps):
    c = CS.case(name)
    A = c["A"]
    B0 = np.random.default_rng(2).standard_normal((A.n_rows, nB)) if nB != c["B"].shape[1] else c["B"]
    ref = O.smooth_candidates(A.rowptr, A.colind, A.vals, B0, sweeps, 2.0 / 3.0)
    B = dev(np.ascontiguousarray(B0, np.float64))
    ctx.smooth_candidates(dev_matrix(R, c), B, sweeps, 2.0 / 3.0)
    assert np.array_equal(host(B), ref)


def test_smooth_candidates_zero_diagonal(R, ctx):
    import torch
    A = W.laplace1d(6)
    vals = A.vals.copy()
    vals[(A.colind == 2) & (np.repeat(np.arange(6), np.diff(A.rowptr)) == 2)] = 0.0
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, vals)
    with pytest.raises(R.RnError) as e:
        ctx.smooth_candidates(dA, torch.ones((6, 1), dtype=torch.float64, device="cuda"), 2, 0.5)
    assert e.value.status == R._lib.RN_ESINGULAR


PCG_CASES = ["poisson32", "aniso40", "twocand13", "elastic7", "elastic32", "lap27_10", "aniso512", "elastic512"]


@pytest.mark.parametrize("name", PCG_CASES)
def test_pcg_jacobi(R, ctx, name):
    c = CS.case(name)
    A = c["A"]
    K = c["iters"]
    ref, info = O.emin_pcg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                           c["B"].shape[1], c["T"], K)
    assert info["status"] == 0
    g = run_path(R, ctx, c)
    P, st, hist = ctx.energy_min(g["plan"], g["A"].vals, g["T"], R.RN_PCG_JACOBI, K, R.RN_FP64, want_hist=True)
    err = CS.rel_max(host(P), ref)
    print(f"{name}: PCG(Jacobi) {st.iters_done} steps, max|dP|/max|P| = {err:.2e}")
    assert st.iters_done == info["iters"]
    assert err <= tol(name)
    h = host(hist)[0]
    it = info["iters"]
    assert np.allclose(h[:it + 1], info["gamma"][:it + 1], rtol=1e-9, atol=0)
    assert np.allclose(h[1 + K:1 + K + it], info["delta"][:it], rtol=1e-9, atol=0)
    g["plan"].close()


def test_pcg_batched(R, ctx):
    A0, vals, _, _ = W.aniso_batch(32, 3, 0)
    st = O.setup(A0, W.ones(A0.n_rows), 1, 0.0, 2)
    dA = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    Np, Nj, isr = dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"])
    plan = ctx.plan(dA, st["nc"], Np, Nj, isr, dev(st["Bc"]))
    P, s, _ = ctx.energy_min(plan, dev(vals), dev(st["T"]), R.RN_PCG_JACOBI, 6, R.RN_FP64)
    P = host(P)
    for b in range(3):
        ref, info = O.emin_pcg(A0.rowptr, A0.colind, vals[b], st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"],
                               1, st["T"], 6)
        assert CS.rel_max(P[b], ref) <= FP64_TOL
    plan.close()


def test_pcg_through_setup(R, ctx):
    c = CS.case("aniso40")
    A = c["A"]
    ref, _ = O.emin_pcg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"], 1, c["T"],
                        c["iters"])
    s = ctx.setup_native(dev_matrix(R, c), dev(c["B"]), dev(c["agg"]), dev(c["roots"]), c["theta"], c["degree"],
                         c["iters"], R.RN_PCG_JACOBI, R.RN_FP64)
    assert CS.rel_max(host(s.tensor("P")), ref) <= FP64_TOL
    s.close()


CGNR_CASES = ["upwind64", "asym20", "aniso40", "elastic7", "elastic32", "poisson37", "upwind1024"]


@pytest.mark.parametrize("name", CGNR_CASES)
def test_cgnr(R, ctx, name):
    c = CS.case(name)
    A = c["A"]
    K = c["iters"]
    ref, info = O.emin_cgnr(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                            c["B"].shape[1], c["T"], K)
    assert info["status"] == 0
    g = run_path(R, ctx, c)
    P, st, hist = ctx.energy_min(g["plan"], g["A"].vals, g["T"], R.RN_CGNR, K, R.RN_FP64, want_hist=True)
    err = CS.rel_max(host(P), ref)
    print(f"{name}: CGNR {st.iters_done} steps, max|dP|/max|P| = {err:.2e}")
    assert st.iters_done == info["iters"]
    assert err <= tol(name)
    h = host(hist)[0]
    it = info["iters"]
    assert np.allclose(h[:it + 1], info["gamma"][:it + 1], rtol=1e-9, atol=0)
    g["plan"].close()


def test_variant_argument_errors(R, ctx):
    import torch
    c = CS.case("aniso40")
    g = run_path(R, ctx, c)
    for method, prec, batch in ((R.RN_PCG_JACOBI, R.RN_FP32_MIXED, 1), (R.RN_CGNR, R.RN_FP32_MIXED, 1),
                                (R.RN_CGNR, R.RN_FP64, 2)):
        with pytest.raises(R.RnError) as e:
            ctx.energy_min(g["plan"], g["A"].vals.repeat(batch) if batch > 1 else g["A"].vals, g["T"], method, 3,
                           prec, batch=batch)
        assert e.value.status == R._lib.RN_EINVAL
    # a diagonal entry that is not positive: the Jacobi preconditioner refuses
    vals = g["A"].vals.clone()
    Ap = c["A"].rowptr
    rows = np.repeat(np.arange(c["A"].n_rows), np.diff(Ap))
    k = int(np.flatnonzero((rows == 5) & (c["A"].colind == 5))[0])
    vals[k] = -1.0
    with pytest.raises(R.RnError) as e:
        ctx.energy_min(g["plan"], vals, g["T"], R.RN_PCG_JACOBI, 3, R.RN_FP64)
    assert e.value.status == R._lib.RN_ESINGULAR
    g["plan"].close()
