"""Fused CG steps (RN_OPT_FUSED_CG; Sec. 4.1 CG form), through the C ABI.

With the option on, each CG direction D_k = R_k + beta_{k-1} D_{k-1} is
formed while the next product stages its X window (two launches per step,
two D buffers); with it off a separate direction pass forms it.  The two
paths evaluate the same expressions in the same order, so P, the Krylov
history and the step count must agree bit for bit; the fused result is
also held to the FP64 bar against the oracle, including a run that stops
early inside a fused product, a one-step run and a batch.  In the
FP32-mixed form the fused step rounds each window element of D_k to FP32
where the separate pass writes D's FP32 shadow: the same bits again, and
the mixed bar against the FP64 oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS
from tests.test_gpu_parity import FP64_TOL, MIXED_TOL, dev, host, run_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


def _run(R, c, fused, K, prec=None):
    ctx = R.Context()
    ctx.set_option(R._lib.RN_OPT_FUSED_CG, 1 if fused else 0)
    g = run_path(R, ctx, c)
    prec = R.RN_FP64 if prec is None else prec
    P, st, hist = ctx.energy_min(g["plan"], g["A"].vals, g["T"], R.RN_CG, K, prec, want_hist=True)
    out = host(P), st, host(hist)
    g["plan"].close()
    ctx.close()
    return out


# (case, steps, whether the persistent product serves the plan)
RUNS = [("poisson32", 4, 1), ("aniso40", 5, 1), ("twocand13", 5, 0), ("aniso512", 6, 1),
        ("poisson37", 4, 1), ("elastic7", 3, 0), ("lap27_10", 3, 0),
        ("poisson32", 40, 1),   # converges after 31 steps: the stop is taken inside a fused product
        ("aniso40", 1, 1), ("aniso40", 2, 1)]


@pytest.mark.parametrize("name,K,fuses", RUNS)
def test_fused_equals_separate_and_oracle(R, name, K, fuses):
    c = CS.case(name)
    A = c["A"]
    Pf, sf, hf = _run(R, c, True, K)
    Ps, ss, hs = _run(R, c, False, K)
    assert sf.fused_cg == fuses and ss.fused_cg == 0
    assert sf.iters_done == ss.iters_done and sf.status_code == ss.status_code == 0
    assert np.array_equal(Pf, Ps), f"{name}: fused and separate P differ by {np.max(np.abs(Pf - Ps)):.3e}"
    assert np.array_equal(hf, hs)
    assert sf.last == ss.last and sf.first == ss.first
    ref, info = O.emin_cg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                          c["B"].shape[1], c["T"], K)
    assert sf.iters_done == info["iters"]
    err = CS.rel_max(Pf, ref)
    tol = CS.ELASTIC_FP64_TOL if name.startswith("elastic") else FP64_TOL
    print(f"{name} K={K}: {sf.iters_done} steps, fused={sf.fused_cg}, max|dP|/max|P| = {err:.2e}")
    assert err <= tol
    it = info["iters"]
    g0 = info["gamma"][0]
    np.testing.assert_allclose(hf[0][:it + 1], info["gamma"][:it + 1], rtol=1e-10, atol=1e-20 * g0)
    # (after convergence both sides hold round-off-level scalars)
    np.testing.assert_allclose(hf[0][1 + K:1 + K + it], info["delta"][:it], rtol=1e-10, atol=1e-20 * g0)


# 16 x 64^2: the persistent grid per problem is set by occupancy, not by the
# block count, so the step products must share one grid to agree bit for bit
@pytest.mark.parametrize("nx,batch", [(32, 3), (64, 16)])
def test_fused_batch(R, nx, batch):
    A0, vals, _, _ = W.aniso_batch(nx, batch, 0)
    st = O.setup(A0, W.ones(A0.n_rows), 1, 0.0, 2)
    outs = []
    for fused in (1, 0):
        ctx = R.Context()
        ctx.set_option(R._lib.RN_OPT_FUSED_CG, fused)
        dA = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
        plan = ctx.plan(dA, st["nc"], dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"]), dev(st["Bc"]))
        P, s, hist = ctx.energy_min(plan, dev(vals), dev(st["T"]), R.RN_CG, 6, R.RN_FP64, want_hist=True)
        outs.append((host(P), s, host(hist)))
        plan.close()
        ctx.close()
    (Pf, sf, hf), (Ps, ss, hs) = outs
    assert sf.fused_cg == 1 and ss.fused_cg == 0
    assert np.array_equal(Pf, Ps) and np.array_equal(hf, hs)
    for b in range(batch):
        ref, _ = O.emin_cg(A0.rowptr, A0.colind, vals[b], st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"],
                           1, st["T"], 6)
        assert CS.rel_max(Pf[b], ref) <= FP64_TOL


# FP32-mixed: (case, steps, whether the persistent product serves the plan)
MIXED_RUNS = [("poisson32", 4, 1), ("aniso40", 5, 1), ("aniso512", 6, 1), ("poisson37", 4, 1), ("twocand13", 5, 0),
              ("poisson32", 40, 1), ("aniso40", 1, 1)]


@pytest.mark.parametrize("name,K,fuses", MIXED_RUNS)
def test_fused_mixed_equals_separate_and_oracle(R, name, K, fuses):
    c = CS.case(name)
    A = c["A"]
    Pf, sf, hf = _run(R, c, True, K, R.RN_FP32_MIXED)
    Ps, ss, hs = _run(R, c, False, K, R.RN_FP32_MIXED)
    assert sf.fused_cg == fuses and ss.fused_cg == 0
    assert sf.iters_done == ss.iters_done and sf.status_code == ss.status_code == 0
    assert np.array_equal(Pf, Ps), f"{name}: fused and separate P differ by {np.max(np.abs(Pf - Ps)):.3e}"
    assert np.array_equal(hf, hs)
    if K > 6:  # (past the FP64 run's convergence the mixed iterates are FP32 noise: bit equality only)
        return
    ref, info = O.emin_cg(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["nc"], c["Bc"],
                          c["B"].shape[1], c["T"], K)
    err = CS.rel_max(Pf, ref)
    print(f"{name} K={K} mixed: {sf.iters_done} steps, fused={sf.fused_cg}, max|dP|/max|P| = {err:.2e}")
    assert err <= MIXED_TOL


def test_fused_mixed_batch(R):
    A0, vals, _, _ = W.aniso_batch(32, 3, 0)
    st = O.setup(A0, W.ones(A0.n_rows), 1, 0.0, 2)
    outs = []
    for fused in (1, 0):
        ctx = R.Context()
        ctx.set_option(R._lib.RN_OPT_FUSED_CG, fused)
        dA = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
        plan = ctx.plan(dA, st["nc"], dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"]), dev(st["Bc"]))
        P, s, hist = ctx.energy_min(plan, dev(vals), dev(st["T"]), R.RN_CG, 6, R.RN_FP32_MIXED, want_hist=True)
        outs.append((host(P), s, host(hist)))
        plan.close()
        ctx.close()
    (Pf, sf, hf), (Ps, ss, hs) = outs
    assert sf.fused_cg == 1 and ss.fused_cg == 0
    assert np.array_equal(Pf, Ps) and np.array_equal(hf, hs)
    for b in range(3):
        ref, _ = O.emin_cg(A0.rowptr, A0.colind, vals[b], st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"],
                           1, st["T"], 6)
        assert CS.rel_max(Pf[b], ref) <= MIXED_TOL


def test_option_values(R):
    ctx = R.Context()
    with pytest.raises(R.RnError):
        ctx.set_option(R._lib.RN_OPT_FUSED_CG, 2)
    ctx.close()
