"""The allocation-free energy minimisation (rn_energy_min_noalloc) against
rn_energy_min on the same plan, through the C ABI.

Two calls in a row on one GPU, the second on a smaller problem: each result
must equal rn_energy_min's (same kernels, same order: bit-identical, so the
FP64 bar 1e-12 holds trivially) and the oracle's to the usual bars, and no
device memory may be requested through the context's allocator during the
calls.  A call that needs more than the scratch array is refused before any
launch.
"""
import gc

import numpy as np
import pytest

from tests import cases as CS
from tests.test_gpu_parity import dev, host, run_path

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


def _counting_ctx(R):
    counts = {"alloc": 0}

    def on_alloc(n):
        counts["alloc"] += 1

    ctx = R.Context()
    ctx.use_torch_allocator(on_alloc)
    return ctx, counts


def _check(R, ctx, counts, name, method, precision):
    import torch
    c = CS.case(name)
    g = run_path(R, ctx, c)
    K = c["iters"]
    nz = g["Nj"].numel()
    ref, st_ref, hist_ref = ctx.energy_min(g["plan"], g["A"].vals, g["T"], method, K, precision, want_hist=True)
    torch.cuda.synchronize()
    P = torch.full((nz,), np.nan, dtype=torch.float64, device="cuda")
    hist = torch.full((1, 3 * K + 1), np.nan, dtype=torch.float64, device="cuda")
    # (tensors held in reference cycles by earlier tests are freed by the
    # collector whenever it runs: collect first and keep it off meanwhile, so
    # the count below sees the call alone)
    gc.collect()
    gc.disable()
    try:
        before = counts["alloc"]
        mem0 = torch.cuda.memory_allocated()
        st = ctx.energy_min_noalloc(g["plan"], g["A"].vals, g["T"], P, method, K, precision, hist=hist)
        torch.cuda.synchronize()
        mem1 = torch.cuda.memory_allocated()
    finally:
        gc.enable()
    assert counts["alloc"] == before, "the allocation-free call requested device memory"
    assert mem1 == mem0
    Pn, Pr = host(P), host(ref)
    d = CS.rel_max(Pn, Pr)
    print(f"{name} {'gmres' if method else 'cg'} {'mixed' if precision else 'fp64'}: "
          f"no-alloc vs rn_energy_min {d:.3e}, vs oracle {CS.rel_max(Pn, c['P']):.3e}")
    assert d <= FP64_TOL
    assert np.array_equal(host(hist), host(hist_ref))
    assert st.iters_done == st_ref.iters_done and st.status_code == 0
    tol = MIXED_TOL if precision else (CS.ELASTIC_FP64_TOL if name.startswith("elastic") else FP64_TOL)
    assert CS.rel_max(Pn, c["P"]) <= tol
    g["plan"].close()


def test_two_calls_second_smaller(R):
    ctx, counts = _counting_ctx(R)
    _check(R, ctx, counts, "aniso512", R.RN_CG, R.RN_FP64)
    _check(R, ctx, counts, "aniso40", R.RN_CG, R.RN_FP64)
    ctx.close()


def test_two_calls_gmres_and_mixed(R):
    ctx, counts = _counting_ctx(R)
    _check(R, ctx, counts, "aniso512", R.RN_CG, R.RN_FP32_MIXED)
    _check(R, ctx, counts, "upwind64", R.RN_GMRES, R.RN_FP64)
    _check(R, ctx, counts, "elastic7", R.RN_CG, R.RN_FP64)
    ctx.close()


def test_beyond_the_scratch_is_refused(R):
    """A batch whose Krylov vectors exceed the scratch array: RN_ELIMIT, and
    the output is left untouched (nothing was launched)."""
    import torch
    import workloads as W
    ctx = R.Context()
    A0, vals, _, _ = W.aniso_batch(256, 10, 0)
    A = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    Sp, Sj = ctx.strength(A, 0.0)
    agg, roots = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = dev(agg), dev(roots)
    Np, Nj, is_root = ctx.pattern(Sp, Sj, agg, roots, 2, 1)
    T, Bc, _ = ctx.tentative(Np, Nj, is_root, agg, roots, 1,
                             torch.ones((A0.n_rows, 1), dtype=torch.float64, device="cuda"))
    plan = ctx.plan(A, int(roots.numel()), Np, Nj, is_root, Bc)
    a = dev(vals)
    nz = Nj.numel()
    assert 10 * 3 * 8 * nz > R._lib.NOALLOC_SCRATCH_BYTES
    P = torch.full((10, nz), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(R.RnError) as e:
        ctx.energy_min_noalloc(plan, a, T, P, R.RN_CG, 6, R.RN_FP64, batch=10)
    assert e.value.status == R._lib.RN_ELIMIT
    torch.cuda.synchronize()
    assert bool((P == 7.0).all())
    # a batch that fits runs and matches the allocating call
    P2 = torch.empty((2, nz), dtype=torch.float64, device="cuda")
    ctx.energy_min_noalloc(plan, a[:2].contiguous(), T, P2, R.RN_CG, 6, R.RN_FP64, batch=2)
    ref, _, _ = ctx.energy_min(plan, a[:2].contiguous(), T, R.RN_CG, 6, R.RN_FP64)
    assert CS.rel_max(host(P2), host(ref)) <= FP64_TOL
    plan.close()
    ctx.close()
