"""The batched differentiable form at full size: 16 rotated anisotropic
problems on 256 x 256 grids (eps = 10^U(-3,0), angle U(0,pi), seed 0), shared
structure, theta = 0, pattern S^2 C, 6 FP64 CG steps -- the launch
configuration the benchmark times (EnergyMinOperator: forward with the tape,
backward through the library).

Forward: every entry of P against the oracle's CG for each problem, 1e-12.
Backward: <J^T W, v> (GPU reverse mode) against <W, J v> (the oracle's
tangent-linear model) along random directions v, for every problem.
"""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import cases as CS

pytestmark = pytest.mark.gpu

NX, BATCH, K = 256, 16, 6
FP64_TOL = 1e-12
JVP_TOL = 1e-9


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


@pytest.fixture(scope="module")
def ctx(R):
    import torch
    assert torch.cuda.is_available()
    return R.Context()


def dev(x, dtype=None):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda", dtype=dtype)


@functools.lru_cache(maxsize=None)
def full_batch():
    A0, vals, params, rng = W.aniso_batch(NX, BATCH, 0)
    st = O.setup(A0, W.ones(A0.n_rows), 1, 0.0, 2)
    Wt = W.loss_weights(rng, BATCH, st["Nj"].size)
    refs = []
    for b in range(BATCH):
        P, info = O.emin_cg(A0.rowptr, A0.colind, vals[b], st["Np"], st["Nj"], st["is_root"], st["nc"],
                            st["Bc"], 1, st["T"], K)
        assert info["status"] == 0
        refs.append(P)
    return A0, vals, st, Wt, np.stack(refs)


@pytest.fixture(scope="module")
def op(R, ctx):
    A0, vals, st, Wt, refs = full_batch()
    # the structure through the GPU path (strength, pattern, tentative) on the
    # oracle's aggregation, as the benchmark builds it
    A = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    Sp, Sj = ctx.strength(A, 0.0)
    agg, roots = dev(st["agg"]), dev(st["roots"])
    Np, Nj, is_root = ctx.pattern(Sp, Sj, agg, roots, 2, 1)
    assert np.array_equal(Nj.cpu().numpy(), st["Nj"])
    import torch
    T, Bc, _ = ctx.tentative(Np, Nj, is_root, agg, roots, 1,
                             torch.ones((A0.n_rows, 1), dtype=torch.float64, device="cuda"))
    o = R.EnergyMinOperator(ctx, A, int(roots.numel()), Np, Nj, is_root, T, Bc, K)
    yield o
    o.close()


def test_batched_forward_full_size(R, ctx, op):
    import torch
    A0, vals, st, Wt, refs = full_batch()
    a = dev(vals)
    with torch.no_grad():
        P = op(a).cpu().numpy()
    Pt = op(a.clone().requires_grad_(True)).detach().cpu().numpy()  # the taped forward
    errs = [CS.rel_max(P[b], refs[b]) for b in range(BATCH)]
    print(f"batched 16 x {NX}^2 forward: worst max|dP|/max|P| = {max(errs):.3e}")
    assert max(errs) <= FP64_TOL, errs
    assert np.array_equal(P, Pt)
    # the constraint holds per problem (B = 1: every F row of P sums to one)
    for b in (0, BATCH - 1):
        assert O.constraint_residual(st["Np"], st["Nj"], P[b], st["Bc"], W.ones(A0.n_rows)) < 1e-12


def test_batched_adjoint_full_size(R, ctx, op):
    import torch
    A0, vals, st, Wt, refs = full_batch()
    a = dev(vals).requires_grad_(True)
    P = op(a)
    (g,) = torch.autograd.grad((P * dev(Wt)).sum(), a)
    g = g.cpu().numpy()
    rng = np.random.default_rng(5)
    for b in range(BATCH):
        v = rng.standard_normal(A0.nnz)
        _, dP = O.emin_cg_jvp(A0.rowptr, A0.colind, vals[b], v, st["Np"], st["Nj"], st["is_root"], st["nc"],
                              st["Bc"], 1, st["T"], K)
        lhs, rhs = float(g[b] @ v), float(Wt[b] @ dP)
        assert abs(lhs - rhs) <= JVP_TOL * (abs(rhs) + np.linalg.norm(g[b]) * np.linalg.norm(v) * 1e-3), \
            (b, lhs, rhs)
