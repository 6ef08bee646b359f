"""Benchmark: energy-minimisation setup of the root-node interpolation on one GPU.

Workload (one "step" = the whole hot path over one operator, inputs resident
in HBM before timing): rotated anisotropic diffusion, Q1 FEM, eps = 1e-3,
angle pi/8, 512 x 512 interior nodes (n = 262144, nnz(A) = 2353156), B = ones,
symmetric strength theta = 0.1, pattern S^2 C, 6 CG iterations, FP64:

    strength (two-phase) -> pattern (two-phase) -> tentative T, Bc
    -> plan (positions + Gram data) -> 6 CG energy-minimisation steps

The aggregation is an input (computed once on the host before timing).
Printed: ONE JSON line.  value = seconds per step (lower is better).
Extra fields: the same step with the FP32-mixed energy minimisation (error
and constraint residual against the FP64 oracle), the masked-product
kernel's HBM roofline, cold (a 512 MiB buffer read before every launch, so
nothing of the operands survives in the 256 MB last-level cache, which then
holds clean lines) and warm (launches back to back), on this workload and on
the 1024^2 upwind, 512^2 elasticity and 16 x 256^2 batched workloads, the
multilevel set-up of the headline workload (level sizes, operator
complexity), the
headline product also after a 512 MiB buffer is rewritten (the cache then
holds dirty lines the launch has to write back), a plain device copy moving
the product's traffic under the same conditions (what streaming reaches on
this GPU), the batched forward+backward, the other two configurations'
setups, and the CPU oracle on the same step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "energy-min setup s & masked-SpGEMM HBM GB/s; FP32-mix vs FP64; fwd+bwd time"
# HBM bytes per launch of the FP64 product on this workload from the counter
# runs in profiles/k_spgemm_q1aniso512_traffic.md (FETCH_SIZE and WRITE_SIZE
# of cold launches, scaled by the same counters on a copy of known size),
# valid for the kernel sources they were taken on (sha256 prefix below);
# otherwise reported as null.
TRAFFIC_BYTES = 59250064
TRAFFIC_SRC_SHA = "27f6cf77411c89de"
# the other workloads' products (same counters, same calibration, same sources)
TRAFFIC_OTHER = {"upwind1024": 181772974, "elastic512": 223696909, "aniso_batch256x16": 159643539}
TRAFFIC_SRCS = ("paper_1610_03154_amd/csrc/rn_spgemm.hip", "paper_1610_03154_amd/csrc/rn_plan.hip",
                "paper_1610_03154_amd/csrc/rn_emin.h")
HBM_PEAK_GBS = 8000.0
FLUSH_BYTES = 512 << 20
# untimed (flush, launch) pairs before a cold loop: the first loop after a
# pause runs about 10 % slower than the ones after it
COLD_WARMUP = 20
NX, EPS, PSI, THETA, DEGREE, ITERS = 512, 1e-3, np.pi / 8, 0.1, 2, 6


def product_bytes(nnz_a, n_rows, nnz_n, n, m=1, nB=1, n_f=0, batch=1, val=8):
    """Algorithmic bytes of one masked-product launch: A's column indices and
    values, A's and N's row pointers, N's column indices, X read once, Z
    written once (FP64), and the stored Gram data when n_B > m; A's and N's
    structure read once for a batch sharing it.  Returns (bytes, auxiliary
    bytes the implementation also reads: root flags, Bc, and the Gram data
    when n_B <= m)."""
    shared = 4 * nnz_a + 4 * (n_rows + 1) + 4 * nnz_n + 4 * (n + 1)
    per = val * m * m * nnz_a + val * nnz_n + 8 * nnz_n
    gram = 8 * n_f * nB * (nB + 1) // 2
    alg = shared + batch * per + (gram if nB > m else 0)
    aux = n + 8 * (n - n_f) * nB + (gram if nB <= m else 0)
    return float(alg), float(aux)


def build_inputs():
    import workloads as W
    import paper_1610_03154_amd as R
    import torch
    A = W.q1_aniso(NX, EPS, PSI)
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    ctx = R.Context()
    Sp, Sj = ctx.strength(dA, THETA)
    agg, roots = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    B = torch.ones((A.n_rows, 1), dtype=torch.float64, device="cuda")
    return dict(A=A, dA=dA, ctx=ctx, agg=torch.as_tensor(agg, device="cuda"),
                roots=torch.as_tensor(roots, device="cuda"), B=B, agg_host=agg, roots_host=roots)


def gpu_step(inp, precision):
    """One pass of the hot path through the stage calls; returns (P, stats, plan, aux)."""
    import paper_1610_03154_amd as R
    ctx, dA = inp["ctx"], inp["dA"]
    Sp, Sj = ctx.strength(dA, THETA)
    Np, Nj, is_root = ctx.pattern(Sp, Sj, inp["agg"], inp["roots"], DEGREE, 1)
    T, Bc, _ = ctx.tentative(Np, Nj, is_root, inp["agg"], inp["roots"], 1, inp["B"])
    plan = ctx.plan(dA, int(inp["roots"].numel()), Np, Nj, is_root, Bc)
    P, stats, _ = ctx.energy_min(plan, dA.vals, T, R.RN_CG, ITERS, precision)
    return P, stats, plan, (Np, Nj, is_root, T, Bc)


def native_step(inp, precision):
    """One pass of the hot path as one library call (rn_setup: strength ->
    pattern -> T -> plan -> 6 CG steps, the stages back to back inside the
    library); the results stay in the returned handle."""
    import paper_1610_03154_amd as R
    return inp["ctx"].setup_native(inp["dA"], inp["B"], inp["agg"], inp["roots"], THETA, DEGREE, ITERS, R.RN_CG,
                                   precision)


def time_steps(inp, precision, steps, warmup):
    """Seconds per step of the one-call set-up (HIP events and host wall
    clock); the staged calls run once first, their arrays feed the product
    timings."""
    import torch
    P, st, plan, aux = gpu_step(inp, precision)
    plan.close()
    for _ in range(warmup):
        native_step(inp, precision).close()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    s = None
    for _ in range(steps):
        if s is not None:
            s.close()
        s = native_step(inp, precision)
    ev1.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / steps
    P, st = s.tensor("P").clone(), s.stats
    torch.cuda.synchronize()
    s.close()
    return wall, ev0.elapsed_time(ev1) / 1e3 / steps, P, st, aux


class Flush:
    """A 512 MiB device buffer (twice the last-level cache) read before a
    cold launch, on the library's stream (torch's current one): the
    operands are evicted and the caches hold clean lines."""

    def __init__(self):
        import torch
        self.buf = torch.ones(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")

    def __call__(self):
        self.buf.sum()


class WriteFlush:
    """The same buffer rewritten instead: the caches then hold dirty lines,
    which the next launch's misses write back to HBM."""

    def __init__(self):
        import torch
        self.buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda")
        self.k = 0

    def __call__(self):
        self.k += 1
        self.buf.fill_(float(self.k))


def copy_calibration(nbytes, reps, flush):
    """A device copy moving nbytes (half read, half written): seconds per
    launch cold (flush before each, as for the product) and warm."""
    import torch
    n = max(int(nbytes) // 16, 1)
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(COLD_WARMUP):
        flush()
        y.copy_(x)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(reps):
        flush()
        y.copy_(x)
    ev[1].record()
    for _ in range(reps):
        flush()
    ev[2].record()
    torch.cuda.synchronize()
    cold = (ev[0].elapsed_time(ev[1]) - ev[1].elapsed_time(ev[2])) / 1e3 / reps
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(4 * reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    return cold, e0.elapsed_time(e1) / 1e3 / (4 * reps), 16 * n


def time_product(ctx, plan, A_vals, X, precision, reps_warm, reps_cold, flush, batch=None):
    """(cold, warm) seconds per launch of rn_masked_product (project = 1).
    Cold: after COLD_WARMUP untimed pairs, reps_cold pairs (flush, launch)
    back to back between two HIP events,
    less reps_cold flushes alone between two events, per launch (a launch
    bracketed by its own pair of events would add the events' own latency to
    a kernel of tens of microseconds); warm: launches back to back between
    two events."""
    import torch
    flush()  # the first launch (allocating Z) is cold too
    Z = ctx.masked_product(plan, A_vals, X, True, precision)
    torch.cuda.synchronize()
    cold = None
    if reps_cold > 0:
        for _ in range(COLD_WARMUP):  # untimed (flush, launch) pairs, as for the copy
            flush()
            ctx.masked_product(plan, A_vals, X, True, precision, out=Z)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        for _ in range(reps_cold):
            flush()
            ctx.masked_product(plan, A_vals, X, True, precision, out=Z)
        ev[1].record()
        ev[2].record()
        for _ in range(reps_cold):
            flush()
        ev[3].record()
        torch.cuda.synchronize()
        cold = (ev[0].elapsed_time(ev[1]) - ev[2].elapsed_time(ev[3])) / 1e3 / reps_cold
    warm = None
    if reps_warm > 0:
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        # the launches queue faster than they run: the events bracket
        # back-to-back kernels (no allocation inside the loop)
        ev0.record()
        for _ in range(reps_warm):
            ctx.masked_product(plan, A_vals, X, True, precision, out=Z)
        ev1.record()
        torch.cuda.synchronize()
        warm = ev0.elapsed_time(ev1) / 1e3 / reps_warm
    return cold, warm


def roof(kernel, workload, bytes_alg, aux, cold, warm, flops=None):
    d = {"kernel": kernel, "workload": workload, "bytes_per_launch": bytes_alg, "aux_bytes_per_launch": aux,
         "us_cold": None if cold is None else cold * 1e6, "us_warm": None if warm is None else warm * 1e6}
    if cold is not None:
        d["GBps_cold"] = bytes_alg / cold / 1e9
        d["frac_cold"] = d["GBps_cold"] / HBM_PEAK_GBS
    if warm is not None:
        d["GBps_warm"] = bytes_alg / warm / 1e9
        d["frac_warm"] = d["GBps_warm"] / HBM_PEAK_GBS
    if flops is not None:
        d["flops_per_launch"] = flops
    return d


def headline_roofline(inp, aux, reps_warm, reps_cold, flush, fp64_only=False):
    """The FP64 and FP32-mixed products on the 512^2 workload (fp64_only: the
    FP64 launches alone, nothing else launching that kernel)."""
    import torch
    import paper_1610_03154_amd as R
    ctx, dA = inp["ctx"], inp["dA"]
    Np, Nj, is_root, T, Bc = aux
    plan = ctx.plan(dA, int(inp["roots"].numel()), Np, Nj, is_root, Bc)
    X = torch.randn(Nj.numel(), dtype=torch.float64, device="cuda")
    n, nnz_n, nnz_a = dA.n, int(Nj.numel()), dA.nnz
    nc = int(inp["roots"].numel())
    out = {}
    c, w = time_product(ctx, plan, dA.vals, X, R.RN_FP64, reps_warm, reps_cold, flush)
    b, a = product_bytes(nnz_a, n, nnz_n, n, n_f=n - nc)
    out["fp64"] = roof("k_spgemm_p<NB=1,MODE_PRODUCT,fp64,256 lanes> (persistent)", "q1_aniso512", b, a, c, w)
    _, st, _ = ctx.energy_min(plan, dA.vals, T, R.RN_CG, 1, R.RN_FP64)
    out["flops"] = st.spgemm_flops
    if fp64_only:
        plan.close()
        return out
    # FP32-mixed through the C ABI, which takes FP64 A and X and rounds them
    # inside the call (two conversion launches, then the product)
    c32, w32 = time_product(ctx, plan, dA.vals, X, R.RN_FP32_MIXED, reps_warm // 2, reps_cold // 2, flush)
    b32, a32 = product_bytes(nnz_a, n, nnz_n, n, n_f=n - nc, val=4)
    out["fp32_mixed_call"] = roof("rn_masked_product FP32-mixed (A, X rounded inside the call: two conversions + "
                                  "product)", "q1_aniso512", b32, a32, c32, w32)
    # the same product on four copies (values and X per copy, shared structure)
    A4 = dA.vals.repeat(4, 1)
    X4 = torch.randn((4, nnz_n), dtype=torch.float64, device="cuda")
    c4, w4 = time_product(ctx, plan, A4, X4, R.RN_FP64, max(reps_warm // 4, 10), 0, flush)
    b4, a4 = product_bytes(nnz_a, n, nnz_n, n, n_f=n - nc, batch=4)
    out["batch4"] = roof("k_spgemm_p, 4 problems per launch (shared structure counted once)", "4 x q1_aniso512", b4,
                         a4, c4, w4)
    plan.close()
    return out


OTHER_WORKLOADS = ("upwind1024", "elastic512", "aniso_batch256x16")


def other_rooflines(reps_warm, reps_cold, flush, only=None):
    """Cold and warm product launches on the study's other configurations
    (only: that workload alone)."""
    import torch
    import workloads as W
    import paper_1610_03154_amd as R
    ctx = R.Context()
    res = []
    if only in (None, "upwind1024"):
        A = W.upwind_cd(1024)
        dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
        plan, Nj, na = _struct(ctx, dA, torch.ones((A.n_rows, 1), dtype=torch.float64, device="cuda"), 1, 0.0)
        X = torch.randn(Nj.numel(), dtype=torch.float64, device="cuda")
        c, w = time_product(ctx, plan, dA.vals, X, R.RN_FP64, reps_warm, reps_cold, flush)
        b, a = product_bytes(dA.nnz, dA.n, int(Nj.numel()), dA.n, n_f=dA.n - na)
        res.append(roof("k_spgemm_p<NB=1,MODE_PRODUCT,fp64,256 lanes> (the product of each GMRES step)",
                        "upwind1024", b, a, c, w))
        plan.close()
    if only in (None, "elastic512"):
        res += elastic_roofline(ctx, reps_warm, reps_cold, flush)
    if only in (None, "aniso_batch256x16"):
        res += batch_roofline(ctx, reps_warm, reps_cold, flush)
    ctx.close()
    for r in res:
        r["traffic"] = traffic_bytes(r["workload"])
    return res


def _struct(ctx, dA, B, m, theta):
    """Strength, aggregation, pattern, tentative T and the product plan."""
    import torch
    import paper_1610_03154_amd as R
    Sp, Sj = ctx.strength(dA, theta)
    a, r = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(a, device="cuda"), torch.as_tensor(r, device="cuda")
    Np, Nj, is_root = ctx.pattern(Sp, Sj, agg, roots, 2, m)
    T, Bc, _ = ctx.tentative(Np, Nj, is_root, agg, roots, m, B)
    plan = ctx.plan(dA, m * int(roots.numel()), Np, Nj, is_root, Bc)
    return plan, Nj, int(roots.numel())


def elastic_roofline(ctx, reps_warm, reps_cold, flush):
    import torch
    import workloads as W
    import paper_1610_03154_amd as R
    Ab, xy = W.q1_elasticity(512)
    dA = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=Ab.n_nodes * 2, block_m=2)
    plan, Nj, na = _struct(ctx, dA, torch.as_tensor(W.rbm(xy), device="cuda"), 2, 0.0)
    X = torch.randn(Nj.numel(), dtype=torch.float64, device="cuda")
    c, w = time_product(ctx, plan, dA.vals, X, R.RN_FP64, reps_warm, reps_cold, flush)
    n = dA.n
    b, a = product_bytes(dA.nnz, Ab.n_nodes, int(Nj.numel()), n, m=2, nB=3, n_f=n - 2 * na)
    plan.close()
    return [roof("k_spgemm<M=2,NB=3,MODE_PRODUCT,fp64,256> (node-blocked)", "elastic512", b, a, c, w)]


def batch_roofline(ctx, reps_warm, reps_cold, flush):
    import torch
    import workloads as W
    import paper_1610_03154_amd as R
    A0, vals, _, _ = W.aniso_batch(256, 16, 0)
    dA = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    plan, Nj, na = _struct(ctx, dA, torch.ones((A0.n_rows, 1), dtype=torch.float64, device="cuda"), 1, 0.0)
    av = torch.as_tensor(vals, device="cuda")
    X = torch.randn((16, Nj.numel()), dtype=torch.float64, device="cuda")
    c, w = time_product(ctx, plan, av, X, R.RN_FP64, max(reps_warm // 4, 10) if reps_warm else 0, reps_cold, flush)
    b, a = product_bytes(dA.nnz, dA.n, int(Nj.numel()), dA.n, n_f=dA.n - na, batch=16)
    plan.close()
    return [roof("k_spgemm_p, 16 problems per launch (shared structure counted once)", "aniso_batch256x16", b, a,
                 c, w)]


def fwd_bwd(reps):
    """Batched differentiable form: 16 rotated anisotropic problems on 256 x 256
    grids (eps = 10^U(-3,0), angle U(0,pi), seed 0; shared structure, theta = 0,
    pattern S^2 C), loss <W, P> with W ~ N(0,1); one forward (6 CG steps with
    the tape) plus one backward per repetition, structure set up beforehand."""
    import torch
    import workloads as W
    import paper_1610_03154_amd as R
    A0, vals, params, rng = W.aniso_batch(256, 16, 0)
    ctx = R.Context()
    A = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    Sp, Sj = ctx.strength(A, 0.0)
    agg, roots = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(agg, device="cuda"), torch.as_tensor(roots, device="cuda")
    Np, Nj, is_root = ctx.pattern(Sp, Sj, agg, roots, 2, 1)
    B = torch.ones((A0.n_rows, 1), dtype=torch.float64, device="cuda")
    T, Bc, _ = ctx.tentative(Np, Nj, is_root, agg, roots, 1, B)
    op = R.EnergyMinOperator(ctx, A, int(roots.numel()), Np, Nj, is_root, T, Bc, ITERS)
    Wt = torch.as_tensor(W.loss_weights(rng, 16, Nj.numel()), device="cuda")
    a = torch.as_tensor(vals, device="cuda")

    def one(backward):
        x = a.detach().requires_grad_(backward)
        P = op(x)
        if backward:
            (g,) = torch.autograd.grad((P * Wt).sum(), x)
            return g
        return P

    one(True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        one(True)
    ev[1].record()
    with torch.no_grad():
        ev[2].record()
        for _ in range(reps):
            one(False)
        ev[3].record()
    torch.cuda.synchronize()
    t_fb = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    t_f = ev[2].elapsed_time(ev[3]) / 1e3 / reps
    op.close()
    ctx.close()
    return t_fb, t_f, int(Nj.numel())


def traffic_bytes(workload="q1aniso512"):
    """HBM bytes per launch from the FETCH_SIZE and WRITE_SIZE counters, or
    None once the product's sources differ from those the counters were
    taken on."""
    import hashlib
    tb = TRAFFIC_BYTES if workload == "q1aniso512" else TRAFFIC_OTHER.get(workload)
    if tb is None:
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SRCS:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return tb if h.hexdigest()[:16] == TRAFFIC_SRC_SHA else None


def other_configs(reps, check_oracle):
    """The study's other two configurations at full size on the same GPU path,
    aggregation precomputed on the host (an input), seconds per one-call
    set-up (rn_setup: strength -> pattern -> T -> plan -> energy
    minimisation), FP64 and
    FP32-mixed, and the FP32-mixed results against the FP64 oracle:
    upwind1024: first-order upwind convection-diffusion on 1024 x 1024
      (b at 3pi/16, eps 1e-4), B = B^ = ones, theta 0, S^2 C, P by 8 GMRES
      steps on A and R^T by 8 GMRES steps on A^T (transpose included);
    elastic512: Q1 plane-strain elasticity on 512 x 512 nodes, 2 DOFs per node
      (node-blocked CSR), B = 3 rigid-body modes, theta 0, S^2 C, 6 CG steps."""
    import torch
    import workloads as W
    import paper_1610_03154_amd as R
    ctx = R.Context()
    out = {}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            res = fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / 1e3 / reps, res

    A = W.upwind_cd(1024)
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    Sp, Sj = ctx.strength(dA, 0.0)
    a, r = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(a, device="cuda"), torch.as_tensor(r, device="cuda")
    B = torch.ones((A.n_rows, 1), dtype=torch.float64, device="cuda")
    res = {}
    def host(s, name):
        return s.tensor(name).cpu().numpy()

    for prec, key in ((R.RN_FP64, "fp64"), (R.RN_FP32_MIXED, "fp32_mixed")):
        t, s = timed(lambda: ctx.setup_native(dA, B, agg, roots, 0.0, 2, 8, R.RN_GMRES, prec, Bhat=B))
        out["upwind1024_gmres_P_RT_s_" + key] = t
        res[key] = (host(s, "P"), host(s, "RT"), host(s, "N_rowptr"), host(s, "N_colind"), host(s, "Bc"))
        s.close()
    if check_oracle:
        out.update(mixed_vs_oracle_upwind(A, a, r, res))
    Ab, xy = W.q1_elasticity(512)
    dA = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=Ab.n_nodes * 2, block_m=2)
    Sp, Sj = ctx.strength(dA, 0.0)
    a, r = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(a, device="cuda"), torch.as_tensor(r, device="cuda")
    Bh = W.rbm(xy)
    B = torch.as_tensor(Bh, device="cuda")
    res = {}
    for prec, key in ((R.RN_FP64, "fp64"), (R.RN_FP32_MIXED, "fp32_mixed")):
        t, s = timed(lambda: ctx.setup_native(dA, B, agg, roots, 0.0, 2, 6, R.RN_CG, prec))
        out["elastic512_cg_s_" + key] = t
        res[key] = (host(s, "P"), host(s, "N_rowptr"), host(s, "N_colind"), host(s, "Bc"))
        s.close()
    if check_oracle:
        out.update(mixed_vs_oracle_elastic(Ab, Bh, a, r, res))
    ctx.close()
    return out


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def hierarchy_run(inp):
    """The multilevel set-up of the headline workload (rn_hierarchy_build:
    the same theta, pattern degree and CG steps on every level, levels down
    to 500 rows): level sizes, stored entries, operator complexity (Sec.
    2.4) and seconds per build (host aggregation of every level included)."""
    import torch
    import paper_1610_03154_amd as R
    ctx = inp["ctx"]
    B = torch.ones((inp["dA"].n, 1), dtype=torch.float64, device="cuda")

    def build():
        return ctx.hierarchy(inp["dA"], B, max_levels=10, min_coarse=500, theta=THETA, degree=DEGREE, iters=ITERS,
                             method=R.RN_CG, precision=R.RN_FP64)
    build().close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = build()
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    views = [h.view(l) for l in range(h.n_levels)]
    out = {"levels_n": [v.n for v in views], "levels_nnz": [int(v.nnz_A) for v in views],
           "operator_complexity": h.operator_complexity(), "s": t,
           "workload": "q1_aniso512 hierarchy, theta 0.1, S^2 C, 6 CG steps per level, down to 500 rows"}
    h.close()
    return out


def mixed_vs_oracle_upwind(A, agg, roots, res):
    """P and R^T of both precisions against the FP64 oracle's GMRES, with the
    constraint residual of each (Eq. mode_constraint: P Bc = B, R^T Bc^ = B^)."""
    import oracle as O
    import workloads as W
    B = W.ones(A.n_rows)
    st = O.setup(A, B, 1, 0.0, 2, agg=agg, roots=roots)
    Pref, _ = O.emin_gmres(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1,
                           st["T"], 8)
    Tp, Tj, Tx = O.transpose(A.rowptr, A.colind, A.vals)
    RTref, _ = O.emin_gmres(Tp, Tj, Tx, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1, st["T"], 8)
    out = {}
    for key in ("fp64", "fp32_mixed"):
        P, RT, Np, Nj, Bc = res[key]
        assert np.array_equal(Nj, st["Nj"])
        out[f"upwind1024_{key}_max_rel_dP_vs_oracle"] = _rel(P, Pref)
        out[f"upwind1024_{key}_max_rel_dRT_vs_oracle"] = _rel(RT, RTref)
        out[f"upwind1024_{key}_constraint_residual"] = max(O.constraint_residual(Np, Nj, P, Bc, B),
                                                           O.constraint_residual(Np, Nj, RT, Bc, B))
    return out


def mixed_vs_oracle_elastic(Ab, Bh, agg, roots, res):
    import oracle as O
    A = Ab.to_csr()
    st = O.setup(A, Bh, 2, 0.0, 2, agg=agg, roots=roots)
    Pref, _ = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 3,
                        st["T"], 6)
    # rows whose Bc rows do not span the candidates (rank-deficient Gram)
    # cannot meet P Bc = B exactly: the oracle's own residual is the reference
    out = {"elastic512_oracle_constraint_residual": O.constraint_residual(st["Np"], st["Nj"], Pref,
                                                                          st["Bc"].reshape(-1, 3), Bh),
           "elastic512_rank_deficient_rows": int(st["rank_def"])}
    for key in ("fp64", "fp32_mixed"):
        P, Np, Nj, Bc = res[key]
        assert np.array_equal(Nj, st["Nj"])
        out[f"elastic512_{key}_max_rel_dP_vs_oracle"] = _rel(P, Pref)
        out[f"elastic512_{key}_constraint_residual"] = O.constraint_residual(Np, Nj, P, Bc.reshape(-1, 3), Bh)
    return out


def oracle_reference(inp):
    """The FP64 oracle's P on the headline workload (same aggregation)."""
    import oracle as O
    import workloads as W
    A = inp["A"]
    st = O.setup(A, W.ones(A.n_rows), 1, THETA, DEGREE, agg=inp["agg_host"], roots=inp["roots_host"])
    P, _ = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1, st["T"],
                     ITERS)
    return P, st


def cpu_threads():
    env = os.environ.get("OMP_NUM_THREADS")
    avail = len(os.sched_getaffinity(0))
    return min(int(env), avail) if env and env.isdigit() and int(env) > 0 else avail


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(budget_s=12.0):
    """The oracle on the same step (strength, aggregation given, pattern,
    tentative, 6 CG steps): median over repeated runs for about budget_s with
    all the host's available threads, then two runs with one thread."""
    import oracle as O
    import workloads as W
    A = W.q1_aniso(NX, EPS, PSI)
    B = W.ones(A.n_rows)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, THETA)
    agg, roots = O.aggregate(Sp, Sj)

    def one():
        t0 = time.perf_counter()
        st = O.setup(A, B, 1, THETA, DEGREE, agg=agg, roots=roots)
        O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1, st["T"],
                  ITERS)
        return time.perf_counter() - t0

    nt = cpu_threads()
    O.set_threads(nt)
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        times.append(one())
        if time.perf_counter() > t_end or len(times) >= 50:
            break
    O.set_threads(1)
    t1 = [one() for _ in range(2)]
    O.set_threads(nt)
    return float(np.median(times)), len(times), nt, float(np.median(t1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=200, help="back-to-back launches for the warm product timing")
    ap.add_argument("--cold-reps", type=int, default=50, help="launches, each after a cache flush, for the cold timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--fb-reps", type=int, default=5, help="repetitions of the batched forward+backward")
    ap.add_argument("--roofline-only", nargs="?", const="q1aniso512", default=None,
                    choices=("q1aniso512",) + OTHER_WORKLOADS,
                    help="only the cold launches of one workload's product (default the headline's: the "
                         "roofline's own loop)")
    ap.add_argument("--fwd-bwd-only", action="store_true",
                    help="only the batched forward+backward (for a kernel trace of the adjoint)")
    ap.add_argument("--steps-only", action="store_true",
                    help="only the timed FP64 set-up steps (for a kernel trace of the step)")
    ap.add_argument("--other-reps", type=int, default=3,
                    help="repetitions of the upwind1024 and elastic512 setups (0 skips them)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the energy-minimisation path here is single-GPU "
              "(no sharded path is built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1610_03154_amd as R
    torch.cuda.set_device(0)
    inp = build_inputs()
    flush = Flush()
    if args.fwd_bwd_only:
        t_fb, t_f, _ = fwd_bwd(args.fb_reps)
        print(json.dumps({"fwd_bwd_s": t_fb, "fwd_only_s": t_f, "reps": args.fb_reps}))
        return
    if args.roofline_only and args.roofline_only != "q1aniso512":
        print(json.dumps(other_rooflines(0, args.cold_reps, flush, only=args.roofline_only)))
        return
    if args.roofline_only:
        P, st, plan, aux = gpu_step(inp, R.RN_FP64)
        plan.close()
        r = headline_roofline(inp, aux, 0, args.cold_reps, flush, fp64_only=True)["fp64"]
        print(json.dumps(r))
        return
    wall64, ev64, P64, st64, aux = time_steps(inp, R.RN_FP64, args.steps, args.warmup)
    if args.steps_only:
        print(json.dumps({"value": ev64, "unit": "s", "wall_s_per_step": wall64, "steps": args.steps}))
        return
    wall32, ev32, P32, st32, _ = time_steps(inp, R.RN_FP32_MIXED, args.steps, args.warmup)
    head = headline_roofline(inp, aux, args.reps, args.cold_reps, flush)
    wcold = headline_roofline(inp, aux, 0, args.cold_reps, WriteFlush(), fp64_only=True)["fp64"]
    tb = traffic_bytes()
    cc, cw, cb = copy_calibration(tb if tb else TRAFFIC_BYTES, args.cold_reps, flush)
    others = other_rooflines(args.reps, args.cold_reps, flush)
    t_fb, t_f, nnz_n5 = fwd_bwd(args.fb_reps)
    configs = other_configs(args.other_reps, not args.no_cpu) if args.other_reps > 0 else {}
    hier = hierarchy_run(inp)
    r64 = head["fp64"]
    achieved = r64["GBps_cold"]
    p64, p32 = P64.cpu().numpy(), P32.cpu().numpy()
    out = {
        "metric": METRIC,
        "value": ev64,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ev64 * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "q1_aniso_eps1e-3_pi8_512x512_cg6_fp64", "n": int(inp["A"].n_rows),
                   "nnz_A": int(inp["A"].nnz), "nnz_N": int(aux[1].numel()), "iters": ITERS,
                   "degree": DEGREE, "theta": THETA},
        "wall_s_per_step": wall64,
        "fp32_mixed_s_per_step": ev32,
        "fp32_mixed_vs_fp64_time": ev32 / ev64,
        "spgemm_us_fp64_cold": r64["us_cold"],
        "spgemm_us_fp64_warm": r64["us_warm"],
        "spgemm_frac_fp64_warm": r64["frac_warm"],
        "spgemm_us_fp64_cold_after_write_flush": wcold["us_cold"],
        "spgemm_frac_fp64_cold_after_write_flush": wcold["frac_cold"],
        "copy_calibration": {"kernel": "device copy (torch copy_), the product's traffic moved", "bytes": cb,
                             "us_cold": cc * 1e6, "GBps_cold": cb / cc / 1e9, "us_warm": cw * 1e6,
                             "GBps_warm": cb / cw / 1e9},
        "spgemm_fp32_mixed_call": head["fp32_mixed_call"],
        "spgemm_batch4": head["batch4"],
        "rooflines_other": others,
        "fwd_bwd_s": t_fb,
        "fwd_bwd_workload": f"16 x q1_aniso 256x256 (eps 10^U(-3,0), angle U(0,pi), seed 0), theta 0, "
                            f"S^2 C (nnz_N {nnz_n5} each), 6 CG steps FP64, loss <W,P>",
        "fwd_only_s": t_f,
        **configs,
        "hierarchy": hier,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(),
                     "kernel": r64["kernel"], "timing": "cold: a 512 MiB buffer read before every launch; "
                                                       "(flush + launch) x 50 less flush x 50, HIP events",
                     "bytes_per_launch": r64["bytes_per_launch"], "aux_bytes_per_launch": r64["aux_bytes_per_launch"],
                     "flops_per_launch": head["flops"]},
    }
    if not args.no_cpu:
        import oracle as O
        Pref, st = oracle_reference(inp)
        out["fp64_max_rel_dP_vs_oracle"] = _rel(p64, Pref)
        out["fp32_mixed_max_rel_dP_vs_oracle"] = _rel(p32, Pref)
        Np, Nj = aux[0].cpu().numpy(), aux[1].cpu().numpy()
        Bc = aux[4].cpu().numpy()
        ones = np.ones((Np.size - 1, 1))
        out["fp64_constraint_residual"] = O.constraint_residual(Np, Nj, p64, Bc, ones)
        out["fp32_mixed_constraint_residual"] = O.constraint_residual(Np, Nj, p32, Bc, ones)
        med, cnt, nt, t1 = cpu_baseline()
        out["cpu_baseline"] = {"value": med, "unit": "s", "cores": nt, "kind": "oracle",
                               "value_1_thread": t1, "cpu_model": cpu_model(),
                               "sample": f"the full step (strength, pattern, tentative, 6 CG steps) on the 512x512 "
                                         f"workload, median of {cnt} runs with {nt} OpenMP threads (the oracle's "
                                         f"sums are chunked independently of the thread count); 1 thread: "
                                         f"median of 2 runs"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
