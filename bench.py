"""Benchmark: energy-minimisation setup of the root-node interpolation on one GPU.

Workload (one "step" = the whole hot path over one operator, inputs resident
in HBM before timing): rotated anisotropic diffusion, Q1 FEM, eps = 1e-3,
angle pi/8, 512 x 512 interior nodes (n = 262144, nnz(A) = 2353156), B = ones,
symmetric strength theta = 0.1, pattern S^2 C, 6 CG iterations, FP64:

    strength (two-phase) -> pattern (two-phase) -> tentative T, Bc
    -> plan (positions + Gram data) -> 6 CG energy-minimisation steps

The aggregation is an input (computed once on the host before timing).
Printed: ONE JSON line.  value = seconds per step (lower is better).
Extra fields: the same step with the FP32-mixed energy minimisation, the
masked-product kernel's HBM roofline, and the CPU oracle on the same step.
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
# runs in profiles/k_spgemm_q1aniso512_traffic.md (FETCH_SIZE and WRITE_SIZE,
# scaled by the same counters on a copy of known size), valid for the kernel
# sources they were taken on (sha256 prefix below); otherwise reported as null.
TRAFFIC_BYTES = 59249868
TRAFFIC_SRC_SHA = "402451266b617fc8"
TRAFFIC_SRCS = ("paper_1610_03154_amd/csrc/rn_spgemm.hip", "paper_1610_03154_amd/csrc/rn_plan.hip",
                "paper_1610_03154_amd/csrc/rn_emin.h")
HBM_PEAK_GBS = 8000.0
NX, EPS, PSI, THETA, DEGREE, ITERS = 512, 1e-3, np.pi / 8, 0.1, 2, 6


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
    """One pass of the hot path; returns (P, stats, plan)."""
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
    P, st = s.tensor("P"), s.stats
    torch.cuda.synchronize()
    s.close()
    return wall, ev0.elapsed_time(ev1) / 1e3 / steps, P, st, aux


def roofline(inp, aux, precision, reps):
    """Average duration of the masked-product kernel (Z = Pi(M(A X))) timed
    with HIP events on the library's stream, back to back (warm caches)."""
    import torch
    import paper_1610_03154_amd as R
    ctx, dA = inp["ctx"], inp["dA"]
    Np, Nj, is_root, T, Bc = aux
    plan = ctx.plan(dA, int(inp["roots"].numel()), Np, Nj, is_root, Bc)
    X = torch.randn(Nj.numel(), dtype=torch.float64, device="cuda")
    Z = ctx.masked_product(plan, dA.vals, X, True, precision)  # warm-up / allocation
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # the launches queue faster than they run, so the events bracket
    # back-to-back kernels (no allocation inside the loop)
    ev0.record()
    for _ in range(reps):
        ctx.masked_product(plan, dA.vals, X, True, precision, out=Z)
    ev1.record()
    torch.cuda.synchronize()
    dur = ev0.elapsed_time(ev1) / 1e3 / reps
    _, st, _ = ctx.energy_min(plan, dA.vals, T, R.RN_CG, 1, precision)
    plan.close()
    return dur, st.spgemm_bytes, st.spgemm_flops


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
    return t_fb, t_f, int(Nj.numel())


def traffic_bytes():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SRCS:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_BYTES if h.hexdigest()[:16] == TRAFFIC_SRC_SHA else None


def product_batched(inp, aux, batch, reps):
    """The same FP64 product on `batch` copies of the operator (values and X
    per copy, shared structure): seconds per launch.  Context for the
    single-problem roofline: with more blocks in flight the last partial
    generation of wave slots is a smaller share of the launch."""
    import torch
    import paper_1610_03154_amd as R
    ctx, dA = inp["ctx"], inp["dA"]
    Np, Nj, is_root, T, Bc = aux
    plan = ctx.plan(dA, int(inp["roots"].numel()), Np, Nj, is_root, Bc)
    A = dA.vals.repeat(batch, 1)
    X = torch.randn((batch, Nj.numel()), dtype=torch.float64, device="cuda")
    Z = ctx.masked_product(plan, A, X, True, R.RN_FP64)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        ctx.masked_product(plan, A, X, True, R.RN_FP64, out=Z)
    ev1.record()
    torch.cuda.synchronize()
    plan.close()
    return ev0.elapsed_time(ev1) / 1e3 / reps


def other_configs(reps):
    """The study's other two configurations at full size on the same GPU path,
    aggregation precomputed on the host (an input), seconds per setup
    (strength -> pattern -> T -> plan -> energy minimisation), FP64 and
    FP32-mixed:
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

    def rel(a, b):
        a, b = a.double(), b.double()
        return float((a - b).abs().max() / b.abs().max())

    A = W.upwind_cd(1024)
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    Sp, Sj = ctx.strength(dA, 0.0)
    a, r = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(a, device="cuda"), torch.as_tensor(r, device="cuda")
    B = torch.ones((A.n_rows, 1), dtype=torch.float64, device="cuda")
    res = {}
    for prec, key in ((R.RN_FP64, "fp64"), (R.RN_FP32_MIXED, "fp32_mixed")):
        t, s = timed(lambda: R.setup(ctx, dA, B, 0.0, 2, 8, R.RN_GMRES, prec, Bhat=B, agg=agg, roots=roots))
        out["upwind1024_gmres_P_RT_s_" + key] = t
        res[key] = (s.P.clone(), s.RT.clone())
        del s
    out["upwind1024_fp32_mixed_max_rel_dP_dRT_vs_fp64"] = max(rel(res["fp32_mixed"][0], res["fp64"][0]),
                                                               rel(res["fp32_mixed"][1], res["fp64"][1]))
    Ab, xy = W.q1_elasticity(512)
    dA = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=Ab.n_nodes * 2, block_m=2)
    Sp, Sj = ctx.strength(dA, 0.0)
    a, r = R.aggregate_host(Sp.cpu().numpy(), Sj.cpu().numpy())
    agg, roots = torch.as_tensor(a, device="cuda"), torch.as_tensor(r, device="cuda")
    B = torch.as_tensor(W.rbm(xy), device="cuda")
    res = {}
    for prec, key in ((R.RN_FP64, "fp64"), (R.RN_FP32_MIXED, "fp32_mixed")):
        t, s = timed(lambda: R.setup(ctx, dA, B, 0.0, 2, 6, R.RN_CG, prec, agg=agg, roots=roots))
        out["elastic512_cg_s_" + key] = t
        res[key] = s.P.clone()
        del s
    out["elastic512_fp32_mixed_max_rel_dP_vs_fp64"] = rel(res["fp32_mixed"], res["fp64"])
    return out


def cpu_baseline(budget_s=12.0):
    """The oracle (single-threaded C) on the same step, repeated for ~budget."""
    import oracle as O
    import workloads as W
    A = W.q1_aniso(NX, EPS, PSI)
    B = W.ones(A.n_rows)
    Sp, Sj = O.strength(A.rowptr, A.colind, A.vals, 1, THETA)
    agg, roots = O.aggregate(Sp, Sj)
    times = []
    t_end = time.perf_counter() + budget_s
    while True:
        t0 = time.perf_counter()
        st = O.setup(A, B, 1, THETA, DEGREE, agg=agg, roots=roots)
        O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1, st["T"],
                  ITERS)
        times.append(time.perf_counter() - t0)
        if time.perf_counter() > t_end or len(times) >= 50:
            break
    return float(np.median(times)), len(times)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=200, help="launches for the kernel roofline timing")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--fb-reps", type=int, default=5, help="repetitions of the batched forward+backward")
    ap.add_argument("--roofline-only", action="store_true", help="only the masked-product timing loop")
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
    if args.roofline_only:
        P, st, plan, aux = gpu_step(inp, R.RN_FP64)
        plan.close()
        dur, nbytes, _ = roofline(inp, aux, R.RN_FP64, args.reps)
        print(json.dumps({"kernel_avg_us": dur * 1e6, "bytes": nbytes, "GBps": nbytes / dur / 1e9}))
        return
    wall64, ev64, P64, st64, aux = time_steps(inp, R.RN_FP64, args.steps, args.warmup)
    wall32, ev32, P32, st32, _ = time_steps(inp, R.RN_FP32_MIXED, args.steps, args.warmup)
    dur, nbytes, flops = roofline(inp, aux, R.RN_FP64, args.reps)
    dur32, nbytes32, _ = roofline(inp, aux, R.RN_FP32_MIXED, args.reps)
    t_fb, t_f, nnz_n5 = fwd_bwd(args.fb_reps)
    dur_b4 = product_batched(inp, aux, 4, max(args.reps // 4, 10))
    others = other_configs(args.other_reps) if args.other_reps > 0 else {}
    achieved = nbytes / dur / 1e9
    p64 = P64.cpu().numpy()
    mix_err = float(np.max(np.abs(P32.cpu().numpy() - p64)) / np.max(np.abs(p64)))
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
        "fp32_mixed_max_rel_dP_vs_fp64": mix_err,
        "spgemm_GBps_fp64": achieved,
        "spgemm_GBps_fp32_mixed": nbytes32 / dur32 / 1e9,
        "spgemm_us_fp64": dur * 1e6,
        "spgemm_us_fp32_mixed": dur32 * 1e6,
        "spgemm_batch4_us_per_problem": dur_b4 * 1e6 / 4,
        "spgemm_batch4_GBps_fp64": 4 * nbytes / dur_b4 / 1e9,
        "spgemm_batch4_frac_of_peak": 4 * nbytes / dur_b4 / 1e9 / HBM_PEAK_GBS,
        "fwd_bwd_s": t_fb,
        "fwd_bwd_workload": f"16 x q1_aniso 256x256 (eps 10^U(-3,0), angle U(0,pi), seed 0), theta 0, "
                            f"S^2 C (nnz_N {nnz_n5} each), 6 CG steps FP64, loss <W,P>",
        "fwd_only_s": t_f,
        **others,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_bytes(),
                     "kernel": "k_spgemm_p<NB=1,MODE_PRODUCT,fp64,256 lanes> (persistent)",
                     "bytes_per_launch": nbytes, "flops_per_launch": flops},
    }
    if not args.no_cpu:
        med, cnt = cpu_baseline()
        out["cpu_baseline"] = {"value": med, "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": f"the full step (strength, pattern, tentative, 6 CG steps) on the "
                                         f"512x512 workload, median of {cnt} runs"}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
