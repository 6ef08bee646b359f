"""GPU adjoint of the CG energy minimisation (map: stored values of A -> P).

The reverse sweep runs in the library (rn_energy_min_bwd through the C ABI,
and torch.autograd through EnergyMinOperator).  It is checked against
  * the oracle's tangent-linear model (forward mode, pinned itself by central
    differences in the oracle tests): <W, J v> = <J^T W, v> for random v, and
    the full gradient from every unit direction on a 32 x 32 problem;
  * central finite differences of the GPU forward map (FP64), the stated bar
    of rel 1e-6.
The workload is the batched rotated-anisotropic family (theta = 0, pattern
S^2 C, 6 CG steps), shared structure, values per problem.
"""
import functools

import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

K = 6
# <W, J v> from the oracle's forward mode and <J^T W, v> from the GPU reverse
# mode are the same derivative evaluated in different orders; both carry
# rounding of O(1e-16) amplified by the recurrence, so 1e-9 is ample.
JVP_TOL = 1e-9
FD_TOL = 1e-6


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
def problem(nx, batch):
    """Structure, values [batch, nnz], oracle setup (pattern, T, Bc), loss weights."""
    A0, vals, params, rng = W.aniso_batch(nx, batch, 0)
    st = O.setup(A0, W.ones(A0.n_rows), 1, 0.0, 2)
    Wt = W.loss_weights(rng, batch, st["Nj"].size)
    return A0, vals, st, Wt


def operator(R, ctx, A0, st):
    A = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
    return R.EnergyMinOperator(ctx, A, int(st["nc"]), dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"]),
                               dev(st["T"]), dev(st["Bc"]), K)


def oracle_jvp(A0, vals_b, st, v):
    return O.emin_cg_jvp(A0.rowptr, A0.colind, vals_b, v, st["Np"], st["Nj"], st["is_root"], st["nc"],
                         st["Bc"], 1, st["T"], K)


def gpu_grad(R, ctx, op, vals, Wt):
    import torch
    a = dev(vals).requires_grad_(True)
    P = op(a)
    (g,) = torch.autograd.grad((P * dev(Wt).reshape(P.shape)).sum(), a)
    return P.detach().cpu().numpy(), g.cpu().numpy()


def test_forward_with_tape_matches_oracle(R, ctx):
    A0, vals, st, Wt = problem(32, 1)
    op = operator(R, ctx, A0, st)
    P, _ = gpu_grad(R, ctx, op, vals[0], Wt[0])
    Po, info = O.emin_cg(A0.rowptr, A0.colind, vals[0], st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1,
                         st["T"], K)
    assert info["status"] == 0
    assert np.max(np.abs(P - Po)) / np.max(np.abs(Po)) <= 1e-12
    op.close()


def test_adjoint_full_gradient_32(R, ctx):
    """Every one of the nnz(A) unit directions through the oracle's JVP."""
    A0, vals, st, Wt = problem(32, 1)
    op = operator(R, ctx, A0, st)
    _, g = gpu_grad(R, ctx, op, vals[0], Wt[0])
    nnz = A0.nnz
    go = np.empty(nnz)
    e = np.zeros(nnz)
    for t in range(nnz):
        e[t] = 1.0
        _, dP = oracle_jvp(A0, vals[0], st, e)
        go[t] = float(Wt[0] @ dP)
        e[t] = 0.0
    err = np.linalg.norm(g - go) / np.linalg.norm(go)
    assert err <= JVP_TOL, err
    op.close()


@pytest.mark.parametrize("nx,batch", [(32, 4), (64, 3)])
def test_adjoint_dot_product_batched(R, ctx, nx, batch):
    """<J^T W, v> (GPU reverse) == <W, J v> (oracle forward) per batch entry."""
    A0, vals, st, Wt = problem(nx, batch)
    op = operator(R, ctx, A0, st)
    _, g = gpu_grad(R, ctx, op, vals, Wt)
    rng = np.random.default_rng(7)
    for b in range(batch):
        for _ in range(3):
            v = rng.standard_normal(A0.nnz)
            _, dP = oracle_jvp(A0, vals[b], st, v)
            lhs, rhs = float(g[b] @ v), float(Wt[b] @ dP)
            assert abs(lhs - rhs) <= JVP_TOL * (abs(rhs) + np.linalg.norm(g[b]) * np.linalg.norm(v) * 1e-3), \
                (b, lhs, rhs)
    op.close()


def test_adjoint_central_differences_gpu_forward(R, ctx):
    """Central FD (FP64) of the GPU forward map, h = 1e-6 max|a|: over 64
    random stored entries ||g_fd - g|| / ||g|| <= 1e-6, and along 4 random
    directions |fd - <g, v>| <= 1e-6 |<g, v>|.  A single tiny entry is not
    judged on its own: the FD's rounding noise, about eps |L| / h, is ~1e-8
    absolute here."""
    import torch
    A0, vals, st, Wt = problem(32, 1)
    op = operator(R, ctx, A0, st)
    a0 = vals[0]
    _, g = gpu_grad(R, ctx, op, a0, Wt[0])
    h = 1e-6 * np.max(np.abs(a0))

    def loss(a):
        with torch.no_grad():
            P = op(dev(a))
        return float(P.cpu().numpy() @ Wt[0])

    rng = np.random.default_rng(11)
    idx = rng.choice(A0.nnz, 64, replace=False)
    fd = np.empty(idx.size)
    for q, t in enumerate(idx):
        e = np.zeros(A0.nnz)
        e[t] = h
        fd[q] = (loss(a0 + e) - loss(a0 - e)) / (2 * h)
    err = np.linalg.norm(fd - g[idx]) / np.linalg.norm(g[idx])
    assert err <= FD_TOL, err
    for _ in range(4):
        v = rng.standard_normal(A0.nnz)
        v *= h / np.linalg.norm(v) * np.sqrt(A0.nnz)
        fdv = (loss(a0 + v) - loss(a0 - v)) / 2
        assert abs(fdv - g @ v) <= FD_TOL * abs(g @ v), (fdv, g @ v)
    op.close()


def test_adjoint_with_early_stop(R, ctx):
    """A problem whose CG converges before K: the reverse sweep follows the
    forward's own step count."""
    A = W.laplace1d(8)
    st = O.setup(A, W.ones(A.n_rows), 1, 0.25, 1)
    Kbig = 12
    Po, info = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1,
                         st["T"], Kbig)
    assert info["iters"] < Kbig
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    op = R.EnergyMinOperator(ctx, dA, int(st["nc"]), dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"]),
                             dev(st["T"]), dev(st["Bc"]), Kbig)
    rng = np.random.default_rng(3)
    Wt = rng.standard_normal(st["Nj"].size)
    P, g = gpu_grad(R, ctx, op, A.vals, Wt)
    assert np.max(np.abs(P - Po)) <= 1e-12
    v = rng.standard_normal(A.nnz)
    _, dP = O.emin_cg_jvp(A.rowptr, A.colind, A.vals, v, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 1,
                          st["T"], Kbig)
    assert abs(float(g @ v) - float(Wt @ dP)) <= JVP_TOL * max(1.0, abs(float(Wt @ dP)))
    op.close()


def test_bwd_rejects_unrecorded_tape(R, ctx):
    A0, vals, st, Wt = problem(32, 1)
    op = operator(R, ctx, A0, st)
    tape = ctx.tape(op.plan, 1, K)
    with pytest.raises(R.RnError):
        ctx.energy_min_bwd(op.plan, op.plan_T, op.perm, tape, dev(vals[0]), dev(Wt[0]))
    with pytest.raises(R.RnError):  # a tape records the FP64 CG form only
        ctx.energy_min(op.plan, dev(vals[0]), op.T, R.RN_GMRES, K, R.RN_FP64, tape=tape)
    tape.close()
    op.close()


@pytest.mark.parametrize("case", ["batch", "early_stop"])
def test_checkpoint_interval_gives_the_same_gradient(R, case):
    """RN_OPT_TAPE_INTERVAL: the reverse sweep recomputes the steps between
    checkpoints with the recorded step lengths and the forward's own
    expressions, so every interval (1 = every step kept, 0 = ceil(sqrt(K)),
    up to one checkpoint for the whole run) gives the same gradient bit for
    bit, and the default matches the oracle's tangent model.  The taped
    forward with the direction formed inside the next product
    (RN_OPT_FUSED_CG = 1, the default) records the same iterates as with a
    separate direction pass, so the gradient is the same bit for bit too."""
    if case == "batch":
        A0, vals, st, Wt = problem(64, 3)
        Kc = K
    else:
        A0 = W.laplace1d(8)
        st = O.setup(A0, W.ones(A0.n_rows), 1, 0.25, 1)
        vals = A0.vals[None, :].copy()
        Wt = np.random.default_rng(3).standard_normal((1, st["Nj"].size))
        Kc = 12  # converges before K
    grads = {}
    runs = [(c, 1) for c in (1, 0, 2, 4, Kc, Kc + 3)] + [(c, 0) for c in (1, 0, Kc + 3)]
    for c, fused in runs:
        cx = R.Context()
        cx.set_option(R._lib.RN_OPT_TAPE_INTERVAL, c)
        cx.set_option(R._lib.RN_OPT_FUSED_CG, fused)
        dA = R.DeviceCSR.from_host(A0.rowptr, A0.colind, A0.vals)
        op = R.EnergyMinOperator(cx, dA, int(st["nc"]), dev(st["Np"]), dev(st["Nj"]), dev(st["is_root"]),
                                 dev(st["T"]), dev(st["Bc"]), Kc)
        P, g = gpu_grad(R, cx, op, vals if vals.shape[0] > 1 else vals[0], Wt if Wt.shape[0] > 1 else Wt[0])
        grads[(c, fused)] = (P, g)
        op.close()
        cx.close()
    P1, g1 = grads[(1, 0)]
    for (c, fused), (P, g) in grads.items():
        assert np.array_equal(P, P1) and np.array_equal(g, g1), \
            f"interval {c}, fused {fused}: max |dP| {np.max(np.abs(P - P1))}, max |dg| {np.max(np.abs(g - g1))}"
    g = g1.reshape(len(Wt), -1)
    rng = np.random.default_rng(5)
    for b in range(len(Wt)):
        v = rng.standard_normal(A0.nnz)
        _, dP = O.emin_cg_jvp(A0.rowptr, A0.colind, vals[b], v, st["Np"], st["Nj"], st["is_root"], st["nc"],
                              st["Bc"], 1, st["T"], Kc)
        rhs = float(Wt[b] @ dP)
        assert abs(float(g[b] @ v) - rhs) <= JVP_TOL * max(1.0, abs(rhs))


def test_tape_interval_option_values(R):
    cx = R.Context()
    with pytest.raises(R.RnError):
        cx.set_option(R._lib.RN_OPT_TAPE_INTERVAL, -1)
    cx.close()
