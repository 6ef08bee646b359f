"""GPU parity of the masked product's code paths, against the CPU oracle.

The persistent product for scalar operators stages each product block's
A slice, X window and projection data in LDS; blocks whose neighbour rows do
not form a window read X from global memory, and blocks with more A entries
than the LDS capacity read A from global memory too.  These cases make each
path carry whole launches, plus batches with per-entry values.  (The
selectable block sizes and paths are in test_gpu_options.)  Same bars as test_gpu_parity: FP64 1e-12, FP32-mixed
1e-5 relative to max|ref|.
"""
import numpy as np
import pytest

from tests import cases as CS
from tests.test_gpu_parity import R, ctx, dev, host, run_path  # noqa: F401  (fixtures and helpers)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def _product_refs(A, Np, Nj, nc, is_root, Bc, nB, X):
    import oracle as O
    ref = O.masked_product(A.rowptr, A.colind, A.vals, Np, Nj, nc, X)
    root_e = np.repeat(is_root, np.diff(Np)).astype(bool)
    return np.where(root_e, 0.0, ref), O.project(Np, Nj, is_root, Bc, nB, ref), root_e


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_irregular_structure_product_and_cg(R, ctx, precision):
    """Circulant graph with far neighbours: no X windows."""
    c = CS.case("ring20k")
    g = run_path(R, ctx, c)
    prec = R.RN_FP64 if precision == "fp64" else R.RN_FP32_MIXED
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    X = np.random.default_rng(5).standard_normal(c["Nj"].size)
    ref_m, refp, root_e = _product_refs(c["A"], c["Np"], c["Nj"], c["nc"], c["is_root"], c["Bc"], 1, X)
    Z = host(ctx.masked_product(g["plan"], g["A"].vals, dev(X), project=False, precision=prec))
    Zp = host(ctx.masked_product(g["plan"], g["A"].vals, dev(X), project=True, precision=prec))
    scale = np.max(np.abs(ref_m))
    assert np.max(np.abs(Z - ref_m)) <= tol * scale
    assert np.max(np.abs(Zp - refp)) <= tol * scale
    P, st, _ = ctx.energy_min(g["plan"], g["A"].vals, g["T"], R.RN_CG, c["iters"], prec)
    assert CS.rel_max(host(P), c["P"]) <= tol


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batched_product(R, ctx, precision):
    """Three operators on one structure in one launch: each batch entry has its
    own A values and X and must match the oracle on its own."""
    import torch
    c = CS.case("aniso40")
    g = run_path(R, ctx, c)
    A = c["A"]
    rng = np.random.default_rng(8)
    scales = np.array([1.0, 0.5, 3.0])
    vals = np.stack([A.vals * s for s in scales])
    X = rng.standard_normal((3, c["Nj"].size))
    prec = R.RN_FP64 if precision == "fp64" else R.RN_FP32_MIXED
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    Zp = host(ctx.masked_product(g["plan"], dev(vals), dev(X), project=True, precision=prec))
    for b in range(3):
        Ab = type(A)(A.n_rows, A.n_cols, A.rowptr, A.colind, vals[b])
        _, refp, _ = _product_refs(Ab, c["Np"], c["Nj"], c["nc"], c["is_root"], c["Bc"], 1, X[b])
        assert np.max(np.abs(Zp[b] - refp)) <= tol * np.max(np.abs(refp)), b
    torch.cuda.synchronize()


def test_blocks_beyond_lds_capacity(R, ctx):
    """One pattern entry per row (the row's aggregate): 256 rows per product
    block, so every block holds far more A entries than the LDS stages."""
    import oracle as O
    c = CS.case("aniso40")
    A = c["A"]
    n = A.n_rows
    agg, is_root = c["agg"], c["is_root"]
    Np = np.arange(n + 1, dtype=np.int32)
    Nj = agg.astype(np.int32)
    nc = int(c["roots"].size)
    Bc = np.random.default_rng(3).uniform(0.5, 2.0, (nc, 1))
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    plan = ctx.plan(dA, nc, dev(Np), dev(Nj), dev(is_root), dev(Bc))
    X = np.random.default_rng(4).standard_normal(n)
    ref_m, refp, root_e = _product_refs(A, Np, Nj, nc, is_root, Bc, 1, X)
    Z = host(ctx.masked_product(plan, dA.vals, dev(X), project=False))
    Zp = host(ctx.masked_product(plan, dA.vals, dev(X), project=True))
    scale = np.max(np.abs(ref_m))
    assert np.max(np.abs(Z - ref_m)) <= FP64_TOL * scale
    assert np.max(np.abs(Zp - refp)) <= FP64_TOL * scale
    # with one entry per row the projection removes every F entry (G^+ = 1/Bc^2)
    assert np.max(np.abs(Zp[~root_e])) <= 1e-12 * scale
    plan.close()
    del O


def _banded(n, hb):
    """Symmetric banded graph |i - j| <= hb (diagonal included), CSR."""
    rows = [np.arange(max(0, i - hb), min(n, i + hb + 1), dtype=np.int32) for i in range(n)]
    Sp = np.zeros(n + 1, dtype=np.int32)
    Sp[1:] = np.cumsum([r.size for r in rows])
    return Sp, np.concatenate(rows).astype(np.int32)


@pytest.mark.parametrize("hb,d", [(5, 6), (5, 7), (6, 5)])
def test_compact_record_limits(R, ctx, hb, d):
    """The persistent product's 8-byte records hold 11 A terms of 5-bit
    codes.  Banded operators |i - j| <= hb with node-pair aggregates: hb 5,
    degree 6 sits on both limits (11 A entries per row, neighbour rows of
    31 entries: code 30 is used); hb 5, degree 7 has longer rows and hb 6
    more A entries per row, so those plans keep the 12-byte records only."""
    import oracle as O
    import workloads as W
    n = 300
    offs = [(k, 0) for k in range(-hb, hb + 1)]
    A = W._csr_from_offsets(n, 1, offs, [2.0 * hb + 1.5 if k == 0 else -1.0 + 0.05 * k for k, _ in offs])
    Sp, Sj = _banded(n, hb)
    agg = (np.arange(n) // 2).astype(np.int32)
    roots = np.arange(0, n, 2, dtype=np.int32)
    Npn, Njn = O.pattern_nodes(Sp, Sj, agg, roots.size, d)
    Np, Nj, is_root = O.pattern_dofs(Npn, Njn, agg, roots, 1)
    assert int(np.diff(Np).max()) == {(5, 6): 31, (5, 7): 36, (6, 5): 31}[(hb, d)]
    nc = int(roots.size)
    Bc = np.random.default_rng(11).uniform(0.5, 2.0, (nc, 1))
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    plan = ctx.plan(dA, nc, dev(Np), dev(Nj), dev(is_root), dev(Bc))
    try:
        X = np.random.default_rng(12).standard_normal(Nj.size)
        ref_m, refp, _ = _product_refs(A, Np, Nj, nc, is_root, Bc, 1, X)
        Z = host(ctx.masked_product(plan, dA.vals, dev(X), project=False))
        Zp = host(ctx.masked_product(plan, dA.vals, dev(X), project=True))
        scale = np.max(np.abs(ref_m))
        assert np.max(np.abs(Z - ref_m)) <= FP64_TOL * scale
        assert np.max(np.abs(Zp - refp)) <= FP64_TOL * scale
    finally:
        plan.close()


@pytest.mark.parametrize("hb,d", [(20, 1), (8, 2), (35, 2), (0, 0)])
def test_pattern_row_widths(R, ctx, hb, d):
    """Pattern levels of every width: rows gathered in the small window
    (hb 20, d 1), rows gathered by the large-window kernel whose distinct
    columns still fit a padded row (hb 8, d 2), rows with more than 64
    distinct columns (hb 35, d 2: the expansion is redone with CSR levels),
    and degree 0.  Aggregates are node pairs, so odd nodes keep their
    expanded rows."""
    import oracle as O
    n = 300
    Sp, Sj = _banded(n, hb)
    agg = (np.arange(n) // 2).astype(np.int32)
    roots = np.arange(0, n, 2, dtype=np.int32)
    Np, Nj, is_root = ctx.pattern(dev(Sp), dev(Sj), dev(agg), dev(roots), d, 1)
    Npn, Njn = O.pattern_nodes(Sp, Sj, agg, roots.size, d)
    Np_o, Nj_o, ir_o = O.pattern_dofs(Npn, Njn, agg, roots, 1)
    widest = int(np.diff(Npn).max())
    assert (widest > 64) == ((hb, d) == (35, 2))
    assert np.array_equal(host(Np), Np_o) and np.array_equal(host(Nj), Nj_o)
    assert np.array_equal(host(is_root), ir_o)


@pytest.mark.parametrize("name", ["elastic7", "elastic32_t03"])
def test_node_blocked_unaligned_x(R, ctx, name):
    """Node-blocked product: with X aligned to a pair of doubles each term's
    X values come as two-element loads, with X one double off as single
    loads; the arithmetic and its order are the same, so both give the same
    bits and match the oracle."""
    import torch
    import oracle as O
    c = CS.case(name)
    g = run_path(R, ctx, c)
    X = np.random.default_rng(12).standard_normal(c["Nj"].size)
    Xa = dev(X)
    buf = torch.zeros(X.size + 2, dtype=torch.float64, device="cuda")
    buf[1:1 + X.size] = Xa
    Xu = buf[1:1 + X.size]
    assert Xa.data_ptr() % 16 == 0 and Xu.data_ptr() % 16 == 8
    A = c["A"]
    ref = O.masked_product(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["nc"], X)
    refp = O.project(c["Np"], c["Nj"], c["is_root"], c["Bc"], c["B"].shape[1], ref)
    for project in (False, True):
        Za = host(ctx.masked_product(g["plan"], g["A"].vals, Xa, project=project))
        Zu = host(ctx.masked_product(g["plan"], g["A"].vals, Xu, project=project))
        assert np.array_equal(Za, Zu), f"project={project}: max diff {np.max(np.abs(Za - Zu))}"
    assert np.max(np.abs(Za - refp)) <= FP64_TOL * np.max(np.abs(refp))
    g["plan"].close()


@pytest.mark.parametrize("degree", [2, 1])
def test_node_blocked_wide_rows(R, ctx, degree):
    """Node-blocked operator with 25 block terms per row (5 x 5 node stencil,
    2 x 2 SPD blocks) and aggregates of two nodes (an input).  Degree 2:
    pattern rows of up to 45 node entries, so a product block holds 6 to 20
    rows, stages its A slice, and each row's position codes run past the
    first three words of its record; degree 1: blocks of 32 to 42 rows hold
    more A entries than the LDS stages, so they read A from global memory.
    Strength and pattern bit for bit; T, the product (X aligned to a pair of
    doubles and one double off) and 4 CG steps at the FP64 bar against the
    oracle."""
    import torch
    import oracle as O
    import workloads as W
    nx = 12
    nn = nx * nx
    offs = [(dx, dy) for dy in range(-2, 3) for dx in range(-2, 3)]
    S = W._csr_from_offsets(nx, nx, offs, [30.0 if o == (0, 0) else -1.0 for o in offs])
    K2 = np.array([[2.0, 0.5], [0.5, 1.0]])
    Ab = W.BSR(nn, 2, S.rowptr, S.colind, S.vals[:, None, None] * K2)
    A = Ab.to_csr()
    coords = np.stack([(np.arange(nn) % nx + 1) / nx, (np.arange(nn) // nx) / nx], 1)
    B = W.rbm(coords)
    agg = (np.arange(nn) // 2).astype(np.int32)
    roots = np.arange(0, nn, 2).astype(np.int32)
    st = O.setup(A, B, 2, 0.0, degree, agg=agg, roots=roots)
    assert np.max(np.diff(Ab.rowptr)) == 25
    dA = R.DeviceCSR.from_host(Ab.rowptr, Ab.colind, Ab.vals.reshape(-1), n=2 * nn, block_m=2)
    Sp, Sj = ctx.strength(dA, 0.0)
    assert np.array_equal(host(Sp), st["Sp"]) and np.array_equal(host(Sj), st["Sj"])
    Np, Nj, is_root = ctx.pattern(Sp, Sj, dev(agg), dev(roots), degree, 2)
    assert np.array_equal(host(Np), st["Np"]) and np.array_equal(host(Nj), st["Nj"])
    assert np.array_equal(host(is_root), st["is_root"])
    T, Bc, rd = ctx.tentative(Np, Nj, is_root, dev(agg), dev(roots), 2, dev(B))
    assert rd == 0
    assert np.max(np.abs(host(T) - st["T"])) <= FP64_TOL * np.max(np.abs(st["T"]))
    plan = ctx.plan(dA, st["nc"], Np, Nj, is_root, Bc)
    X = np.random.default_rng(21).standard_normal(st["Nj"].size)
    ref = O.masked_product(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["nc"], X)
    refp = O.project(st["Np"], st["Nj"], st["is_root"], st["Bc"], 3, ref)
    Xa = dev(X)
    buf = torch.zeros(X.size + 2, dtype=torch.float64, device="cuda")
    buf[1:1 + X.size] = Xa
    Xu = buf[1:1 + X.size]
    Za = host(ctx.masked_product(plan, dA.vals, Xa, project=True))
    Zu = host(ctx.masked_product(plan, dA.vals, Xu, project=True))
    assert np.array_equal(Za, Zu)
    assert np.max(np.abs(Za - refp)) <= FP64_TOL * np.max(np.abs(refp))
    P, s, _ = ctx.energy_min(plan, dA.vals, T, R.RN_CG, 4, R.RN_FP64)
    Pref, info = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 3,
                           st["T"], 4)
    err = CS.rel_max(host(P), Pref)
    print(f"wide node-blocked rows, degree {degree}: max|dP|/max|P| = {err:.2e}")
    assert s.status_code == 0 and s.iters_done == info["iters"]
    assert err <= FP64_TOL
    plan.close()
