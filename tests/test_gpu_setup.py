"""The one-shot set-up (rn_setup): every stage inside one library call.

It runs the same kernels as the stage calls, so its outputs must equal the
staged path's bit for bit (integer arrays, T, Bc, P, R^T), and P / R^T must
match the oracle to the parity bars (FP64 1e-12, FP32-mixed 1e-5).
"""
import numpy as np
import pytest

from tests import cases as CS
from tests.test_gpu_parity import R, ctx, dev, dev_matrix, host, run_path  # noqa: F401  (fixtures and helpers)

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


@pytest.mark.parametrize("name,precision", [("aniso40", "fp64"), ("aniso40", "mixed"), ("upwind64", "fp64"),
                                            ("elastic7", "fp64"), ("twocand13", "fp64"), ("asym20", "fp64")])
def test_setup_matches_stages_and_oracle(R, ctx, name, precision):
    c = CS.case(name)
    prec = R.RN_FP64 if precision == "fp64" else R.RN_FP32_MIXED
    tol = FP64_TOL if precision == "fp64" else MIXED_TOL
    method = R.RN_GMRES if c["method"] == "gmres" else R.RN_CG
    gm = c["method"] == "gmres"
    A = dev_matrix(R, c)
    agg, roots, B = dev(c["agg"]), dev(c["roots"]), dev(c["B"])
    Bhat = dev(c["Bhat"]) if gm else None
    s = ctx.setup_native(A, B, agg, roots, c["theta"], c["degree"], c["iters"], method, prec, Bhat=Bhat)
    try:
        g = run_path(R, ctx, c)
        for key, ref in (("S_rowptr", g["Sp"]), ("S_colind", g["Sj"]), ("N_rowptr", g["Np"]),
                         ("N_colind", g["Nj"]), ("is_root", g["is_root"]), ("T", g["T"]), ("Bc", g["Bc"])):
            assert np.array_equal(host(s.tensor(key)), host(ref).reshape(-1)), key
        assert s.view.rank_deficient == g["rd"]
        P_ref, _, _ = ctx.energy_min(g["plan"], g["A"].vals, g["T"], method, c["iters"], prec)
        P = host(s.tensor("P"))
        assert np.array_equal(P, host(P_ref))
        assert CS.rel_max(P, c["P"]) <= tol
        assert s.stats.iters_done == c["iters"] or gm
        if gm:
            RT = host(s.tensor("RT"))
            assert CS.rel_max(RT, c["RT"]) <= tol
            assert s.stats_RT is not None and s.stats_RT.iters_done >= 1
        else:
            assert s.tensor("RT") is None
        g["plan"].close()
    finally:
        s.close()


def test_setup_reports_bad_input(R, ctx):
    """A malformed aggregation (an index past n_agg) is an RN_EINVAL of the
    call, and nothing is kept."""
    c = CS.case("poisson32")
    A = dev_matrix(R, c)
    bad = c["agg"].copy()
    bad[5] = c["roots"].size + 3
    with pytest.raises(R.RnError) as e:
        ctx.setup_native(A, dev(c["B"]), dev(bad), dev(c["roots"]), c["theta"], 2, 2)
    from paper_1610_03154_amd import _lib
    assert e.value.status == _lib.RN_EINVAL


def test_setup_wide_pattern_rows(R, ctx):
    """A banded operator (|i - j| <= 35) with node-pair aggregates: the
    distance-2 pattern rows hold 71 aggregates, more than a padded level
    row takes, so the set-up redoes the pattern with exact CSR levels."""
    import oracle as O
    import workloads as W
    n, hb = 300, 35
    offs = [(d, 0) for d in range(-hb, hb + 1)]
    A = W._csr_from_offsets(n, 1, offs, [2.0 * hb + 10.0 if d == 0 else -1.0 for d, _ in offs])
    agg = (np.arange(n) // 2).astype(np.int32)
    roots = np.arange(0, n, 2, dtype=np.int32)
    B = np.ones((n, 1))
    ref = O.setup(A, B, 1, 0.0, 2, agg=agg, roots=roots)
    assert int(np.diff(ref["Npn"]).max()) > 64
    P_ref, _ = O.emin_cg(A.rowptr, A.colind, A.vals, ref["Np"], ref["Nj"], ref["is_root"], ref["nc"], ref["Bc"], 1,
                         ref["T"], 2)
    dA = R.DeviceCSR.from_host(A.rowptr, A.colind, A.vals)
    s = ctx.setup_native(dA, dev(B), dev(agg), dev(roots), 0.0, 2, 2)
    try:
        assert np.array_equal(host(s.tensor("N_rowptr")), ref["Np"])
        assert np.array_equal(host(s.tensor("N_colind")), ref["Nj"])
        assert CS.rel_max(host(s.tensor("P")), P_ref) <= FP64_TOL
    finally:
        s.close()


@pytest.mark.parametrize("name", ["poisson32", "elastic7"])
def test_singular_root_block_is_reported(R, ctx, name):
    """A zero root value of B (m = 1), or a singular 2x2 root block of the
    first two candidates (m = 2: both translations zeroed at one root node),
    cannot normalise T: the tentative stage and the one-call set-up return
    RN_ESINGULAR and keep nothing."""
    from paper_1610_03154_amd import _lib
    c = CS.case(name)
    m = c["m"]
    B = c["B"].copy()
    r = int(c["roots"][3])
    B[m * r:m * r + m, :m] = 0.0
    g = run_path(R, ctx, c)
    with pytest.raises(R.RnError) as e:
        ctx.tentative(g["Np"], g["Nj"], g["is_root"], dev(c["agg"]), dev(c["roots"]), m, dev(B))
    assert e.value.status == _lib.RN_ESINGULAR
    g["plan"].close()
    with pytest.raises(R.RnError) as e:
        ctx.setup_native(dev_matrix(R, c), dev(B), dev(c["agg"]), dev(c["roots"]), c["theta"], c["degree"],
                         c["iters"])
    assert e.value.status == _lib.RN_ESINGULAR
