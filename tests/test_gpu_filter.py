"""GPU parity of the post-filter lines of Alg. root_node_setup (Sec. 3.7):
rn_filter (Alg. filter), rn_enforce (Eq. Tproj) and the extra improve step,
against the oracle, through the C ABI.

The filter's decisions are integer results of FP64 comparisons; fed the same
values as the oracle it must keep exactly the same entries.  Enforce and the
extra step are floating point: 1e-12 (the node-blocked elasticity bar where
the FP64 spread is wider).  The whole pipeline from the GPU's own P is also
compared: its filtered pattern must equal the oracle's wherever no decision
lies within rounding of its threshold.
"""
import numpy as np
import pytest

import oracle as O
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


FILTER_CASES = [("poisson32", 0, 0.25), ("aniso40", 0, 0.1), ("aniso40", 3, 0.0), ("aniso40", 4, 0.2),
                ("upwind64", 0, 0.45), ("elastic7", 0, 0.5), ("elastic32", 2, 0.3), ("lap27_10", 0, 0.2),
                ("twocand13", 0, 0.3), ("aniso512", 0, 0.1), ("elastic512", 0, 0.3)]


@pytest.mark.parametrize("name,k,theta", FILTER_CASES)
def test_filter_and_enforce_on_oracle_values(R, ctx, name, k, theta):
    c = CS.case(name)
    m = c["m"]
    keep = O.filter_keep(c["Np"], c["Nj"], c["P"], c["agg"], m, k, theta, c["is_root"])
    Np2, Nj2, P2 = O.compact(c["Np"], c["Nj"], keep, c["P"])
    Fp, Fj, Fv = ctx.filter(dev(c["Np"]), dev(c["Nj"]), dev(c["is_root"]), dev(c["agg"]), dev(c["P"]), m, k, theta)
    assert np.array_equal(host(Fp), Np2) and np.array_equal(host(Fj), Nj2)
    assert np.array_equal(host(Fv), P2)
    print(f"{name} k={k} theta={theta}: kept {Nj2.size} of {c['Nj'].size}")
    Pe, rd = O.enforce(Np2, Nj2, c["is_root"], c["Bc"], c["B"], P2)
    V = dev(P2)
    rd_gpu = ctx.enforce(Fp, Fj, dev(c["is_root"]), dev(c["Bc"]), dev(c["B"]), V)
    assert rd_gpu == rd
    err = CS.rel_max(host(V), Pe)
    res = O.constraint_residual(Np2, Nj2, host(V), c["Bc"], c["B"])
    res_o = O.constraint_residual(Np2, Nj2, Pe, c["Bc"], c["B"])
    print(f"  enforce: max|dP|/max|P| = {err:.2e}, residual {res:.1e} (oracle {res_o:.1e}, {rd} rank-deficient rows)")
    assert err <= tol(name)
    # rows left with too few columns for every candidate keep a least-squares
    # residual (the same as the oracle's); otherwise P Bc = B is restored
    assert res <= res_o + 1e-12
    if rd == 0:
        assert res <= 1e-12


def _margin(c, P, theta):
    """Smallest relative distance of an off entry's block magnitude from the
    theta threshold of its row (the decisions a rounding difference could
    flip)."""
    if theta <= 0.0:
        return np.inf
    m, Np, Nj, agg = c["m"], c["Np"], c["Nj"], c["agg"]
    n = Np.size - 1
    rows = np.repeat(np.arange(n), np.diff(Np))
    F = c["is_root"][rows] == 0
    node = rows // m
    q = (np.arange(Nj.size) - Np[rows]) // m
    ident = Np[m * node] + m * q          # first DOF entry of the node entry (row m I)
    mag = np.zeros(Nj.size)
    np.maximum.at(mag, ident[F], np.abs(P[F]))
    rep = F & (rows % m == 0) & ((np.arange(Nj.size) - Np[rows]) % m == 0)
    g, nd = mag[rep], node[rep]
    off = Nj[rep] // m != agg[nd]
    offmax = np.zeros(n // m)
    np.maximum.at(offmax, nd[off], g[off])
    thr = theta * offmax[nd[off]]
    ok = thr > 0
    if not ok.any():
        return np.inf
    return float(np.min(np.abs(g[off][ok] - thr[ok]) / thr[ok]))


PIPE_CASES = [("aniso40", 0.1, "cg"), ("poisson37", 0.3, "cg"), ("upwind64", 0.45, "gmres"),
              ("elastic7", 0.5, "cg"), ("elastic32", 0.3, "cg"), ("aniso512", 0.1, "cg"),
              ("upwind1024", 0.45, "gmres"), ("elastic512", 0.3, "cg")]


@pytest.mark.parametrize("name,theta,method", PIPE_CASES)
def test_postfilter_pipeline_from_gpu_P(R, ctx, name, theta, method):
    c = CS.case(name)
    A = c["A"]
    m = c["m"]
    g = run_path(R, ctx, c)
    meth = R.RN_CG if method == "cg" else R.RN_GMRES
    P, _, _ = ctx.energy_min(g["plan"], g["A"].vals, g["T"], meth, c["iters"], R.RN_FP64)
    Fp, Fj, Pe, Pn, st, plan2 = ctx.postfilter(g["A"], g["Np"], g["Nj"], g["is_root"], g["agg"], g["Bc"],
                                               dev(c["B"]), P, theta=theta, method=meth)
    Np2, Nj2, Pe_o, Pn_o, info = O.postfilter(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["is_root"], c["agg"],
                                              m, c["nc"], c["Bc"], c["B"], c["P"], theta=theta, method=method)
    margin = _margin(c, c["P"], theta)
    print(f"{name} theta={theta}: kept {Nj2.size} of {c['Nj'].size}, smallest threshold margin {margin:.1e}")
    if margin < 1e-9:
        pytest.skip(f"a filter decision lies within {margin:.1e} of its threshold")
    assert np.array_equal(host(Fp), Np2) and np.array_equal(host(Fj), Nj2)
    assert st.status_code == 0 and st.iters_done == info["iters"]
    e1, e2 = CS.rel_max(host(Pe), Pe_o), CS.rel_max(host(Pn), Pn_o)
    print(f"  enforced {e1:.2e}, after the extra step {e2:.2e}")
    assert e1 <= tol(name) and e2 <= tol(name)
    plan2.close()
    g["plan"].close()


def test_filter_keeps_everything_at_zero_threshold(R, ctx):
    c = CS.case("aniso40")
    Fp, Fj, Fv = ctx.filter(dev(c["Np"]), dev(c["Nj"]), dev(c["is_root"]), dev(c["agg"]), dev(c["P"]), 1, 0, 0.0)
    assert np.array_equal(host(Fp), c["Np"]) and np.array_equal(host(Fj), c["Nj"])
    assert np.array_equal(host(Fv), c["P"])


def test_filter_rejects_mismatched_node_rows(R, ctx):
    import torch
    # two DOF rows of one (non-root) node with different lengths
    Np = dev(np.array([0, 4, 6], np.int32))
    Nj = dev(np.array([0, 1, 2, 3, 0, 1], np.int32))
    with pytest.raises(R.RnError) as e:
        ctx.filter(Np, Nj, dev(np.zeros(2, np.uint8)), dev(np.zeros(1, np.int32)),
                   torch.ones(6, dtype=torch.float64, device="cuda"), 2, 0, 0.5)
    assert e.value.status == R._lib.RN_EINVAL


def test_filter_empty_operator(R, ctx):
    import torch
    Np = dev(np.zeros(1, np.int32))
    e = torch.empty(0, dtype=torch.int32, device="cuda")
    Fp, Fj, Fv = ctx.filter(Np, e, torch.empty(0, dtype=torch.uint8, device="cuda"), e,
                            torch.empty(0, dtype=torch.float64, device="cuda"), 1, 0, 0.5)
    assert host(Fp).tolist() == [0] and Fj.numel() == 0
