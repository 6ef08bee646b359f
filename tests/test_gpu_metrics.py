"""GPU metrics against the oracle, through the C ABI (Sec. 4.1 energy, Sec. 4.2
projected residual, Eq. mode_constraint residual, Sec. 2.4 work units):
rn_energy, rn_constraint_residual and the fields RN_OPT_METRICS adds to
rn_emin_stats."""
import numpy as np
import pytest

import oracle as O
from tests import cases as CS
from tests.test_gpu_parity import dev, dev_matrix, host, run_path

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import paper_1610_03154_amd as R
    return R


def _ctx(R, metrics):
    ctx = R.Context()
    ctx.set_option(R._lib.RN_OPT_METRICS, metrics)
    return ctx


def _oracle_metrics(c, P):
    A = c["A"]
    Y = O.masked_product(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["nc"], P)
    E = O.energy(A.rowptr, A.colind, A.vals, c["Np"], c["Nj"], c["nc"], P)
    PY = O.project(c["Np"], c["Nj"], c["is_root"], c["Bc"], c["Bc"].shape[1], Y)
    return E, float(np.linalg.norm(PY)), float(np.linalg.norm(Y))


@pytest.mark.parametrize("name", ["aniso40", "elastic7", "upwind64", "twocand13"])
def test_energy_and_projected_residual(R, name):
    ctx = _ctx(R, 0)
    c = CS.case(name)
    g = run_path(R, ctx, c)
    for P in (c["P"], c["T"]):
        E, r, ny = _oracle_metrics(c, P)
        e_g, r_g = ctx.energy(g["plan"], g["A"].vals, dev(P))
        assert abs(e_g - E) <= 1e-12 * abs(E)
        assert abs(r_g - r) <= 1e-12 * ny + 1e-10 * r
    g["plan"].close()
    ctx.close()


@pytest.mark.parametrize("name", ["aniso40", "elastic7", "twocand13"])
def test_constraint_residual_of_a_perturbed_P(R, name):
    ctx = _ctx(R, 0)
    c = CS.case(name)
    P = c["P"].copy()
    F = np.flatnonzero(c["is_root"] == 0)
    rng = np.random.default_rng(8)
    i = int(F[len(F) // 2])
    P[c["Np"][i] + 1] += 0.375           # one F-row entry moved
    P[c["Np"][F[3]]] -= 1e-3             # and one in another row, the other way
    ref = O.constraint_residual(c["Np"], c["Nj"], P, c["Bc"], c["B"])
    got = ctx.constraint_residual(dev(c["Np"]), dev(c["Nj"]), dev(P), dev(c["Bc"]), dev(c["B"]))
    assert ref > 0.37 * np.max(np.abs(c["Bc"][c["Nj"][c["Np"][i] + 1]])) and got == ref
    # a root row moved off the identity counts too
    r = int(np.flatnonzero(c["is_root"])[0])
    P2 = c["P"].copy()
    P2[c["Np"][r]] = 0.5
    ref2 = O.constraint_residual(c["Np"], c["Nj"], P2, c["Bc"], c["B"])
    got2 = ctx.constraint_residual(dev(c["Np"]), dev(c["Nj"]), dev(P2), dev(c["Bc"]), dev(c["B"]))
    assert ref2 >= 0.5 * np.max(np.abs(c["B"][r])) - 1e-15 and got2 == ref2
    ctx.close()


@pytest.mark.parametrize("name,method", [("aniso40", "cg"), ("elastic7", "cg"), ("upwind64", "gmres")])
def test_stats_with_metrics(R, name, method):
    ctx = _ctx(R, 1)
    c = CS.case(name)
    g = run_path(R, ctx, c)
    meth = R.RN_CG if method == "cg" else R.RN_GMRES
    P, st, _ = ctx.energy_min(g["plan"], g["A"].vals, g["T"], meth, c["iters"], R.RN_FP64)
    E, r, ny = _oracle_metrics(c, c["P"])
    assert abs(st.energy - E) <= 1e-11 * abs(E)
    assert abs(st.proj_residual - r) <= 1e-11 * ny + 1e-9 * r
    assert st.constraint_residual <= 1e-13
    if method == "gmres":  # the Givens estimate of the last step is ||Pi(A P)||
        assert abs(st.last - st.proj_residual) <= 1e-8 * st.proj_residual + 1e-13 * ny
    A = c["A"]
    wu = (st.iters_done + 2) * st.spgemm_flops / (2.0 * A.nnz)
    assert st.work_units == pytest.approx(wu, rel=1e-14)
    # without the option the metric fields are NaN and the work units count
    # the minimisation's products only
    ctx2 = _ctx(R, 0)
    g2 = run_path(R, ctx2, c)
    _, st2, _ = ctx2.energy_min(g2["plan"], g2["A"].vals, g2["T"], meth, c["iters"], R.RN_FP64)
    assert np.isnan(st2.energy) and np.isnan(st2.constraint_residual)
    assert st2.work_units == pytest.approx((st2.iters_done + 1) * st2.spgemm_flops / (2.0 * A.nnz), rel=1e-14)
    g["plan"].close()
    g2["plan"].close()
    ctx.close()
    ctx2.close()


def test_setup_constraint_residual_against_B(R):
    ctx = _ctx(R, 1)
    c = CS.case("elastic32")
    s = ctx.setup_native(dev_matrix(R, c), dev(c["B"]), dev(c["agg"]), dev(c["roots"]), c["theta"], c["degree"],
                         c["iters"], R.RN_CG, R.RN_FP64)
    P = host(s.tensor("P"))
    Bc = host(s.tensor("Bc")).reshape(-1, c["B"].shape[1])
    ref = O.constraint_residual(c["Np"], c["Nj"], P, Bc, c["B"])
    assert s.stats.constraint_residual == ref
    s.close()
    ctx.close()
