"""How far apart two correct FP64 evaluations of the elasticity energy
minimisation land (Sec. 3.6 improve, Sec. 4.1; reading R9 for the least
squares of the projection).

On the node-blocked elasticity workload (three rigid-body candidates, one side
clamped, 512 x 512 nodes, 6 CG steps) the CG iterate is sensitive to rounding:
the projection's per-row least squares have cond(B_J) ~ 1e5, and the first
step lengths amplify any difference.  The CG recurrence is driven here from the
oracle's own masked product and projection, evaluated three ways that are each
correct to FP64 rounding: (a) the oracle's Householder least squares with the
inner products summed pairwise instead of compensated, (b) the least squares
through the normal equations (G = B_J^T B_J, pseudo-inverse with the 1e-12
cutoff), (c) the first step length moved by one ulp.  The spread of these
bounds how closely any other correct FP64 implementation can follow the
oracle, and the GPU parity bar for the elasticity cases is derived from it.
"""
import numpy as np
import pytest

import oracle as O
from tests import cases as CS


def _driver(c, Gp, dot):
    A = c["A"]
    Np, Nj, nc = c["Np"], c["Nj"], c["nc"]
    isr = np.ascontiguousarray(c["is_root"], np.uint8)
    Bc = np.ascontiguousarray(c["Bc"]).ravel()
    nB = c["Bc"].shape[1]
    L = O.lib()

    def Pi(X):
        X = np.ascontiguousarray(X, np.float64).copy()
        L.orc_project(Np.size - 1, Np, Nj, isr, Bc, nB, Gp, X)
        return X

    def AX(X):
        return O.masked_product(A.rowptr, A.colind, A.vals, Np, Nj, nc, X)

    def run(K, bump_alpha0=False):
        P = c["T"].copy()
        R = -Pi(AX(P))
        D = R.copy()
        g = dot(R, R)
        for k in range(K):
            Z = Pi(AX(D))
            al = g / dot(D, Z)
            if bump_alpha0 and k == 0:
                al = np.nextafter(al, np.inf)
            P = P + al * D
            R = R - al * Z
            gn = dot(R, R)
            be = gn / g
            g = gn
            D = R + be * D
        return P

    return run


def _normal_equation_pinv(c):
    Np, Nj = c["Np"], c["Nj"]
    Bcm = np.ascontiguousarray(c["Bc"])
    n = Np.size - 1
    BJ = Bcm[Nj]
    G = np.add.reduceat(BJ[:, :, None] * BJ[:, None, :], Np[:-1], axis=0)
    Gn = np.linalg.pinv(G, rcond=1e-12, hermitian=True)
    Gn[np.asarray(c["is_root"], bool)] = 0.0
    return np.ascontiguousarray(Gn.reshape(n, -1)).ravel()


@pytest.mark.slow
def test_elastic512_spread_of_correct_fp64_evaluations():
    c = CS.case("elastic512")
    K = c["iters"]
    Gq, _ = O.gram_rows(c["Np"], c["Nj"], c["is_root"], c["Bc"], c["Bc"].shape[1])
    scale = float(np.max(np.abs(c["P"])))

    def shift(P):
        return float(np.max(np.abs(P - c["P"]))) / scale

    pairwise = lambda x, y: float(np.sum(x * y))
    s_pair = shift(_driver(c, Gq, pairwise)(K))
    s_normal = shift(_driver(c, _normal_equation_pinv(c), pairwise)(K))
    s_ulp = shift(_driver(c, Gq, pairwise)(K, bump_alpha0=True))
    spread = max(s_pair, s_normal, s_ulp)
    print(f"elastic512 FP64 spread: pairwise dots {s_pair:.3e}, normal equations {s_normal:.3e}, "
          f"alpha_0 + 1 ulp {s_ulp:.3e}; bar {CS.ELASTIC_FP64_TOL:.1e}")
    # 1e-12 is out of reach for any other correct FP64 evaluation ...
    assert s_pair > 2e-12 and s_normal > 2e-12 and s_ulp > 2e-12
    # ... and the elasticity bar sits within a small multiple of the spread
    assert 1.5 * spread <= CS.ELASTIC_FP64_TOL <= 10 * spread


@pytest.mark.slow
def test_elastic512_prefiltered_spread_of_correct_fp64_evaluations():
    """The same measurement on the pattern pre-filtered with theta_f = 0.2
    (Sec. 3.5), where two rows become rank-deficient: the least squares of
    those rows (pseudo-inverse through the cutoff) differ between the
    Householder and normal-equation evaluations."""
    c0 = CS.case("elastic512")
    A = c0["A"]
    st = O.prefilter_setup(A, c0["B"], 2, c0["theta"], 2, theta_f=0.2, agg=c0["agg"], roots=c0["roots"])
    K = c0["iters"]
    P, info = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"], st["Bc"], 3,
                        st["T"], K)
    c = dict(A=A, Np=st["Np"], Nj=st["Nj"], nc=st["nc"], is_root=st["is_root"], Bc=st["Bc"], T=st["T"], P=P)
    Gq, rd = O.gram_rows(c["Np"], c["Nj"], c["is_root"], c["Bc"], 3)
    assert rd == 2
    scale = float(np.max(np.abs(P)))
    shift = lambda Q: float(np.max(np.abs(Q - P))) / scale
    pairwise = lambda x, y: float(np.sum(x * y))
    s_pair = shift(_driver(c, Gq, pairwise)(K))
    s_normal = shift(_driver(c, _normal_equation_pinv(c), pairwise)(K))
    s_ulp = shift(_driver(c, Gq, pairwise)(K, bump_alpha0=True))
    spread = max(s_pair, s_normal, s_ulp)
    print(f"pre-filtered elastic512 FP64 spread: pairwise {s_pair:.3e}, normal equations {s_normal:.3e}, "
          f"alpha_0 + 1 ulp {s_ulp:.3e}; bar {CS.ELASTIC_PREFILTER_FP64_TOL:.1e}")
    assert 1.5 * spread <= CS.ELASTIC_PREFILTER_FP64_TOL <= 10 * spread
