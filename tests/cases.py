"""Seeded parity cases: inputs from workloads/, expected values from oracle/.

Each case is a named configuration (at full or reduced size) with the
oracle's strength graph, aggregation, pattern, tentative operator and
energy-minimised P (and R^T for non-symmetric A).  Results are cached per
process so several tests can share one oracle run.
"""
from __future__ import annotations

import functools
import math

import numpy as np

import oracle as O
import workloads as W

# name -> (builder, theta, degree, iters, method, m)
CASES = {
    "laplace1d_8": (lambda: (W.laplace1d(8), W.ones(8), None, None), 0.0, 2, 3, "cg", 1),
    "poisson32": (lambda: (W.poisson5(32), W.ones(1024), None, None), 0.25, 2, 4, "cg", 1),
    "poisson37": (lambda: (W.poisson5(37), W.ones(37 * 37), None, None), 0.25, 2, 5, "cg", 1),
    "aniso40": (lambda: (W.q1_aniso(40), W.ones(1600), None, None), 0.1, 2, 6, "cg", 1),
    "aniso512": (lambda: (W.q1_aniso(512), W.ones(512 * 512), None, None), 0.1, 2, 6, "cg", 1),
    "upwind64": (lambda: (W.upwind_cd(64), W.ones(4096), W.ones(4096), None), 0.0, 2, 8, "gmres", 1),
    "upwind1024": (lambda: (W.upwind_cd(1024), W.ones(1 << 20), W.ones(1 << 20), None), 0.0, 2, 8, "gmres", 1),
    "elastic7": None,
    "elastic32": None,
    "elastic512": None,
    "twocand13": None,
    # 3D 27-point: rows of 27 A entries (the product's generic term loop) and
    # pattern rows gathering more than 64 candidates (the expansion's
    # large-window kernel)
    "lap27_10": (lambda: (W.laplace27(10), W.ones(1000), None, None), 0.0, 2, 4, "cg", 1),
    # irregular structure: neighbour rows far apart in the numbering, so no
    # product block gets an X window (the persistent product reads X from
    # global memory)
    "ring20k": (lambda: (W.ring_graph(20000), W.ones(20000), None, None), 0.0, 1, 4, "cg", 1),
    # structurally non-symmetric stencil (entries at (+1,+1) and (0,-1) with no mirror): the
    # strength symmetrises through an explicit transpose
    "asym20": (lambda: (W.stencil_grid(20, 20, {(0, 0): 4.0, (-1, 0): -1.0, (1, 0): -0.5, (0, -1): -1.0,
                                                (1, 1): -0.6}), W.ones(400), W.ones(400), None),
               0.25, 2, 4, "gmres", 1),
}


def _elastic(nx):
    Ab, xy = W.q1_elasticity(nx)
    return Ab.to_csr(), W.rbm(xy), None, Ab


def _twocand(nx):
    A = W.poisson5(nx)
    n = nx * nx
    x = (np.arange(n) % nx) / nx
    y = (np.arange(n) // nx) / nx
    return A, np.stack([np.ones(n), x, y], 1), None, None


CASES["elastic7"] = (lambda: _elastic(7), 0.0, 2, 6, "cg", 2)
CASES["elastic32"] = (lambda: _elastic(32), 0.0, 2, 6, "cg", 2)
CASES["elastic512"] = (lambda: _elastic(512), 0.0, 2, 6, "cg", 2)
CASES["twocand13"] = (lambda: _twocand(13), 0.0, 3, 5, "cg", 1)
# theta > 0 on the node-blocked operator: blocks mix strong and weak DOF
# entries, so the amalgamation rule decides which node pairs are strong
CASES["elastic7_t03"] = (lambda: _elastic(7), 0.3, 2, 6, "cg", 2)
CASES["elastic32_t03"] = (lambda: _elastic(32), 0.3, 2, 6, "cg", 2)


# FP64 parity bar of the node-blocked elasticity cases, max|dP| / max|P|.
# Two correct FP64 evaluations of the 512 x 512 elasticity minimisation (the
# oracle's Householder least squares with pairwise instead of compensated
# inner products; the least squares through the normal equations; the first
# step length moved by one ulp) land 1.3e-11 to 5.3e-11 from the oracle
# (tests/test_fp64_spread.py measures it): 1e-12 is out of reach, and the
# bar is twice the largest of these.
ELASTIC_FP64_TOL = 1e-10
# The same bar for the elasticity minimisation on the pattern pre-filtered
# with theta_f = 0.2 (Sec. 3.5): there two rows keep too few columns for all
# three candidates, and the correct evaluations spread up to 1.4e-10
# (tests/test_fp64_spread.py): twice the largest, rounded up.
ELASTIC_PREFILTER_FP64_TOL = 3e-10


@functools.lru_cache(maxsize=None)
def case(name: str) -> dict:
    build, theta, degree, iters, method, m = CASES[name]
    A, B, Bhat, Ab = build()
    st = O.setup(A, B, m, theta, degree)
    out = dict(name=name, A=A, Ab=Ab, B=B, Bhat=Bhat, m=m, theta=theta, degree=degree, iters=iters,
               method=method, **st)
    nB = B.shape[1]
    if method == "cg":
        P, info = O.emin_cg(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"],
                            st["Bc"], nB, st["T"], iters)
    else:
        P, info = O.emin_gmres(A.rowptr, A.colind, A.vals, st["Np"], st["Nj"], st["is_root"], st["nc"],
                               st["Bc"], nB, st["T"], iters)
    out["P"], out["info"] = P, info
    if Bhat is not None:
        Tp, Tj, Tx = O.transpose(A.rowptr, A.colind, A.vals)
        That, Bch, _ = O.tentative(st["Np"], st["Nj"], st["is_root"], st["agg"], st["roots"], m, Bhat)
        RT, rinfo = O.emin_gmres(Tp, Tj, Tx, st["Np"], st["Nj"], st["is_root"], st["nc"], Bch, Bhat.shape[1],
                                 That, iters)
        out.update(AT=(Tp, Tj, Tx), That=That, Bch=Bch, RT=RT, rinfo=rinfo)
    return out


def rel_max(a, b) -> float:
    """max |a - b| / max |b| (the parity norm for P and R^T: max |P| = 1 through
    the root rows)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return float(np.max(np.abs(a - b))) / den if a.size else 0.0


def rel_close(a, b) -> float:
    return abs(a - b) / max(abs(b), 1e-300) if not (math.isnan(a) or math.isnan(b)) else math.inf
