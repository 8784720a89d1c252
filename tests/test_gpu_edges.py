"""GPU parity on the degenerate and boundary cases of the method: no
structure at all, points without springs, springs of zero stiffness, points
on grid lines and at the edges of the periodic square with springs across
it, and the smallest hierarchies (two levels, 8 over 4) with the
Schur-complement and multiplicative smoothers.  Every call is compared with
the oracle on the same inputs: the operator on every level, the smoother,
one V-cycle, the solve, and spreading / interpolation where there are
points; and the FP32-smoother form reaches the tolerance."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ib as oib
from oracle.solver import Problem
from _parity import assert_classes, face_classes, level_classes

pytestmark = pytest.mark.gpu

OPS_TOL = 1e-12
SOLVE_TOL = 1e-10


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _mk(name, N, coarse, X, S, kap, rho=1.0, mu=0.1, dt=1e-2, **kw):
    return W.Workload(name, N, coarse, rho, mu, dt, np.asarray(X, dtype=np.float64),
                      np.asarray(S, dtype=np.int32).reshape(-1, 2), np.asarray(kap, dtype=np.float64), **kw)


def _cases():
    out = [_mk("no_structure_16", 16, 4, np.zeros((0, 2)), np.zeros((0, 2)), np.zeros(0), box=4, overlap=1)]
    rng = np.random.default_rng(9)
    out.append(_mk("points_no_springs_32", 32, 8, rng.uniform(0, 1, (50, 2)), np.zeros((0, 2)), np.zeros(0)))
    X, S = W.membrane(64, 0.3)
    out.append(_mk("kappa_zero_32", 32, 8, X, S, np.zeros(64), rho=0.0, mu=1.0))
    # a point at the origin, one a hair below x = 1 and one below y = 1, one
    # on grid lines, two near opposite corners, springs across both edges
    Xb = [[0.0, 0.0], [0.5, 0.25], [1 - 1e-12, 0.5], [0.25, 1 - 1e-9], [3 / 32, 5 / 32], [0.999, 0.001],
          [0.001, 0.999]]
    Sb = [[0, 1], [1, 2], [2, 3], [3, 4], [5, 6], [6, 0], [5, 0]]
    out.append(_mk("boundary_points_32", 32, 8, Xb, Sb, np.full(len(Sb), 50.0), rho=0.0, mu=1.0))
    X8, S8 = W.membrane(16, 0.3)
    out.append(_mk("two_levels_8_sc", 8, 4, X8, S8, np.full(16, 10.0), rho=0.0, mu=1.0, smoother="sc", box=2,
                   overlap=1))
    out.append(_mk("two_levels_8_rms", 8, 4, X8, S8, np.full(16, 10.0), smoother="rms", box=2, overlap=1))
    return out


CASES = _cases()


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c.name for c in CASES])
def pair(request):
    from paper_1612_02208_amd import StokesIB
    wl = CASES[request.param]
    print(f"[case] {wl.name} N={wl.N} M={wl.M}", flush=True)
    P = Problem(wl)
    G = StokesIB(wl)
    yield wl, P, G
    G.close()


def test_operator_every_level(pair):
    wl, P, G = pair
    rng = np.random.default_rng(1)
    for l, lev in enumerate(P.levels):
        w = rng.uniform(-1, 1, lev.n)
        cl = level_classes(lev.N, lev.T)
        assert_classes(host(G.apply(dev(w), level=l)), lev.L @ w, cl, OPS_TOL, f"apply {l}")
        assert_classes(host(G.apply(dev(w), level=l, transpose=True)), lev.L.T @ w, cl, OPS_TOL, f"apply_T {l}")


def test_smoother_vcycle_and_solve(pair):
    wl, P, G = pair
    rng = np.random.default_rng(2)
    r = rng.uniform(-1, 1, P.levels[-1].n)
    cl = level_classes(P.fine.N, P.fine.T)
    assert_classes(host(G.smoother_apply(-1, dev(r))), P.mg.smoothers[-1](r), cl, SOLVE_TOL, "smoother")
    assert_classes(host(G.vcycle(dev(r))), P.mg.vcycle(r), cl, SOLVE_TOL, "V-cycle")
    b = W.rhs(wl.N, 1)
    x, info = G.solve(dev(b), rtol=1e-12, max_it=100)
    xo, io = P.solve(b, rtol=1e-12, max_it=100)
    assert info["converged"] and io["converged"]
    assert abs(info["iters"] - io["iters"]) <= 1
    assert_classes(host(x), xo, cl, SOLVE_TOL, "solve at 1e-12")


def test_spread_and_interp(pair):
    wl, P, G = pair
    if wl.M == 0:
        pytest.skip("no points")
    N = wl.N
    rng = np.random.default_rng(3)
    F = rng.uniform(-1, 1, (wl.M, 2))
    f = host(G.spread(dev(F.ravel())))
    touched = np.concatenate([np.asarray(oib.interp_pattern(wl.X, N, c).sum(0)).ravel() > 0 for c in (0, 1)])
    assert_classes(f, np.concatenate([oib.spread_matrix(wl.X, N, c) @ F[:, c] for c in (0, 1)]),
                   face_classes(N, touched), OPS_TOL, "spread")
    u = rng.uniform(-1, 1, 2 * N * N)
    U = host(G.interp(dev(u))).reshape(-1, 2)
    for c in (0, 1):
        assert rel(U[:, c], oib.interp_matrix(wl.X, N, c) @ u[c * N * N:(c + 1) * N * N]) < OPS_TOL


def test_fp32_smoother_reaches_tolerance(pair):
    from paper_1612_02208_amd import StokesIB
    wl, P, G = pair
    b = W.rhs(wl.N, 4)
    G32 = StokesIB(wl, precision="fp32")
    x, info = G32.solve(dev(b), rtol=1e-8)
    G32.close()
    assert info["converged"] and info["rel_res_true"] <= 1.2e-8
    xo, _ = P.solve(b, rtol=1e-12, max_it=100)
    assert_classes(host(x), xo, level_classes(P.fine.N, P.fine.T), 1e-5, "fp32 solve at 1e-8 vs oracle at 1e-12")
