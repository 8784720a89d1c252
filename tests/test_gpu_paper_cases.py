"""GPU parity on the results section's test structures (Sec. 5.1 thick shell,
Sec. 5.2 thin membrane) at N = 64 with dt = 0.32 h: the right-hand side of
one semi-implicit step from the background flow, and its solve to a 1e-12
residual reduction, against the oracle's, for each smoother family."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import Problem
from oracle.timestep import step_rhs
from _parity import assert_classes, level_classes

pytestmark = pytest.mark.gpu

CASES = [("thick", 64, 50.0, "mu0.1", "ras", 8, 2),
         ("thick", 64, 500.0, "stokes", "rms", 8, 2),
         ("thin", 64, 5.0, "mu1", "ras", 16, 4),
         ("thin", 64, 5.0, "stokes", "sc", 8, 2),
         ("thick", 64, 5.0, "mu0.01", "sc", 8, 2)]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("case", CASES, ids=[W.paper_case(*c).name for c in CASES])
def test_paper_case_step_solve(case):
    from paper_1612_02208_amd import StokesIB
    wl = W.paper_case(*case)
    print(f"[case] {wl.name}", flush=True)
    u = W.background_flow(wl.N)
    b = step_rhs(wl, u)
    P = Problem(wl)
    x, info = P.solve(b, rtol=1e-12, max_it=100)
    assert info["converged"]
    G = StokesIB(wl)
    bg = G.step_rhs(torch.from_numpy(u).cuda())
    torch.cuda.synchronize()
    cl = level_classes(P.fine.N, P.fine.T)
    assert_classes(bg.cpu().numpy(), b, cl, 1e-12, "step rhs")
    xg, ginfo = G.solve(bg, rtol=1e-12, max_it=100)
    xg = xg.cpu().numpy()
    G.close()
    assert ginfo["converged"], ginfo
    assert abs(ginfo["iters"] - info["iters"]) <= 1, (ginfo["iters"], info["iters"])
    # the GPU solution's true residual under the oracle's operator
    bp = P.project(b)
    assert np.linalg.norm(bp - P.apply(xg)) <= 2e-12 * np.linalg.norm(bp)
    assert_classes(xg, x, cl, 1e-10, "solve at 1e-12")
