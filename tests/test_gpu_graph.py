"""GPU: the captured V-cycle graph against eager launches, and determinism.

The library replays one HIP graph per V-cycle.  Each replay must equal the
eager V-cycle bitwise (same kernels in the same order, fixed reduction
orders, no atomics), also when eager work and synchronisations run between
replays; repeated runs must be bitwise identical.
"""
import os

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


def _solver(wl, graph, precision="fp64"):
    from paper_1612_02208_amd import StokesIB
    old = os.environ.get("IBMG_GRAPH")
    os.environ["IBMG_GRAPH"] = "1" if graph else "0"
    try:
        return StokesIB(wl, precision=precision)
    finally:
        if old is None:
            del os.environ["IBMG_GRAPH"]
        else:
            os.environ["IBMG_GRAPH"] = old


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("which", ["plain_32", "annulus_64"])
def test_graph_replays_equal_eager(which, precision):
    if which == "plain_32":
        wl = W.plain_32()
    else:
        X, S = W.annulus(4, 150, 0.2, 0.25)
        wl = W.Workload("annulus_64", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4))
    print(f"[case] graph {which} {precision}", flush=True)
    ge = _solver(wl, graph=False, precision=precision)
    gg = _solver(wl, graph=True, precision=precision)
    rng = np.random.default_rng(0)
    n = 3 * wl.N * wl.N
    for rep in range(4):
        r = torch.from_numpy(rng.uniform(-1, 1, n)).cuda()
        ze = ge.vcycle(r)
        torch.cuda.synchronize()
        zg = gg.vcycle(r)
        # eager work on the same stream between replays
        _ = ge.apply(zg)
        torch.cuda.synchronize()
        assert torch.equal(ze, zg), (rep, float((ze - zg).abs().max()))
    ge.close()
    gg.close()


def test_solve_is_deterministic():
    wl = W.plain_32()
    g = _solver(wl, graph=True)
    b = torch.from_numpy(W.rhs(wl.N, 3)).cuda()
    x1, i1 = g.solve(b, rtol=1e-10)
    x2, i2 = g.solve(b, rtol=1e-10)
    torch.cuda.synchronize()
    assert torch.equal(x1, x2) and i1["history"] == i2["history"]
    g.close()
