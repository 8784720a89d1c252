"""GPU tests of the batched form (many independent systems, one persistent
Schwarz launch per sweep across all of them).

The batch runs the same method as the single-system path with different
reduction trees, so it is compared with the oracle (small systems) and with
the single-system library path to the solve tolerance; the 64-system
workload is checked by properties that hold at any size (every system's true
residual, evaluated with the oracle's assembled operator on sampled systems).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import hierarchy, mac
from oracle import ib as oib
from oracle.solver import Problem
from _parity import assert_classes, level_classes

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-10


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def classes_of(wl):
    return level_classes(wl.N, oib.ib_term(wl.X, wl.springs, wl.kappa, wl.N, wl.dt))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _mixed(rho=0.0, mu=1.0, dt=1e-3):
    """Five systems of two grid sizes, given out of size order, with
    different membranes (radius, centre, point count) and stiffnesses."""
    specs = [(32, 0.25, 1e2, (0.5, 0.5)), (64, 0.2, 1e4, (0.4, 0.55)), (32, 0.18, 3e3, (0.6, 0.45)),
             (64, 0.27, 50.0, (0.5, 0.5)), (64, 0.12, 1e5, (0.3, 0.7))]
    out = []
    for i, (N, r, k, c) in enumerate(specs):
        X, S = W.membrane(4 * N - 3 * i, r, centre=c)
        out.append(W.Workload(f"mix_{i}", N, 8, rho, mu, dt, X, S, np.full(len(S), k), rhs_seed=100 + i))
    return out


CONFIGS = {"stokes": dict(), "reynolds": dict(rho=1.0, mu=1e-2, dt=5e-4)}


@pytest.fixture(scope="module", params=list(CONFIGS), ids=list(CONFIGS))
def mixed(request):
    from paper_1612_02208_amd import StokesIB, StokesIBBatch
    systems = _mixed(**CONFIGS[request.param])
    print(f"[case] batch {request.param} sizes={[s.N for s in systems]}", flush=True)
    B = StokesIBBatch(systems, precision="fp64")
    singles = [StokesIB(s, precision="fp64") for s in systems]
    yield systems, B, singles
    B.close()
    for G in singles:
        G.close()


def test_batch_vcycle_matches_single_and_oracle(mixed):
    systems, B, singles = mixed
    P0 = Problem(systems[0])
    rs = []
    for i, s in enumerate(systems):
        r = W.rhs(s.N, 11 + i)
        if i == 0:
            r = P0.project(r)
        rs.append(dev(r))
    zs = B.vcycle(rs)
    for i, G in enumerate(singles):
        z1 = host(G.vcycle(rs[i]))
        assert_classes(host(zs[i]), z1, classes_of(systems[i]), SOLVE_TOL, f"batch V-cycle system {i}")
    assert_classes(host(zs[0]), P0.mg.vcycle(host(rs[0])), level_classes(P0.fine.N, P0.fine.T), SOLVE_TOL,
                   "batch V-cycle vs oracle")


def test_batch_solve_matches_single(mixed):
    systems, B, singles = mixed
    bs = [dev(W.rhs(s.N, s.rhs_seed)) for s in systems]
    xs, info = B.solve(bs, rtol=1e-8)
    assert info["converged"]
    for i, G in enumerate(singles):
        x1, i1 = G.solve(bs[i], rtol=1e-8)
        si = info["systems"][i]
        assert abs(si["iters"] - i1["iters"]) <= 1, (i, si["iters"], i1["iters"])
        assert si["rel_res_true"] <= 1.2e-8
        assert abs(si["rhs_null_norm"] - i1["rhs_null_norm"]) <= 1e-12 * max(1.0, i1["rhs_null_norm"])
    # both to 1e-12: the solutions agree to the conditioning of the systems
    xs12, info12 = B.solve(bs, rtol=1e-12, max_it=200)
    assert info12["converged"]
    for i, G in enumerate(singles):
        x1, _ = G.solve(bs[i], rtol=1e-12, max_it=200)
        assert_classes(host(xs12[i]), host(x1), classes_of(systems[i]), SOLVE_TOL, f"system {i} at 1e-12")


def test_batch_solution_against_oracle(mixed):
    systems, B, singles = mixed
    bs = [dev(W.rhs(s.N, s.rhs_seed)) for s in systems]
    xs, info = B.solve(bs, rtol=1e-12, max_it=200)
    for i in (0, 1):
        P = Problem(systems[i])
        b = W.rhs(systems[i].N, systems[i].rhs_seed)
        xo, _ = P.solve(b, rtol=1e-12, max_it=200)
        assert_classes(host(xs[i]), xo, level_classes(P.fine.N, P.fine.T), SOLVE_TOL, f"system {i} vs oracle")
        bp = P.project(b)
        assert np.linalg.norm(bp - P.L @ host(xs[i])) <= 1.2e-12 * np.linalg.norm(bp)


def test_batch_deterministic(mixed):
    systems, B, singles = mixed
    bs = [dev(W.rhs(s.N, 7)) for s in systems]
    xa, ia = B.solve(bs, rtol=1e-8)
    xb, ib = B.solve(bs, rtol=1e-8)
    for a, b in zip(xa, xb):
        assert torch.equal(a, b)
    assert [s["iters"] for s in ia["systems"]] == [s["iters"] for s in ib["systems"]]


def test_batch_fp32_smoother():
    from paper_1612_02208_amd import StokesIBBatch
    systems = _mixed()
    B32 = StokesIBBatch(systems, precision="fp32")
    B64 = StokesIBBatch(systems, precision="fp64")
    bs = [dev(W.rhs(s.N, s.rhs_seed)) for s in systems]
    x32, i32 = B32.solve(bs, rtol=1e-8)
    x64, i64 = B64.solve(bs, rtol=1e-8)
    assert i32["converged"] and i64["converged"]
    for i, s in enumerate(systems):
        assert i32["systems"][i]["rel_res_true"] <= 1.2e-8
        # both solutions are within cond * 1e-8 of the exact one
        assert_classes(host(x32[i]), host(x64[i]), classes_of(s), 1e-5, f"system {i} fp32 vs fp64")
    P = Problem(systems[3])
    b = W.rhs(systems[3].N, systems[3].rhs_seed)
    bp = P.project(b)
    assert np.linalg.norm(bp - P.L @ host(x32[3])) <= 1.2e-8 * np.linalg.norm(bp)
    B32.close()
    B64.close()


def test_batch_64_systems():
    """The batching workload: 64 systems, N in {64, 128, 256}, FP32 smoother,
    every system to 1e-8, and every system's solution checked by its true
    residual under the oracle's operator (App. A.1 assembled as a sparse
    matrix, without the oracle's hierarchy)."""
    from paper_1612_02208_amd import StokesIBBatch
    systems = W.batch_systems(64)
    B = StokesIBBatch(systems, precision="fp32")
    st = B.stats()
    assert st["nsys"] == 64
    for lv in st["levels"][1:]:
        assert lv["tile"] in (16, 32, 64) and lv["grid"] >= 1
    bs = [dev(W.rhs(s.N, s.rhs_seed)) for s in systems]
    xs, info = B.solve(bs, rtol=1e-8)
    assert info["converged"]
    for i, si in enumerate(info["systems"]):
        assert si["rel_res_true"] <= 1.2e-8, (i, si)
        assert si["iters"] <= 30
    for i, s in enumerate(systems):
        N = s.N
        A = mac.momentum(N, s.rho, s.mu, s.dt) + oib.ib_term(s.X, s.springs, s.kappa, N, s.dt)
        L = mac.stokes_ib(A.tocsr(), mac.gradient(N), mac.divergence(N)).tocsr()
        bp = hierarchy.project_range(W.rhs(N, s.rhs_seed), N, s.rho)
        assert np.linalg.norm(bp - L @ host(xs[i])) <= 1.2e-8 * np.linalg.norm(bp), i
    B.close()
