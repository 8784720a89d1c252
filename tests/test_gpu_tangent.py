"""GPU tests of the tangent spring model (springs with rest lengths, the 2x2
blocks of the linearised force coupling u and v; Sec. 5 fibre model, Sec. 6):
the FP32-smoother form against the FP64 oracle, two semi-implicit steps
against the oracle's (the right-hand side uses the nonlinear force and the
operator is rebuilt at the moved structure), and Laplace's law for a
membrane held at a rest-length tension at a size the oracle is not run on.
The per-call parity (operators on every level, smoothers, V-cycle, FGMRES,
gradient) runs in the main parity file's tangent cases."""
import copy

import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import Problem
from oracle import ib as oib
from oracle.timestep import step_rhs, time_step
from _parity import assert_classes, level_classes


def classes_at(wl):
    # the rows that carry an IB term are the same for both spring models
    return level_classes(wl.N, oib.ib_term(wl.X, wl.springs, wl.kappa, wl.N, wl.dt))

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lengths(X, S):
    d = X[S[:, 1]] - X[S[:, 0]]
    d -= np.round(d)
    return np.hypot(d[:, 0], d[:, 1])


def _annulus():
    X, S = W.annulus(4, 150, 0.2, 0.25)
    return W.Workload("annulus_64_tangent", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4),
                      spring_model="tangent", rest=0.7 * lengths(X, S))


def _ellipse(smoother):
    M = 128
    th = 2 * np.pi * np.arange(M) / M
    X = np.stack([0.5 + 0.3 * np.cos(th), 0.5 + 0.2 * np.sin(th)], 1)
    S = np.stack([np.arange(M), (np.arange(M) + 1) % M], 1).astype(np.int32)
    # rest length: the mean spacing of a circle of the ellipse's area
    rest = np.full(M, 2 * np.pi * np.sqrt(0.3 * 0.2) / M * 0.9)
    return W.Workload(f"ellipse_32_tangent_{smoother}", 32, 8, 1.0, 0.1, 2e-3, X, S, np.full(M, 3e2),
                      smoother=smoother, spring_model="tangent", rest=rest)


def test_fp32_smoother_form():
    from paper_1612_02208_amd import StokesIB
    wl = _annulus()
    print(f"[case] fp32 {wl.name}", flush=True)
    P = Problem(wl)
    b = W.rhs(wl.N, 0)
    xo, _ = P.solve(b, rtol=1e-12, max_it=200)
    G = StokesIB(wl, precision="fp32")
    x, info = G.solve(dev(b), rtol=1e-8)
    G.close()
    assert info["converged"] and info["rel_res_true"] <= 1.2e-8
    # FP32 smoothing changes the iterates, not the accuracy of the result
    assert_classes(host(x), xo, level_classes(P.fine.N, P.fine.T), 1e-5, "fp32 at 1e-8 vs oracle at 1e-12")


@pytest.mark.parametrize("smoother", ["ras", "rms", "sc"])
def test_two_tangent_steps_match_oracle(smoother):
    from paper_1612_02208_amd import StokesIB
    wl = _ellipse(smoother)
    print(f"[case] two steps {wl.name}", flush=True)
    G = StokesIB(copy.deepcopy(wl))
    ow = copy.deepcopy(wl)
    w = 0.1 * np.random.default_rng(4).uniform(-1, 1, 3 * wl.N * wl.N)
    assert_classes(host(G.step_rhs(dev(w))), step_rhs(ow, w), classes_at(ow), 1e-12, "step rhs")
    wg = dev(w)
    for k in range(2):
        wg, info = G.time_step(wg, rtol=1e-12, max_it=200)
        assert info["converged"], (k, info)
        cl = classes_at(ow)
        w, Xn, _ = time_step(ow, w, rtol=1e-12)
        ow.X = Xn
        assert_classes(host(wg), w, cl, 1e-10, f"step {k}")
        assert np.abs(G.positions() - Xn).max() < 1e-12, k
    G.close()


def test_laplace_law_with_rest_length_on_the_gpu():
    """Pressure jump kappa (l - L) M sin(pi/M) / (pi R) across a circular
    membrane of springs at length l > L (Stokes flow), at N = 128."""
    from paper_1612_02208_amd import StokesIB
    N, M, R, kap = 128, 512, 0.25, 1e2
    X, S = W.membrane(M, R)
    l = 2 * R * np.sin(np.pi / M)
    wl = W.Workload("laplace_rest_128", N, 8, 0.0, 1.0, 1e-3, X, S, np.full(M, kap), spring_model="tangent",
                    rest=np.full(M, 0.5 * l))
    G = StokesIB(wl)
    w, info = G.time_step(dev(np.zeros(3 * N * N)), rtol=1e-10)
    assert info["converged"]
    p = host(w)[2 * N * N:].reshape(N, N)
    c = N // 2
    dp = p[c - 1:c + 1, c - 1:c + 1].mean() - p[0:2, 0:2].mean()
    exact = kap * 0.5 * l * M * np.sin(np.pi / M) / (np.pi * R)
    assert abs(dp / exact - 1) < 1e-4
    assert np.abs(host(w)[:2 * N * N]).max() < 1e-3 * exact
    G.close()


def test_batch_rejects_tangent_springs():
    from paper_1612_02208_amd import IbmgError, StokesIBBatch
    with pytest.raises(IbmgError):
        StokesIBBatch([_ellipse("ras"), _ellipse("ras")])
