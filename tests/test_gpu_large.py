"""GPU parity at a grid size where the stencil kernels march several rows per
thread (N >= 2048): the finest-level operator, its transpose and the
residual against the oracle's assembled L_IB (App. A.1, Eq. matrix-impib)
on the whole vector, and a full solve (which runs the fused operator and
dot-product kernel in the smoother and the outer FGMRES) checked through its
true residual under the oracle's operator."""
import numpy as np
import pytest
import torch

import workloads as W
from _parity import assert_classes, level_classes
from oracle import ib as oib
from oracle import mac

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def large():
    from paper_1612_02208_amd import StokesIB
    N = 2048
    X, S = W.membrane(1024, 0.21, centre=(0.43, 0.57))
    wl = W.Workload("membrane_2048", N, 8, 1.0, 1e-2, 2e-4, X, S, np.full(len(S), 1e3), box=8, overlap=2)
    print(f"[case] {wl.name} N={N} M={wl.M}", flush=True)
    A = mac.momentum(N, wl.rho, wl.mu, wl.dt) + oib.ib_term(X, S, wl.kappa, N, wl.dt)
    L = mac.stokes_ib(A.tocsr(), mac.gradient(N), mac.divergence(N)).tocsr()
    cl = level_classes(N, oib.ib_term(X, S, wl.kappa, N, wl.dt))
    G = StokesIB(wl)
    yield wl, L, G, cl
    G.close()


def test_operator_transpose_and_residual(large):
    wl, L, G, cl = large
    w = np.random.default_rng(21).uniform(-1, 1, L.shape[0])
    y = host(G.apply(dev(w)))
    assert_classes(y, L @ w, cl, 1e-12, "apply")
    yt = host(G.apply(dev(w), transpose=True))
    assert_classes(yt, L.T @ w, cl, 1e-12, "apply_T")


def test_solve_true_residual(large):
    wl, L, G, cl = large
    b = W.rhs(wl.N, 3)
    x, info = G.solve(dev(b), rtol=1e-8)
    assert info["converged"], info
    xh = host(x)
    # the library projects b onto range(L_IB): block means of p (rho > 0)
    n = wl.N * wl.N
    bp = b.copy()
    bp[2 * n:] -= bp[2 * n:].mean()
    true = np.linalg.norm(bp - L @ xh) / np.linalg.norm(bp)
    assert true <= 1.2e-8, true
    assert abs(info["rel_res_true"] - true) < 1e-10
