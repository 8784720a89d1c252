"""Pins of the oracle's semi-implicit time step (Sec. 2.2 without
convection) against physics the scheme must reproduce:

* Laplace's law: a circular membrane of zero-rest-length springs in Stokes
  flow is held by a pressure jump equal to its discrete force density,
  2 kappa M sin^2(pi / M) / pi for M equally spaced nodes (tension over
  radius in the continuum limit), with the fluid nearly at rest; the error
  falls under refinement;
* incompressibility: an elliptical membrane relaxes toward a circle (its
  aspect ratio falls every step) while its enclosed area stays fixed;
* the spread force has zero total (springs exert equal and opposite forces,
  and the kernel sums to one);
* the periodic reading: a membrane straddling the domain's corner gives the
  same pressure jump as the same membrane centred (minimum-image spring
  separations).
"""
import numpy as np

import workloads as W
from oracle.timestep import advance_positions, step_rhs, time_step


def _circle(N, centre=(0.5, 0.5), R=0.25, kap=1e2):
    X, S = W.membrane(4 * N, R, centre=centre)
    return W.Workload("laplace", N, 8, 0.0, 1.0, 1e-3, X, S, np.full(len(S), kap))


def _jump(wl, centre):
    N = wl.N
    n = N * N
    x, Xn, info = time_step(wl, np.zeros(3 * n), rtol=1e-10)
    p = x[2 * n:].reshape(N, N)
    ci, cj = int(round(centre[0] * N)) % N, int(round(centre[1] * N)) % N
    oi, oj = (ci + N // 2) % N, (cj + N // 2) % N
    inside = np.mean([p[(cj + a) % N, (ci + b) % N] for a in (-1, 0) for b in (-1, 0)])
    outside = np.mean([p[(oj + a) % N, (oi + b) % N] for a in (-1, 0) for b in (-1, 0)])
    return inside - outside, x, Xn


def test_laplace_law_and_refinement():
    errs = []
    for N in (32, 64):
        wl = _circle(N)
        M = wl.X.shape[0]
        exact = 2 * 1e2 * M * np.sin(np.pi / M) ** 2 / np.pi
        dp, x, Xn = _jump(wl, (0.5, 0.5))
        errs.append(abs(dp / exact - 1))
        # the fluid is nearly at rest: the force is balanced by pressure
        umax = np.abs(x[:2 * N * N]).max()
        assert umax < 1e-2 * dp * 0.25 / 1.0
        assert np.abs(Xn - wl.X).max() < 1e-5
    assert errs[0] < 1e-3 and errs[1] < errs[0] / 2


def test_periodic_membrane_across_the_corner():
    N = 32
    dp0, _, _ = _jump(_circle(N), (0.5, 0.5))
    dp1, _, _ = _jump(_circle(N, centre=(0.0, 0.0)), (0.0, 0.0))
    assert abs(dp1 - dp0) <= 1e-9 * abs(dp0)


def test_spread_force_has_zero_total():
    wl = _circle(32, R=0.2)
    rhs = step_rhs(wl, np.zeros(3 * 32 * 32))
    n = 32 * 32
    for c in (0, 1):
        assert abs(rhs[c * n:(c + 1) * n].sum()) < 1e-10 * np.abs(rhs[c * n:(c + 1) * n]).max()


def test_ellipse_relaxes_at_fixed_area():
    N = 32
    M = 4 * N
    th = 2 * np.pi * np.arange(M) / M
    X = np.stack([0.5 + 0.3 * np.cos(th), 0.5 + 0.2 * np.sin(th)], 1)
    S = np.stack([np.arange(M), (np.arange(M) + 1) % M], 1).astype(np.int32)
    wl = W.Workload("ellipse", N, 8, 0.0, 1.0, 2e-3, X, S, np.full(M, 1e2))

    def area(Y):
        return 0.5 * abs(np.dot(Y[:, 0], np.roll(Y[:, 1], -1)) - np.dot(Y[:, 1], np.roll(Y[:, 0], -1)))

    def aspect(Y):
        d = Y - Y.mean(0)
        return np.abs(d[:, 0]).max() / np.abs(d[:, 1]).max()

    A0 = area(X)
    w = np.zeros(3 * N * N)
    prev = aspect(X)
    for _ in range(2):
        w, Xn, _ = time_step(wl, w, rtol=1e-10)
        assert aspect(Xn) < prev - 1e-4
        assert abs(area(Xn) / A0 - 1) < 1e-5
        prev = aspect(Xn)
        wl.X = Xn
    # advancing with a zero velocity leaves the structure in place
    assert np.array_equal(advance_positions(wl, np.zeros(3 * N * N)), wl.X)


def test_backward_euler_shear_decay():
    """Without stiffness, a divergence-free shear mode u = sin(2 pi y) decays
    in one step by the backward-Euler factor of its discrete Laplacian
    eigenvalue: u^{n+1} = u^n (rho/dt) / (rho/dt + mu (4/h^2) sin^2(pi h)),
    with the pressure constant."""
    N, rho, mu, dt = 32, 1.0, 0.1, 1e-2
    X, S = W.membrane(64, 0.25)
    wl = W.Workload("shear", N, 8, rho, mu, dt, X, S, np.zeros(len(S)))
    n = N * N
    h = 1.0 / N
    y = (np.arange(N) + 0.5) * h
    w = np.zeros(3 * n)
    w[:n] = np.repeat(np.sin(2 * np.pi * y), N)       # u[j][i] = sin(2 pi y_j)
    x, Xn, info = time_step(wl, w, rtol=1e-13)
    factor = (rho / dt) / (rho / dt + mu * 4.0 / h ** 2 * np.sin(np.pi * h) ** 2)
    assert np.linalg.norm(x[:n] - factor * w[:n]) <= 1e-10 * np.linalg.norm(w[:n])
    assert np.abs(x[n:2 * n]).max() < 1e-10
    assert np.abs(x[2 * n:] - x[2 * n:].mean()).max() < 1e-10
