"""One step of the semi-implicit IB scheme (Sec. 2.2, Eqs. imp-momentum to
imp-F, without the convection term, which the paper also omits):

    L_IB(X^n) [u; p]^{n+1} = [(rho/dt) u^n + S_h^n K_h X^n; 0]   (Eq. matrix-impib)
    X^{n+1} = X^n + dt J_h^n u^{n+1}                              (Eq. imp-X-new)

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Positions live on the periodic unit square: spring separations are the
minimum-image displacements, and updated positions are wrapped into [0, 1).
"""
import numpy as np

from . import ib
from .solver import Problem


def fibre_force_periodic(X, springs, kappa):
    """Nodal forces F = K_h X of the linear springs, each spring's
    separation taken as the minimum-image displacement X_b - X_a."""
    X = np.asarray(X, dtype=np.float64)
    F = np.zeros_like(X)
    for e in range(springs.shape[0]):
        a, b = int(springs[e, 0]), int(springs[e, 1])
        d = X[b] - X[a]
        d -= np.round(d)
        F[a] += kappa[e] * d
        F[b] -= kappa[e] * d
    return F


def step_rhs(wl, w):
    """[(rho/dt) u^n + S_h F^n; 0] for w = [u; v; p] (the pressure part of w
    is not used)."""
    N = wl.N
    n = N * N
    F = fibre_force_periodic(wl.X, wl.springs, wl.kappa)
    rhs = np.zeros(3 * n)
    rhs[:2 * n] = (wl.rho / wl.dt) * np.asarray(w, dtype=np.float64)[:2 * n]
    for c in (0, 1):
        rhs[c * n:(c + 1) * n] += ib.spread_matrix(wl.X, N, c) @ F[:, c]
    return rhs


def advance_positions(wl, w):
    """X^{n+1} = X^n + dt J_h^n u^{n+1}, wrapped into [0, 1)."""
    N = wl.N
    n = N * N
    U = np.stack([ib.interp_matrix(wl.X, N, c) @ w[c * n:(c + 1) * n] for c in (0, 1)], 1)
    Xn = np.mod(wl.X + wl.dt * U, 1.0)
    Xn[Xn >= 1.0] = 0.0     # a tiny negative coordinate rounds up to 1.0 in mod
    return Xn


def time_step(wl, w, rtol=1e-12, max_it=200):
    """(w^{n+1}, X^{n+1}, solve info) from w^n and the workload's X^n."""
    P = Problem(wl)
    x, info = P.solve(step_rhs(wl, w), rtol=rtol, max_it=max_it)
    return x, advance_positions(wl, x), info
