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
from .hierarchy import rest_lengths, spring_model
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


def nodal_force(wl):
    """F^n: the linear springs' K_h X^n, or with the tangent model the force
    of the springs with rest lengths (``ib.spring_force``), whose Jacobian is
    the operator's stiffness."""
    if spring_model(wl) == "tangent":
        return ib.spring_force(wl.X, wl.springs, wl.kappa, rest_lengths(wl))
    return fibre_force_periodic(wl.X, wl.springs, wl.kappa)


def step_rhs(wl, w):
    """[(rho/dt) u^n + S_h F^n; 0] for w = [u; v; p] (the pressure part of w
    is not used).  With the tangent model the step is linearly implicit:
    F(X^{n+1}) ~ F^n + dt (dF/dX)(X^n) J_h u^{n+1}, the second term being the
    operator's IB part."""
    N = wl.N
    n = N * N
    F = nodal_force(wl)
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
