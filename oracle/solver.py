"""Outer solve of the Stokes-IB system (Eq. matrix-impib) with the multigrid
preconditioner, and the spring-stiffness gradient of a loss through the
adjoint system.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The periodic system is singular; the right-hand side is projected onto the
range of L_IB (block means removed) and the returned solution has no
null-space component.  The paper does not treat this case (its tests use a
lid-driven cavity); this is the reading for a periodic domain.
"""
import numpy as np

from . import hierarchy, ib
from .hierarchy import rest_lengths, spring_model
from .krylov import fgmres
from .multigrid import Multigrid


class Problem:
    def __init__(self, wl, build_mg=True):
        self.wl = wl
        self.levels = hierarchy.build(wl)
        self.fine = self.levels[-1]
        self.mg = Multigrid(self.levels, wl) if build_mg else None

    @property
    def L(self):
        return self.fine.L

    def apply(self, w):
        return self.L @ w

    def project(self, v):
        return hierarchy.project_range(v, self.wl.N, self.wl.rho)

    def solve(self, b, rtol=1e-8, restart=30, max_it=100):
        bp = self.project(b)
        x, info = fgmres(self.apply, self.mg, bp, restart=restart, rtol=rtol, max_it=max_it)
        x = self.project(x)
        r = bp - self.apply(x)
        info["rel_res_true"] = float(np.linalg.norm(r) / max(np.linalg.norm(bp), 1e-300))
        info["rhs_null_norm"] = float(np.linalg.norm(b - bp))
        return x, info


def spring_gradient(wl, w, lam):
    """dL/dkappa_e = -lam^T (dL_IB/dkappa_e) w for a loss L(w) with
    L_IB^T lam = dL/dw.  dL_IB/dkappa_e is the IB block -dt S (dK/dkappa_e) J,
    with dK/dkappa_e the stiffness matrix of spring e alone at unit kappa."""
    N = wl.N
    n = N * N
    M = wl.X.shape[0]
    g = np.zeros(wl.springs.shape[0])
    Us, Ls, Ss = [], [], []
    for comp in (0, 1):
        J = ib.interp_matrix(wl.X, N, comp)
        S = ib.spread_matrix(wl.X, N, comp)
        Us.append(J @ w[comp * n:(comp + 1) * n])
        Ls.append(S.T @ lam[comp * n:(comp + 1) * n])
    if spring_model(wl) == "tangent":
        # K'_tan is linear in each kappa_e: dK'/dkappa_e is spring e's
        # tangent stiffness at unit kappa
        U2 = np.concatenate(Us)
        L2 = np.concatenate(Ls)
        rest = rest_lengths(wl)
        for e in range(wl.springs.shape[0]):
            Ke = ib.tangent_stiffness(wl.X, wl.springs[e:e + 1], np.ones(1), rest[e:e + 1])
            g[e] = -wl.dt * (L2 @ (Ke @ U2))
        return g
    for e in range(wl.springs.shape[0]):
        a, b = int(wl.springs[e, 0]), int(wl.springs[e, 1])
        Ke = ib.stiffness_matrix(M, wl.springs[e:e + 1], np.ones(1))
        tot = 0.0
        for comp in (0, 1):
            tot += Ls[comp] @ (Ke @ Us[comp])
        g[e] = wl.dt * tot
    return g
