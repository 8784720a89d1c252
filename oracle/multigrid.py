"""Recursive V-cycle (Sec. 3.1, Alg. 1) with FGMRES-wrapped smoothing
(Sec. 3.3) and a direct solve on the coarsest level.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Coarsest solve: the periodic L_IB^0 is singular (constant pressure, and
constant velocity components when rho = 0), so the direct solve uses the
bordered matrix [[L0, C], [C^T, 0]] with C the null vectors; it returns the
solution orthogonal to the null space.
"""
import numpy as np
import scipy.linalg as la

from . import transfer
from .hierarchy import null_space
from .krylov import fgmres_smooth, richardson_smooth
from .schur import SchurSmoother
from .schwarz import RAS, RMS, structural_pattern


class CoarseSolver:
    def __init__(self, level, rho):
        L0 = level.L.toarray()
        C = null_space(level.N, rho)
        k = C.shape[1]
        B = np.block([[L0, C], [C.T, np.zeros((k, k))]])
        self.n = L0.shape[0]
        self.k = k
        self.lu = la.lu_factor(B)

    def __call__(self, r):
        rhs = np.concatenate([r, np.zeros(self.k)])
        return la.lu_solve(self.lu, rhs)[:self.n]


class Multigrid:
    def __init__(self, levels, wl):
        self.levels = levels
        self.wl = wl
        self.coarse = CoarseSolver(levels[0], wl.rho)
        self.smoothers = [None]
        self.R = [None]
        self.P = [None]
        for l in range(1, len(levels)):
            lev = levels[l]
            combine = getattr(wl, "combine", "restricted")
            if combine != "restricted" and wl.smoother != "ras":
                raise ValueError("the summed combination applies to additive Schwarz only")
            if wl.smoother == "ras":
                self.smoothers.append(RAS(lev.L, lev.N, wl.box, wl.overlap, combine))
            elif wl.smoother == "rms":
                self.smoothers.append(RMS(lev.L, structural_pattern(lev), lev.N, wl.box, wl.overlap))
            elif wl.smoother == "sc":
                self.smoothers.append(SchurSmoother(lev, wl.rho, wl.cheb_its))
            else:
                raise ValueError(wl.smoother)
            Nc = levels[l - 1].N
            self.R.append(transfer.restriction(Nc))
            self.P.append(transfer.prolongation(Nc))

    def smooth(self, l, w, b, nu):
        """Sec. 3.3 smoothing: nu FGMRES iterations preconditioned by the basic
        smoother, or (sweep "richardson", the Sec. 6 reading) nu Richardson
        steps with it."""
        L = self.levels[l].L
        sweep = getattr(self.wl, "sweep", "fgmres")
        if sweep == "richardson":
            return richardson_smooth(lambda x: L @ x, self.smoothers[l], w, b, nu)
        if sweep != "fgmres":
            raise ValueError(sweep)
        return fgmres_smooth(lambda x: L @ x, self.smoothers[l], w, b, nu)

    def mg(self, l, w, b):
        """Alg. 1: w <- MG(w, b, Omega^l, nu1, nu2)."""
        if l == 0:
            return self.coarse(b)
        L = self.levels[l].L
        w = self.smooth(l, w, b, self.wl.nu1)
        r = b - L @ w
        rc = self.R[l] @ r
        ec = self.mg(l - 1, np.zeros_like(rc), rc)
        w = w + self.P[l] @ ec
        w = self.smooth(l, w, b, self.wl.nu2)
        return w

    def vcycle(self, r):
        """Preconditioner application z = MG(0, r) on the finest level."""
        top = len(self.levels) - 1
        return self.mg(top, np.zeros_like(r), r)

    __call__ = vcycle
