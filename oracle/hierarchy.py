"""Grid hierarchy and level operators (Sec. 3.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Levels l = 0 (coarsest, coarse_N x coarse_N cells) .. lmax (finest, N x N),
refinement ratio 2.  A^l, G^l, D^l are rediscretisations on each level; the
Eulerian elasticity operator [S K J]^l is the Galerkin product
R_u [S K J]^{l+1} P_u for l < lmax (equation following Eq. matrix-h-impib).
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from . import ib, mac, transfer


@dataclass
class Level:
    N: int
    A: sp.csr_matrix        # rho/dt I - mu Lap_h on both components
    T: sp.csr_matrix        # -dt [S K J]^l (2N^2 square, PSD)
    G: sp.csr_matrix
    D: sp.csr_matrix
    L: sp.csr_matrix        # L_IB^l
    T_pattern: sp.csr_matrix  # structural 0/1 pattern of T

    @property
    def h(self):
        return 1.0 / self.N

    @property
    def n(self):
        return 3 * self.N * self.N

    @property
    def A_ib(self):
        return (self.A + self.T).tocsr()


def level_sizes(N, coarse_N):
    sizes = [N]
    while sizes[-1] > coarse_N:
        if sizes[-1] % 2:
            raise ValueError("N must be coarse_N * 2^k")
        sizes.append(sizes[-1] // 2)
    if sizes[-1] != coarse_N:
        raise ValueError("N must be coarse_N * 2^k")
    return sizes[::-1]


def spring_model(wl):
    m = getattr(wl, "spring_model", "linear")
    if m not in ("linear", "tangent"):
        raise ValueError(f"unknown spring model {m!r}")
    if m == "linear" and getattr(wl, "rest", None) is not None and np.any(np.asarray(wl.rest) != 0):
        raise ValueError("rest lengths need the tangent spring model")
    return m


def rest_lengths(wl):
    r = getattr(wl, "rest", None)
    return np.zeros(len(wl.springs)) if r is None else np.asarray(r, dtype=np.float64)


def build(wl, T_fine=None):
    """Build all levels for a workload (see ``workloads.Workload``)."""
    sizes = level_sizes(wl.N, wl.coarse_N)
    X, S, kap = wl.X, wl.springs, wl.kappa
    # Finest-level IB term -dt S K J and its structural pattern J^T K J; the
    # tangent model couples the two velocity components (Sec. 6).
    if spring_model(wl) == "tangent":
        T = ib.ib_term_tangent(X, S, kap, rest_lengths(wl), wl.N, wl.dt) if T_fine is None else T_fine
        TP = ib.tangent_pattern(X, S, wl.N)
    else:
        T = ib.ib_term(X, S, kap, wl.N, wl.dt) if T_fine is None else T_fine
        KP = ib.stiffness_pattern(X.shape[0], S)
        pats = []
        for comp in (0, 1):
            JP = ib.interp_pattern(X, wl.N, comp)
            pats.append(JP.T @ (KP @ JP))
        TP = sp.block_diag(pats, format="csr")
        TP.data[:] = 1.0
    levels = [None] * len(sizes)
    for l in range(len(sizes) - 1, -1, -1):
        N = sizes[l]
        if l < len(sizes) - 1:
            Ru = transfer.velocity_restriction(N)
            Pu = transfer.velocity_prolongation(N)
            T = (Ru @ (T @ Pu)).tocsr()
            TP = (Ru @ (TP @ Pu)).tocsr()
            TP.data[:] = 1.0
        A = mac.momentum(N, wl.rho, wl.mu, wl.dt)
        G = mac.gradient(N)
        D = mac.divergence(N)
        L = mac.stokes_ib((A + T).tocsr(), G, D)
        levels[l] = Level(N=N, A=A, T=T, G=G, D=D, L=L, T_pattern=TP)
    return levels


def null_space(N, rho):
    """Null vectors of the periodic L_IB: constant pressure always; constant u
    and constant v when rho = 0 (A then annihilates constants and the IB term
    does too, because the kernel rows sum to one and K_h kills translations)."""
    n = N * N
    vecs = []
    if rho == 0.0:
        c = np.zeros(3 * n)
        c[:n] = 1.0
        vecs.append(c)
        c = np.zeros(3 * n)
        c[n:2 * n] = 1.0
        vecs.append(c)
    c = np.zeros(3 * n)
    c[2 * n:] = 1.0
    vecs.append(c)
    return np.stack(vecs, 1)


def project_range(v, N, rho):
    """Remove the null-space components (block means) of a level vector."""
    n = N * N
    out = np.array(v, dtype=np.float64, copy=True)
    blocks = [(0, n), (n, 2 * n), (2 * n, 3 * n)] if rho == 0.0 else [(2 * n, 3 * n)]
    for a, b in blocks:
        out[a:b] -= out[a:b].mean()
    return out
