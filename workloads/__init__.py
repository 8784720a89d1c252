"""Seeded synthetic inputs for the Stokes-IB solver.

This module only builds inputs: Lagrangian point positions, spring lists,
per-spring stiffnesses and right-hand sides.  It holds none of the solver's
arithmetic, so both the plain CPU oracle and the HIP library read the same
inputs from here.

Geometry follows the paper's test structures: a thin circular membrane
X(s1) = xc + r (cos s1, sin s1) (Sec. 5.2, circle configuration) and a thick
annulus X(s1, s2) = xc + (r + s2)(cos s1, sin s1) (Sec. 5.1, annulus
configuration), discretised by rings of equally spaced angles.  Each ring is a
closed fibre; the annulus also gets springs between the same angle index on
neighbouring rings.  Springs are linear with zero rest length (Sec. 5, linear
fibre force), so a stiffness per spring fully defines the elasticity operator.

Right-hand sides are drawn i.i.d. uniform[-1, 1] with
``numpy.random.default_rng(seed)`` in the order u-faces, v-faces, cells, each
N*N values in row-major (j, i) order.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Workload:
    """One Stokes-IB linear system: grid, fluid parameters and structure."""
    name: str
    N: int
    coarse_N: int
    rho: float
    mu: float
    dt: float
    X: np.ndarray            # [M, 2] float64 positions in [0, 1)^2
    springs: np.ndarray      # [E, 2] int32 node ids (a_e, b_e)
    kappa: np.ndarray        # [E] float64 spring stiffness
    smoother: str = "ras"    # "ras" | "sc"
    box: int = 8
    overlap: int = 2
    nu1: int = 2
    nu2: int = 2
    cheb_its: int = 2
    rhs_seed: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.X.shape[0])

    @property
    def levels(self) -> int:
        n, l = self.N, 0
        while n > self.coarse_N:
            n //= 2
            l += 1
        return l + 1


def ring(M: int, radius: float, centre=(0.5, 0.5)) -> np.ndarray:
    """M equally spaced points on a circle: theta_k = 2 pi k / M."""
    th = 2.0 * np.pi * np.arange(M, dtype=np.float64) / M
    X = np.empty((M, 2), dtype=np.float64)
    X[:, 0] = centre[0] + radius * np.cos(th)
    X[:, 1] = centre[1] + radius * np.sin(th)
    return np.mod(X, 1.0)


def ring_springs(M: int, offset: int = 0) -> np.ndarray:
    """Closed fibre: springs (k, k+1 mod M)."""
    k = np.arange(M, dtype=np.int64)
    return np.stack([offset + k, offset + (k + 1) % M], axis=1).astype(np.int32)


def membrane(M: int, radius: float = 0.25, centre=(0.5, 0.5)):
    X = ring(M, radius, centre)
    return X, ring_springs(M)


def annulus(n_rings: int, per_ring: int, r_in: float, r_out: float, centre=(0.5, 0.5)):
    """Rings at r_q = r_in + q (r_out - r_in)/(n_rings - 1), aligned angles;
    springs along each ring plus radial springs (q, k)-(q+1, k)."""
    Xs, S = [], []
    for q in range(n_rings):
        r = r_in + q * (r_out - r_in) / (n_rings - 1)
        Xs.append(ring(per_ring, r, centre))
        S.append(ring_springs(per_ring, q * per_ring))
    k = np.arange(per_ring, dtype=np.int64)
    for q in range(n_rings - 1):
        S.append(np.stack([q * per_ring + k, (q + 1) * per_ring + k], axis=1).astype(np.int32))
    return np.concatenate(Xs, 0), np.concatenate(S, 0)


def rhs(N: int, seed: int) -> np.ndarray:
    """Raw right-hand side: u, v, p blocks, i.i.d. uniform[-1, 1]."""
    g = np.random.default_rng(seed)
    bu = g.uniform(-1.0, 1.0, N * N)
    bv = g.uniform(-1.0, 1.0, N * N)
    bp = g.uniform(-1.0, 1.0, N * N)
    return np.concatenate([bu, bv, bp])


def random_points(M: int, seed: int) -> np.ndarray:
    g = np.random.default_rng(seed)
    return g.uniform(0.0, 1.0, (M, 2))


# --------------------------------------------------------------------------
# Named workloads (sizes and parameters of the solver's benchmark systems)
# --------------------------------------------------------------------------

def plain_32(**kw) -> Workload:
    """32x32 periodic Stokes (rho=0, mu=1), dt=1e-2; membrane r=0.25 with 128
    points, kappa=1e2; 3-level V-cycle, additive Vanka 8x8/2, nu=2+2."""
    X, S = membrane(128, 0.25)
    w = Workload("plain_32", 32, 8, 0.0, 1.0, 1e-2, X, S, np.full(len(S), 1e2))
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def smoother_256(kappa: float = 1e4, smoother: str = "ras", **kw) -> Workload:
    """256x256 periodic Stokes (mu=1), dt=1e-3; membrane r=0.25 with 1024
    points; 6-level V-cycle."""
    X, S = membrane(1024, 0.25)
    w = Workload(f"smoother_256_k{kappa:g}_{smoother}", 256, 8, 0.0, 1.0, 1e-3, X, S,
                 np.full(len(S), float(kappa)), smoother=smoother)
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def annulus_512(N: int = 512, **kw) -> Workload:
    """512x512 periodic, rho=1, mu=1e-2, dt=5e-4; annulus r in [0.2, 0.25]
    with 4 rings x 2048 points, ring and radial springs, kappa=1e4;
    7-level V-cycle (512 -> 8)."""
    X, S = annulus(4, 2048, 0.2, 0.25)
    w = Workload(f"annulus_{N}", N, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4))
    for k, v in kw.items():
        setattr(w, k, v)
    return w


def batch_systems(n_sys: int = 64, seed0: int = 1000, sizes=(64, 128, 256)) -> List[Workload]:
    """Independent Stokes systems (rho=0, mu=1, dt=1e-3): system s draws, with
    seed seed0+s and in this order, N from ``sizes``, kappa log-uniform in
    [1e1, 1e5] and a membrane radius uniform in [0.15, 0.3]; the membrane has
    4N points.  Its RHS seed is seed0+s as well."""
    out = []
    for s in range(n_sys):
        g = np.random.default_rng(seed0 + s)
        N = int(sizes[int(g.integers(0, len(sizes)))])
        kap = float(10.0 ** g.uniform(1.0, 5.0))
        r = float(g.uniform(0.15, 0.3))
        X, S = membrane(4 * N, r)
        w = Workload(f"batch_{s}", N, 8, 0.0, 1.0, 1e-3, X, S, np.full(len(S), kap),
                     rhs_seed=seed0 + s)
        out.append(w)
    return out


def diff_256(field_seed: int = 1, N: int = 256, M: int = 1024) -> Workload:
    """256x256 Stokes (mu=1, dt=1e-3), membrane of 1024 points,
    kappa_i = 1e3 (1 + 0.5 u_i) with u_i ~ U[-1, 1] from ``field_seed``."""
    X, S = membrane(M, 0.25)
    g = np.random.default_rng(field_seed)
    kap = 1e3 * (1.0 + 0.5 * g.uniform(-1.0, 1.0, len(S)))
    return Workload(f"diff_{N}_s{field_seed}", N, 8, 0.0, 1.0, 1e-3, X, S, kap)


def fd_springs(n_springs: int, count: int = 16, seed: int = 3) -> np.ndarray:
    g = np.random.default_rng(seed)
    return np.sort(g.choice(n_springs, size=count, replace=False))
