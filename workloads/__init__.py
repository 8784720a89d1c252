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
    # "linear": zero-rest-length springs, force kappa_e (X_b - X_a);
    # "tangent": springs with rest lengths ``rest`` [E] (None = all zero), the
    # operator linearised at X
    spring_model: str = "linear"
    rest: Optional[np.ndarray] = None
    # additive Schwarz combination: "restricted" (each unknown from its owner
    # box) or "sum" (summed over every box holding it)
    combine: str = "restricted"
    # a smoothing step: "fgmres" (FGMRES iterations preconditioned by the
    # basic smoother) or "richardson" (undamped Richardson steps)
    sweep: str = "fgmres"

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


def suspension_points(n_side: int, radius: float, per_ring: int) -> np.ndarray:
    """Points of a suspension of n_side x n_side circular membranes (the
    layout of the paper's suspension test, Sec. 5.3, at any count): ring
    (a, b) is centred at ((a + 1/2), (b + 1/2)) / n_side with the given
    radius and per_ring equally spaced points; rings follow each other in
    row-major order and each ring's points run along the fibre."""
    out = []
    for b_ in range(n_side):
        for a_ in range(n_side):
            out.append(ring(per_ring, radius, ((a_ + 0.5) / n_side, (b_ + 0.5) / n_side)))
    return np.concatenate(out, 0)


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


# --------------------------------------------------------------------------
# The paper's test structures (Sec. 5.1 thick elastic shell, Sec. 5.2 thin
# elastic membrane) at their stated resolutions, on the periodic unit square
# --------------------------------------------------------------------------

#: the stiffness scale of Sec. 5.1: alpha = gamma * 3.93 / 0.005 (the largest
#: stiffness an explicit scheme takes for the shell at h = 1/64, dt = 0.005)
ALPHA_EXPLICIT = 3.93 / 0.005
#: thickness and inner radius of the shell, radius of the membrane (Sec. 5.1,
#: Eq. annulus; Sec. 5.2, Eq. circle); both centred at (0.5, 0.5)
SHELL_WIDTH = 1.0 / 16.0
SHELL_RADIUS = 0.25
MEMBRANE_RADIUS = 0.25


def paper_counts(N: int):
    """(M1, M2) = (19 N / 8, 3 N / 32 + 1) Lagrangian points along and across
    the fibres (Sec. 5.1); both exact for N a multiple of 32."""
    if N % 32:
        raise ValueError("the paper's point counts need N to be a multiple of 32")
    return 19 * N // 8, 3 * N // 32 + 1


def thick_shell(N: int, gamma: float, centre=(0.5, 0.5)):
    """Thick annulus X(s1, s2) = c + (r + s2)(cos s1, sin s1), s1 in [0, 2 pi),
    s2 in [0, w] (Sec. 5.1), M1 x M2 nodes; fibres run along s1 only (force
    density alpha d^2 X / ds1^2, Eq. F-lin-functional).  The half-index
    differences of App. A.2 with the nodal quadrature weight ds1 ds2 of the
    spreading sum make the nodal force of node l on fibre m
        alpha ds2 / ds1 (X_{l+1,m} - 2 X_{l,m} + X_{l-1,m}),
    i.e. zero-rest-length springs of stiffness kappa = alpha ds2 / ds1 between
    fibre neighbours.  Returns (X [M1 M2, 2], springs, kappa, (ds1, ds2))."""
    M1, M2 = paper_counts(N)
    ds1 = 2.0 * np.pi / M1
    ds2 = SHELL_WIDTH / (M2 - 1)
    alpha = gamma * ALPHA_EXPLICIT
    Xs, S = [], []
    for m in range(M2):
        Xs.append(ring(M1, SHELL_RADIUS + m * ds2, centre))
        S.append(ring_springs(M1, m * M1))
    S = np.concatenate(S, 0)
    return np.concatenate(Xs, 0), S, np.full(len(S), alpha * ds2 / ds1), (ds1, ds2)


def thin_membrane(N: int, gamma: float, centre=(0.5, 0.5)):
    """Thin circle X(s1) = c + r (cos s1, sin s1) (Sec. 5.2) with M1 = 19 N / 8
    nodes and alpha = 7 gamma 3.93 / 0.005; the nodal weight ds1 makes the
    spring stiffness kappa = alpha / ds1.  Returns (X, springs, kappa, ds1)."""
    M1, _ = paper_counts(N)
    ds1 = 2.0 * np.pi / M1
    alpha = 7.0 * gamma * ALPHA_EXPLICIT
    X, S = membrane(M1, MEMBRANE_RADIUS, centre)
    return X, S, np.full(len(S), alpha / ds1), ds1


def background_flow(N: int) -> np.ndarray:
    """A velocity u^n of unit speed for the first step: the periodic cell flow
    of the stream function psi = sin(2 pi x) sin(2 pi y) / (2 pi), sampled at
    the grid nodes (i h, j h) and differenced onto the faces,
        u[j, i] = (psi[j+1, i] - psi[j, i]) / h   at (i h, (j + 1/2) h)
        v[j, i] = -(psi[j, i+1] - psi[j, i]) / h  at ((i + 1/2) h, j h),
    so its MAC divergence vanishes to rounding.  Returns [u | v | 0] (3 N^2);
    it stands in for the unit lid speed that sets the flow scale of the
    paper's cavity tests."""
    h = 1.0 / N
    t = np.arange(N + 1) * h
    psi = np.outer(np.sin(2 * np.pi * t), np.sin(2 * np.pi * t)) / (2 * np.pi)   # psi[j, i]
    u = (psi[1:, :-1] - psi[:-1, :-1]) / h
    v = -(psi[:-1, 1:] - psi[:-1, :-1]) / h
    return np.concatenate([u.ravel(), v.ravel(), np.zeros(N * N)])


#: flow conditions of the results section: Stokes (rho = 0, mu = 1) and
#: time-dependent flow with rho = 1, mu = 1 / Re
FLOWS = {"stokes": (0.0, 1.0), "mu1": (1.0, 1.0), "mu0.1": (1.0, 0.1),
         "mu0.01": (1.0, 0.01), "mu0.001": (1.0, 0.001)}


def paper_case(structure: str, N: int, gamma: float, flow: str = "stokes",
               smoother: str = "ras", box: int = 8, overlap: int = 2, **kw) -> Workload:
    """One linear system of the results section: the thick shell ("thick") or
    thin membrane ("thin") at N, stiffness ratio gamma, a flow of ``FLOWS``,
    dt = 0.32 h, an 8 x 8 coarsest grid (Sec. 5)."""
    rho, mu = FLOWS[flow]
    if structure == "thick":
        X, S, kap, _ = thick_shell(N, gamma)
    elif structure == "thin":
        X, S, kap, _ = thin_membrane(N, gamma)
    else:
        raise ValueError(f"unknown structure {structure!r}")
    tag = f"{structure}_N{N}_g{gamma:g}_{flow}_{smoother}"
    if smoother != "sc":
        tag += f"_b{box}o{overlap}"
    w = Workload(tag, N, 8, rho, mu, 0.32 / N, X, S, kap, smoother=smoother, box=box, overlap=overlap)
    for k, v in kw.items():
        setattr(w, k, v)
    return w
