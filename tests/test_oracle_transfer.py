"""Pins for the oracle's transfers and coarse operators (Sec. 3.1-3.2).

* R_u = P_u^* in the grid inner products (h_f^2 <R... > identity).
* Raviart-Thomas prolongation preserves divergence: D_f P_u u_c equals D_c u_c
  copied to the four fine cells of each coarse cell.
* P_u and P_p reproduce constants; R_p P_p maps constants to themselves.
* R_p is the four-cell mean: it returns a coarse field from its piecewise
  constant injection, and R_u G_f = G_c R_p holds exactly (the transpose of
  the RT0 divergence identity, with G = -D^T and R_u = P_u^T / 4).
* The Galerkin coarse IB operator R_u [SKJ]^{l+1} P_u equals
  dt/h_l^2 J_l^T K' J_l with J_l = J_{l+1} P_u (composed in the test), is
  symmetric positive semidefinite and annihilates constant velocities.
"""
import numpy as np

import workloads as W
from oracle import hierarchy, ib, mac, transfer


def test_velocity_restriction_is_adjoint():
    Nc = 8
    hf, hc = 1.0 / (2 * Nc), 1.0 / Nc
    rng = np.random.default_rng(0)
    P = transfer.velocity_prolongation(Nc)
    R = transfer.velocity_restriction(Nc)
    uf = rng.standard_normal(P.shape[0])
    uc = rng.standard_normal(P.shape[1])
    assert abs(hc ** 2 * np.dot(R @ uf, uc) - hf ** 2 * np.dot(uf, P @ uc)) < 1e-13


def test_rt0_preserves_divergence():
    Nc = 8
    Nf = 2 * Nc
    rng = np.random.default_rng(1)
    uc = rng.standard_normal(2 * Nc * Nc)
    dc = (mac.divergence(Nc) @ uc).reshape(Nc, Nc)
    df = (mac.divergence(Nf) @ (transfer.velocity_prolongation(Nc) @ uc)).reshape(Nf, Nf)
    inj = np.kron(dc, np.ones((2, 2)))
    np.testing.assert_allclose(df, inj, atol=1e-12)


def test_transfers_reproduce_constants():
    Nc = 6
    Pu = transfer.velocity_prolongation(Nc)
    Pp = transfer.pressure_prolongation(Nc)
    Rp = transfer.pressure_restriction(Nc)
    Ru = transfer.velocity_restriction(Nc)
    c = np.concatenate([np.full(Nc * Nc, 2.0), np.full(Nc * Nc, -1.0)])
    f = Pu @ c
    n = 4 * Nc * Nc
    np.testing.assert_allclose(f[:n], 2.0)
    np.testing.assert_allclose(f[n:], -1.0)
    np.testing.assert_allclose(Ru @ f, c)
    np.testing.assert_allclose(Pp @ np.full(Nc * Nc, 3.0), 3.0)
    np.testing.assert_allclose(Rp @ (Pp @ np.full(Nc * Nc, 3.0)), 3.0)


def test_pressure_restriction_inverts_injection():
    """A fine field constant on every 2 x 2 block of a coarse cell restricts
    to that coarse field (Sec. 3.2: R_p averages the four fine cells)."""
    rng = np.random.default_rng(11)
    for Nc in (3, 4, 8):
        pc = rng.standard_normal((Nc, Nc))
        pf = np.kron(pc, np.ones((2, 2))).ravel()
        np.testing.assert_allclose(transfer.pressure_restriction(Nc) @ pf, pc.ravel(), rtol=0, atol=1e-14)


def test_pressure_restriction_commutes_with_gradient():
    """R_u G_f p = G_c R_p p for every fine p.  RT0 prolongation preserves the
    divergence, D_f P_u = I_0 D_c with I_0 the injection into the four fine
    cells; transposing with G = -D^T, R_u = P_u^T / 4 (h_f / h_c = 1/2) and
    R_p = I_0^T / 4 gives the identity, with no rounding beyond the sums."""
    rng = np.random.default_rng(12)
    for Nc in (4, 6, 8):
        p = rng.standard_normal(4 * Nc * Nc)
        lhs = transfer.velocity_restriction(Nc) @ (mac.gradient(2 * Nc) @ p)
        rhs = mac.gradient(Nc) @ (transfer.pressure_restriction(Nc) @ p)
        assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()


def test_pressure_prolongation_is_bilinear():
    Nc = 8
    hc = 1.0 / Nc
    j, i = np.meshgrid(np.arange(Nc), np.arange(Nc), indexing="ij")
    # a globally linear field is periodic only if constant, so test a smooth
    # field away from the wrap: bilinear interpolation is exact for x*y.
    pc = (((i + 0.5) * hc) * ((j + 0.5) * hc)).ravel()
    pf = (transfer.pressure_prolongation(Nc) @ pc).reshape(2 * Nc, 2 * Nc)
    J, I = np.meshgrid(np.arange(2 * Nc), np.arange(2 * Nc), indexing="ij")
    hf = hc / 2
    ex = ((I + 0.5) * hf) * ((J + 0.5) * hf)
    inner = (I >= 1) & (I < 2 * Nc - 1) & (J >= 1) & (J < 2 * Nc - 1)
    np.testing.assert_allclose(pf[inner], ex[inner], atol=1e-14)


def test_galerkin_ib_operator_two_routes():
    wl = W.plain_32()
    levels = hierarchy.build(wl)
    K = ib.stiffness_matrix(wl.M, wl.springs, wl.kappa)
    Jf = [ib.interp_matrix(wl.X, wl.N, c) for c in (0, 1)]
    Jl = [J.toarray() for J in Jf]
    for l in range(len(levels) - 2, -1, -1):
        Nc = levels[l].N
        Pu = transfer.velocity_prolongation(Nc).toarray()
        nc, nf = Nc * Nc, 4 * Nc * Nc
        Jl = [Jl[0] @ Pu[:nf, :nc], Jl[1] @ Pu[nf:, nc:]]
        h = 1.0 / Nc
        T = levels[l].T.toarray()
        for c in (0, 1):
            route2 = (wl.dt / h ** 2) * Jl[c].T @ (-K.toarray()) @ Jl[c]
            blk = T[c * nc:(c + 1) * nc, c * nc:(c + 1) * nc]
            np.testing.assert_allclose(blk, route2, atol=1e-12 * np.abs(route2).max())
        assert np.abs(T - T.T).max() <= 1e-12 * np.abs(T).max()
        ev = np.linalg.eigvalsh(0.5 * (T + T.T))
        assert ev.min() > -1e-10 * ev.max()
        one = np.concatenate([np.ones(nc), np.zeros(nc)])
        assert np.abs(T @ one).max() < 1e-9 * np.abs(T).max()
