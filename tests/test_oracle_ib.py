"""Pins for the oracle's coupling and elasticity operators (App. A.2-A.3, Sec. 5).

* Adjointness S = J^* under the grid weight h^2 and unit Lagrangian weights:
  h^2 <S F, u> = <F, J u>.
* Interpolating a constant field returns the constant (partition of unity).
* A single point: J S F = (sum_j phi^2)^2 F / h^2 = (9/64) F / h^2 wherever the
  point is.
* K_h X equals the spring-by-spring fibre force; K_h kills rigid translations.
* -dt S K J is symmetric positive semidefinite, annihilates constants and
  never couples the two velocity components.
"""
import numpy as np

import workloads as W
from oracle import ib


def test_spread_is_adjoint_of_interp():
    N = 32
    h = 1.0 / N
    rng = np.random.default_rng(1)
    X = W.random_points(50, 7)
    for comp in (0, 1):
        S = ib.spread_matrix(X, N, comp)
        J = ib.interp_matrix(X, N, comp)
        F = rng.standard_normal(50)
        u = rng.standard_normal(N * N)
        lhs = h * h * np.dot(S @ F, u)
        rhs = np.dot(F, J @ u)
        assert abs(lhs - rhs) < 1e-12 * (abs(lhs) + 1)


def test_interp_constant_and_single_point():
    N = 16
    h = 1.0 / N
    X = np.array([[0.0, 0.0], [0.999, 0.5], [0.3125, 0.71875], [0.123456, 0.987654]])
    for comp in (0, 1):
        J = ib.interp_matrix(X, N, comp)
        np.testing.assert_allclose(J @ np.full(N * N, 3.5), 3.5, atol=1e-14)
        for l in range(X.shape[0]):
            Xl = X[l:l + 1]
            Jl = ib.interp_matrix(Xl, N, comp)
            Sl = ib.spread_matrix(Xl, N, comp)
            np.testing.assert_allclose((Jl @ (Sl @ np.array([2.0])))[0], 2.0 * 9.0 / 64.0 / h ** 2,
                                       rtol=2e-15)


def test_stiffness_matches_fibre_force():
    X, S = W.annulus(3, 17, 0.2, 0.3)
    rng = np.random.default_rng(2)
    kap = rng.uniform(0.5, 2.0, S.shape[0])
    K = ib.stiffness_matrix(X.shape[0], S, kap)
    F = ib.fibre_force(X, S, kap)
    np.testing.assert_allclose(K @ X, F, atol=1e-13)
    np.testing.assert_allclose(K @ np.ones(X.shape[0]), 0.0, atol=1e-13)
    assert abs(K - K.T).max() == 0.0


def test_ib_term_psd_symmetric_translation_free():
    wl = W.plain_32()
    N = wl.N
    n = N * N
    T = ib.ib_term(wl.X, wl.springs, wl.kappa, N, wl.dt)
    Td = T.toarray()
    assert np.abs(Td - Td.T).max() < 1e-10 * np.abs(Td).max()
    assert np.abs(Td[:n, n:]).max() == 0.0 and np.abs(Td[n:, :n]).max() == 0.0
    ev = np.linalg.eigvalsh(0.5 * (Td + Td.T))
    assert ev.min() > -1e-9 * ev.max()
    np.testing.assert_allclose(T @ np.concatenate([np.ones(n), np.zeros(n)]), 0.0,
                               atol=1e-9 * np.abs(Td).max())
    np.testing.assert_allclose(T @ np.concatenate([np.zeros(n), np.ones(n)]), 0.0,
                               atol=1e-9 * np.abs(Td).max())


def test_interpolation_is_second_order_at_the_points():
    """The kernel's zeroth and first moment conditions make J_h u a second-order
    approximation of the continuous field at X_l (face positions of App. A.1)."""
    tp = 2 * np.pi
    X = W.random_points(40, 11)

    def err(N, comp):
        h = 1.0 / N
        j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
        x = i * h + (0.0 if comp == 0 else 0.5 * h)
        y = j * h + (0.5 * h if comp == 0 else 0.0)
        f = np.sin(tp * x) * np.cos(tp * y + 0.3)
        U = ib.interp_matrix(X, N, comp) @ f.ravel()
        ex = np.sin(tp * X[:, 0]) * np.cos(tp * X[:, 1] + 0.3)
        return np.max(np.abs(U - ex))

    for comp in (0, 1):
        e = [err(N, comp) for N in (32, 64, 128)]
        rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(rates > 1.85), rates
