"""Pins of the oracle's springs with rest lengths and their tangent stiffness
(the Sec. 5 fibre model with a tension that vanishes at the rest length,
App. A.2; the Jacobian a Newton-Krylov step uses, Sec. 6).

Each test checks against something the mathematics fixes:
* the nodal force is minus the gradient of the spring energy
  sum_e kappa_e (l_e - L_e)^2 / 2 (central differences of the energy);
* the tangent stiffness is minus the Jacobian of that force (central
  differences of the force), also for a spring across the periodic boundary;
* with zero rest lengths the tangent operator is the linear one, exactly;
* rigid motions: a translation is in the null space, and an infinitesimal
  rotation A (X - c) maps to -A F (forces turn with the body);
* the coupled A_IB stays symmetric and its cross blocks are nonzero;
* Laplace's law with a rest length: a circular membrane of M springs at
  length l > L is held by the pressure jump kappa (l - L) M sin(pi/M) / (pi R),
  the tension over the radius in the continuum limit; at l = L there is no
  force;
* the stiffness gradient of a loss through the tangent operator matches
  central differences of dense solves.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import hierarchy, ib
from oracle.solver import spring_gradient
from oracle.timestep import step_rhs, time_step


def _config(seed=0):
    g = np.random.default_rng(seed)
    X = g.uniform(0.3, 0.7, (7, 2))
    X[6] = [0.98, 0.52]                       # its springs cross x = 1
    S = np.array([[0, 1], [1, 2], [2, 3], [3, 4], [4, 0], [1, 5], [5, 6], [6, 2]], dtype=np.int32)
    X[5] = [0.03, 0.50]
    kap = g.uniform(20.0, 80.0, len(S))
    rest = g.uniform(0.02, 0.25, len(S))
    rest[2] = 0.0                             # one zero-rest-length spring
    return X, S, kap, rest


def _energy(X, S, kap, rest):
    E = 0.0
    for e, (a, b) in enumerate(S):
        d = X[b] - X[a]
        d -= np.round(d)
        E += 0.5 * kap[e] * (np.hypot(*d) - rest[e]) ** 2
    return E


def test_force_is_minus_energy_gradient():
    X, S, kap, rest = _config()
    F = ib.spring_force(X, S, kap, rest)
    eps = 1e-6
    for l in range(X.shape[0]):
        for c in (0, 1):
            Xp, Xm = X.copy(), X.copy()
            Xp[l, c] += eps
            Xm[l, c] -= eps
            fd = -(_energy(Xp, S, kap, rest) - _energy(Xm, S, kap, rest)) / (2 * eps)
            assert abs(F[l, c] - fd) <= 1e-7 * np.abs(F).max(), (l, c)


def test_tangent_is_minus_force_jacobian():
    X, S, kap, rest = _config(1)
    M = X.shape[0]
    K = ib.tangent_stiffness(X, S, kap, rest).toarray()
    assert np.allclose(K, K.T, atol=1e-12 * np.abs(K).max())
    eps = 1e-6
    for l in range(M):
        for c in (0, 1):
            Xp, Xm = X.copy(), X.copy()
            Xp[l, c] += eps
            Xm[l, c] -= eps
            dF = (ib.spring_force(Xp, S, kap, rest) - ib.spring_force(Xm, S, kap, rest)) / (2 * eps)
            col = -np.concatenate([dF[:, 0], dF[:, 1]])          # planar order
            assert np.abs(K[:, c * M + l] - col).max() <= 1e-6 * np.abs(K).max(), (l, c)


def test_zero_rest_length_is_the_linear_operator():
    X, S, kap, _ = _config(2)
    z = np.zeros(len(S))
    K = ib.tangent_stiffness(X, S, kap, z)
    Kl = -ib.stiffness_matrix(X.shape[0], S, kap)
    assert abs(K - sp.block_diag([Kl, Kl])).max() == 0.0
    N = 16
    T = ib.ib_term_tangent(X, S, kap, z, N, 1e-2)
    Tl = ib.ib_term(X, S, kap, N, 1e-2)
    assert abs(T - Tl).max() <= 1e-14 * abs(Tl).max()
    F0 = ib.spring_force(X, S, kap, z)
    d = X[S[:, 1]] - X[S[:, 0]]
    d -= np.round(d)
    Fl = np.zeros_like(X)
    np.add.at(Fl, S[:, 0], kap[:, None] * d)
    np.add.at(Fl, S[:, 1], -kap[:, None] * d)
    assert np.abs(F0 - Fl).max() <= 1e-14 * np.abs(Fl).max()


def test_rigid_motions():
    X, S, kap, rest = _config(3)
    X[5] = [0.35, 0.50]
    X[6] = [0.62, 0.55]                        # keep this configuration unwrapped
    M = X.shape[0]
    K = ib.tangent_stiffness(X, S, kap, rest)
    F = ib.spring_force(X, S, kap, rest)
    tx = np.concatenate([np.ones(M), np.zeros(M)])
    ty = np.concatenate([np.zeros(M), np.ones(M)])
    scale = abs(K).max()
    assert np.abs(K @ tx).max() <= 1e-12 * scale and np.abs(K @ ty).max() <= 1e-12 * scale
    c = np.array([0.5, 0.5])
    R = X - c
    rot = np.concatenate([-R[:, 1], R[:, 0]])   # A (X - c), A = [[0, -1], [1, 0]]
    AF = np.concatenate([-F[:, 1], F[:, 0]])
    assert np.abs(K @ rot + AF).max() <= 1e-12 * np.abs(F).max() * 10


def test_coupled_operator_is_symmetric_with_cross_blocks():
    N, M = 32, 96
    X, S = W.membrane(M, 0.3)
    chord = 2 * 0.3 * np.sin(np.pi / M)
    wl = W.Workload("t", N, 8, 1.0, 0.1, 1e-3, X, S, np.full(M, 1e3), spring_model="tangent",
                    rest=np.full(M, 0.6 * chord))
    levels = hierarchy.build(wl)
    n = N * N
    for lev in levels:
        A = lev.A_ib
        assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
        m = lev.N * lev.N
        assert abs(lev.T[:m, m:]).max() > 1e-3 * abs(lev.T).max()
        # the structural pattern covers every entry
        nz = (abs(lev.T) > 0).astype(np.float64)
        outside = nz - nz.multiply(lev.T_pattern > 0)
        outside.eliminate_zeros()
        assert outside.nnz == 0
    assert levels[-1].T.shape == (2 * n, 2 * n)


def test_unknown_model_and_stray_rest_lengths_are_rejected():
    X, S = W.membrane(32, 0.25)
    wl = W.Workload("t", 16, 8, 0.0, 1.0, 1e-2, X, S, np.ones(32), spring_model="bent")
    with pytest.raises(ValueError):
        hierarchy.build(wl)
    wl = W.Workload("t", 16, 8, 0.0, 1.0, 1e-2, X, S, np.ones(32), rest=np.full(32, 0.01))
    with pytest.raises(ValueError):
        hierarchy.build(wl)


@pytest.mark.parametrize("frac", [0.5, 0.8])
def test_laplace_law_with_rest_length(frac):
    N, R, kap = 32, 0.25, 1e2
    M = 4 * N
    X, S = W.membrane(M, R)
    l = 2 * R * np.sin(np.pi / M)
    wl = W.Workload("laplace_rest", N, 8, 0.0, 1.0, 1e-3, X, S, np.full(M, kap), spring_model="tangent",
                    rest=np.full(M, frac * l))
    x, Xn, info = time_step(wl, np.zeros(3 * N * N), rtol=1e-10)
    assert info["converged"]
    n = N * N
    p = x[2 * n:].reshape(N, N)
    c = N // 2
    dp = p[c - 1:c + 1, c - 1:c + 1].mean() - p[0:2, 0:2].mean()
    exact = kap * (l - frac * l) * M * np.sin(np.pi / M) / (np.pi * R)
    assert abs(dp / exact - 1) < 1e-3
    assert np.abs(x[:2 * n]).max() < 1e-2 * dp * R
    assert np.abs(Xn - X).max() < 1e-5


def test_membrane_at_rest_length_has_no_force():
    N, R, M = 32, 0.25, 128
    X, S = W.membrane(M, R)
    l = 2 * R * np.sin(np.pi / M)
    wl = W.Workload("rest", N, 8, 0.0, 1.0, 1e-3, X, S, np.full(M, 1e2), spring_model="tangent",
                    rest=np.full(M, l))
    assert np.abs(step_rhs(wl, np.zeros(3 * N * N))).max() <= 1e-12 * 1e2 * l * N * N


def test_tangent_gradient_matches_central_differences():
    N = 16
    X, S = W.membrane(24, 0.22)
    chord = 2 * 0.22 * np.sin(np.pi / 24)
    g0 = np.random.default_rng(7)
    kap = 50.0 * (1 + 0.5 * g0.uniform(-1, 1, S.shape[0]))
    rest = chord * g0.uniform(0.3, 0.9, S.shape[0])
    b = hierarchy.project_range(W.rhs(N, 0), N, 0.0)
    ut = hierarchy.project_range(W.rhs(N, 5), N, 0.0)
    n = N * N

    def wl_of(k):
        return W.Workload("g", N, 8, 0.0, 1.0, 1e-2, X, S, k, spring_model="tangent", rest=rest)

    def dense(L, rhs):
        C = hierarchy.null_space(N, 0.0)
        k = C.shape[1]
        B = np.block([[L.toarray(), C], [C.T, np.zeros((k, k))]])
        return np.linalg.solve(B, np.concatenate([rhs, np.zeros(k)]))[:L.shape[0]]

    def loss(k):
        L = hierarchy.build(wl_of(k))[-1].L
        w = dense(L, b)
        return 0.5 * np.sum((w[:2 * n] - ut[:2 * n]) ** 2), w, L

    f0, w, L = loss(kap)
    g_rhs = np.zeros(3 * n)
    g_rhs[:2 * n] = w[:2 * n] - ut[:2 * n]
    lam = dense(L.T.tocsr(), hierarchy.project_range(g_rhs, N, 0.0))
    g = spring_gradient(wl_of(kap), w, lam)
    for e in (0, 9, 17):
        step = 1e-4 * kap[e]
        kp, km = kap.copy(), kap.copy()
        kp[e] += step
        km[e] -= step
        fd = (loss(kp)[0] - loss(km)[0]) / (2 * step)
        assert abs(fd - g[e]) <= 1e-6 * abs(fd) + 1e-12, (e, fd, g[e])
