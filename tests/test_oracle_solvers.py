"""Pins for the oracle's smoothers, Krylov solver and V-cycle (Sec. 3, Alg. 1-2,
Eq. fact-Stokes-IB and approx-fact-Stokes-IB).

Each test checks against something the mathematics fixes, not against the
oracle's own formulas:
* FGMRES with a fixed preconditioner sequence returns x0 + Z y with y the
  least-squares minimiser of ||b - A Z y|| (brute force over the recorded Z);
  with the identity it is GMRES, the minimal residual over the Krylov space.
* Restarted FGMRES: every cycle adds to x the minimiser of the residual over
  that cycle's Krylov space of the current residual (brute force per cycle),
  and each recorded estimate is the true residual of the partial minimiser.
* RAS: owned sets partition the unknowns; for any e supported in a box's index
  set, RAS(L e) reproduces e on that box's owned set.
* SC composition with exact inner solves is L_IB^{-1} (Eq. fact-Stokes-IB).
* Chebyshev on a diagonal matrix equals the closed-form residual polynomial
  T_k((theta - lam)/delta) / T_k(theta/delta).
* Multicolour symmetric Gauss-Seidel with every row its own colour is the
  textbook forward/backward triangular-solve sweep; greedy colours are proper;
  SGS-preconditioned SPD spectra lie in (0, 1].
* Arnoldi on an operator with <= 10 distinct eigenvalues returns the largest.
* The bordered coarsest solve returns the minimum-norm-in-null-space solution.
* FGMRES + V-cycle reaches 1e-8 and agrees with a dense direct solve.
* The spring-stiffness gradient matches central differences of dense solves.
"""
import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import workloads as W
from oracle import hierarchy, krylov, mac, schur, schwarz
from oracle.multigrid import CoarseSolver
from oracle.solver import Problem, spring_gradient


def test_fgmres_identity_is_minimal_residual():
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n)
    for k in (1, 3, 7):
        dx, steps, est = krylov.fgmres_cycle(lambda x: A @ x, lambda x: x, b, k)
        Kr = np.stack([np.linalg.matrix_power(A, i) @ b for i in range(k)], 1)
        Q, _ = np.linalg.qr(Kr)
        y = np.linalg.lstsq(A @ Q, b, rcond=None)[0]
        np.testing.assert_allclose(dx, Q @ y, rtol=1e-9, atol=1e-11)
        assert abs(est - np.linalg.norm(b - A @ dx)) < 1e-9


def test_fgmres_flexible_minimises_over_z():
    rng = np.random.default_rng(4)
    n = 30
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    b = rng.standard_normal(n)
    Zs = []
    mats = [np.eye(n) + 0.3 * rng.standard_normal((n, n)) for _ in range(5)]
    calls = {"i": 0}

    def prec(v):
        z = mats[calls["i"]] @ v
        calls["i"] += 1
        Zs.append(z)
        return z

    dx, k, est = krylov.fgmres_cycle(lambda x: A @ x, prec, b, 5)
    Z = np.stack(Zs, 1)
    y = np.linalg.lstsq(A @ Z, b, rcond=None)[0]
    np.testing.assert_allclose(dx, Z @ y, rtol=1e-9, atol=1e-11)


def _restarted_gmres_brute(A, b, restart, iters):
    """Restarted GMRES written from its definition: per cycle, the residual
    minimiser over span{r, A r, ..., A^(k-1) r} of the current residual r,
    added to x; returns x and the residual norm after every iteration."""
    x = np.zeros_like(b)
    hist = []
    done = 0
    while done < iters:
        r = b - A @ x
        k = min(restart, iters - done)
        best = None
        for j in range(1, k + 1):
            Kr = np.stack([np.linalg.matrix_power(A, i) @ r for i in range(j)], 1)
            Q, _ = np.linalg.qr(Kr)
            y = np.linalg.lstsq(A @ Q, r, rcond=None)[0]
            best = Q @ y
            hist.append(float(np.linalg.norm(r - A @ best)))
        x = x + best
        done += k
    return x, hist


def test_fgmres_restarts_accumulate_minimal_residual_cycles():
    """FGMRES(3) with the identity preconditioner for 12 iterations is four
    GMRES(3) cycles (Saad's restarted GMRES, the outer method of Sec. 3): the
    iterate keeps every cycle's correction, and the history holds each
    iteration's minimal residual.  A restart that dropped x, reused a stale
    residual or skipped the last partial cycle fails here."""
    rng = np.random.default_rng(21)
    n = 36
    A = np.diag(np.linspace(1.0, 12.0, n)) + 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    for restart, iters in ((3, 12), (5, 12), (4, 9)):
        x, info = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=restart, rtol=1e-300, max_it=iters)
        assert info["iters"] == iters and not info["converged"]
        xb, hb = _restarted_gmres_brute(A, b, restart, iters)
        np.testing.assert_allclose(x, xb, rtol=1e-9, atol=1e-12 * np.linalg.norm(xb))
        np.testing.assert_allclose(info["history"], hb, rtol=1e-8)
        # restarting loses optimality: one unrestarted cycle does better
        xf, _ = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=iters, rtol=1e-300, max_it=iters)
        assert np.linalg.norm(b - A @ xf) < np.linalg.norm(b - A @ x)


def test_ras_partition_and_local_reproduction():
    wl = W.plain_32()
    lev = hierarchy.build(wl)[-1]
    parts = schwarz.patches(lev.N, wl.box, wl.overlap)
    own = np.concatenate([p.own_global for p in parts])
    assert np.array_equal(np.sort(own), np.arange(lev.n))
    ras = schwarz.RAS(lev.L, lev.N, wl.box, wl.overlap)
    rng = np.random.default_rng(5)
    for k in (0, 5, 10, 15):
        e = np.zeros(lev.n)
        e[parts[k].idx] = rng.standard_normal(parts[k].idx.size)
        z = ras(lev.L @ e)
        np.testing.assert_allclose(z[parts[k].own_global], e[parts[k].own_global], rtol=1e-9, atol=1e-9)


def test_ras_box_geometry():
    assert schwarz.level_box(16, 8, 2) == (8, 2)
    assert schwarz.level_box(8, 8, 2) == (4, 1)
    p = schwarz.patches(16, 8, 2)[0]
    m = 12
    assert p.idx.size == m * m + 2 * m * (m + 1)
    assert p.own_global.size == 3 * 64


class _ExactSC(schur.SchurSmoother):
    def __init__(self, level):
        self.n = level.N * level.N
        self.G, self.D = level.G, level.D
        self.Ainv = np.linalg.inv(level.A_ib.toarray())
        self.Mexact = self.D.toarray() @ self.Ainv @ self.G.toarray()

    def A_tilde_inv(self, r):
        return self.Ainv @ r

    def M_tilde_inv(self, s):
        y = np.linalg.lstsq(self.Mexact, s, rcond=None)[0]
        return y - y.mean()


def test_sc_with_exact_inner_solves_is_exact_inverse():
    wl = W.plain_32(rho=1.0, mu=0.05)
    lev = hierarchy.build(wl)[1]   # 16 x 16 level
    sc = _ExactSC(lev)
    rng = np.random.default_rng(6)
    r = hierarchy.project_range(rng.standard_normal(lev.n), lev.N, 1.0)
    z = sc(r)
    np.testing.assert_allclose(lev.L @ z, r, atol=1e-8 * np.abs(r).max())


def test_chebyshev_closed_form():
    lam = np.linspace(0.2, 3.0, 25)
    b = np.random.default_rng(7).standard_normal(lam.size)
    lmin, lmax = 0.15, 3.3
    th, de = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    for its in (1, 2, 3, 5):
        x = schur.chebyshev(lambda v: lam * v, lambda v: v, b, lmin, lmax, its)
        Tk = np.polynomial.chebyshev.Chebyshev.basis(its)
        res = Tk((th - lam) / de) / Tk(th / de)
        np.testing.assert_allclose(x, (1 - res) / lam * b, rtol=1e-12, atol=1e-13)


def test_sgs_matches_triangular_sweeps_and_colouring():
    rng = np.random.default_rng(8)
    n = 30
    B = rng.standard_normal((n, n))
    A = B @ B.T + n * np.eye(n)
    b = rng.standard_normal(n)
    cols = schur.greedy_colouring(sp.csr_matrix(np.ones((n, n))))
    assert np.array_equal(cols, np.arange(n))
    x = schur.SGS(sp.csr_matrix(A), cols)(b)
    Lw = np.tril(A)
    Up = np.triu(A)
    x1 = la.solve_triangular(Lw, b, lower=True)
    x2 = x1 + la.solve_triangular(Up, b - A @ x1, lower=False)
    np.testing.assert_allclose(x, x2, rtol=1e-12)
    # proper colouring on a stencil pattern, spectrum of SGS^{-1} A in (0, 1]
    N = 10
    P = mac.stencil_pattern(N)
    c = schur.greedy_colouring(P)
    P = P.tocoo()
    off = P.row != P.col
    assert np.all(c[P.row[off]] != c[P.col[off]])
    A2 = (np.eye(N * N) * 4.5 - (P.toarray() - np.eye(N * N)))
    S = schur.SGS(sp.csr_matrix(A2), c)
    E = np.stack([S(A2[:, i]) for i in range(N * N)], 1)
    ev = np.linalg.eigvals(E).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12


def test_arnoldi_exact_for_few_eigenvalues():
    lam = np.repeat([0.5, 1.0, 2.5, 4.0], 10)
    v0 = schur.weyl_vector(lam.size)
    assert abs(krylov.arnoldi_ritz_max(lambda v: lam * v, v0, 10) - 4.0) < 1e-10


def test_bordered_coarse_solve():
    wl = W.plain_32()
    lev = hierarchy.build(wl)[0]
    cs = CoarseSolver(lev, wl.rho)
    rng = np.random.default_rng(9)
    r = rng.standard_normal(lev.n)
    x = cs(r)
    C = hierarchy.null_space(lev.N, wl.rho)
    np.testing.assert_allclose(C.T @ x, 0, atol=1e-10)
    rp = hierarchy.project_range(r, lev.N, wl.rho)
    np.testing.assert_allclose(lev.L @ x, rp, atol=1e-9)


def _dense_solve(L, b, N, rho):
    C = hierarchy.null_space(N, rho)
    k = C.shape[1]
    B = np.block([[L.toarray(), C], [C.T, np.zeros((k, k))]])
    return np.linalg.solve(B, np.concatenate([b, np.zeros(k)]))[:L.shape[0]]


def test_fgmres_vcycle_matches_dense_solve():
    for sm in ("ras", "sc"):
        wl = W.plain_32(smoother=sm)
        P = Problem(wl)
        b = W.rhs(wl.N, 0)
        x, info = P.solve(b, rtol=1e-11)
        assert info["converged"] and info["rel_res_true"] < 1e-10
        xd = _dense_solve(P.L, P.project(b), wl.N, wl.rho)
        assert np.linalg.norm(x - xd) / np.linalg.norm(xd) < 1e-9
        x8, info8 = P.solve(b, rtol=1e-8)
        assert info8["rel_res_true"] < 1.5e-8 and info8["iters"] <= 15


def test_spring_gradient_matches_central_differences():
    N = 16
    X, S = W.membrane(20, 0.22)
    kap = 50.0 * (1 + 0.5 * np.random.default_rng(1).uniform(-1, 1, S.shape[0]))
    wl = W.Workload("g", N, 8, 0.0, 1.0, 1e-2, X, S, kap)
    b = hierarchy.project_range(W.rhs(N, 0), N, 0.0)
    ut = hierarchy.project_range(W.rhs(N, 5), N, 0.0)
    n = N * N

    def loss(k):
        wl2 = W.Workload("g", N, 8, 0.0, 1.0, 1e-2, X, S, k)
        L = hierarchy.build(wl2)[-1].L
        w = _dense_solve(L, b, N, 0.0)
        return 0.5 * np.sum((w[:2 * n] - ut[:2 * n]) ** 2), w, L

    f0, w, L = loss(kap)
    g_rhs = np.zeros(3 * n)
    g_rhs[:2 * n] = w[:2 * n] - ut[:2 * n]
    lam = _dense_solve(L.T.tocsr(), hierarchy.project_range(g_rhs, N, 0.0), N, 0.0)
    g = spring_gradient(wl, w, lam)
    for e in (0, 7, 13):
        step = 1e-4 * kap[e]
        kp, km = kap.copy(), kap.copy()
        kp[e] += step
        km[e] -= step
        fd = (loss(kp)[0] - loss(km)[0]) / (2 * step)
        assert abs(fd - g[e]) <= 1e-6 * abs(fd) + 1e-12, (e, fd, g[e])


def test_ras_owned_set_reading():
    """Owned set of a box: its b x b cells' pressures, left x-faces and bottom
    y-faces (each face belongs to the cell on its right / above)."""
    N, b = 16, 8
    n = N * N
    for k, p in enumerate(schwarz.patches(N, b, 2)):
        pi, pj = k % (N // b), k // (N // b)
        jj, ii = np.meshgrid(np.arange(pj * b, pj * b + b), np.arange(pi * b, pi * b + b), indexing="ij")
        cells = (jj * N + ii).ravel()
        np.testing.assert_array_equal(np.sort(p.own_global),
                                      np.sort(np.concatenate([cells, n + cells, 2 * n + cells])))


def test_vcycle_iterations_match_paper_statement():
    """Sec. 5.2.1: a relative tolerance of 1e-6 takes 4-5 multigrid
    iterations in all but the most difficult cases (additive Schwarz, low
    Reynolds number).  The Stokes systems here are such easy cases."""
    for wl in (W.plain_32(), W.smoother_256(1e4, "ras", N=64)):
        P = Problem(wl)
        _, info = P.solve(W.rhs(wl.N, 0), rtol=1e-6)
        assert info["iters"] <= 5, (wl.name, info["iters"])
