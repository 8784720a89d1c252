"""Pins for the oracle's staggered-grid operators (App. A.1, Eq. matrix-impib).

* G = -D^T exactly (discrete gradient and divergence are negative adjoints).
* The five-point Laplacian's eigenvalues on Fourier modes are
  -(4/h^2)(sin^2(pi k/N) + sin^2(pi l/N)).
* A discrete stream function gives an exactly divergence-free face field.
* Smooth periodic fields: A u + G p and D u converge at second order to the
  continuous rho/dt u - mu Lap u + grad p and div u at the staggered points.
* With no structure the periodic Stokes system diagonalises by the DFT into
  one 3x3 system per mode; the oracle operator reproduces that solution.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle import hierarchy, mac


def test_gradient_is_minus_divergence_transpose():
    for N in (4, 8, 13):
        G = mac.gradient(N).toarray()
        D = mac.divergence(N).toarray()
        np.testing.assert_array_equal(G, -D.T)


def test_laplacian_fourier_symbol():
    N = 12
    h = 1.0 / N
    L = mac.scalar_laplacian(N)
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    for k, l in [(0, 0), (1, 0), (3, 5), (6, 6), (11, 2)]:
        mode = np.exp(2j * np.pi * (k * i + l * j) / N).ravel()
        lam = -(4 / h ** 2) * (np.sin(np.pi * k / N) ** 2 + np.sin(np.pi * l / N) ** 2)
        np.testing.assert_allclose(L @ mode, lam * mode, atol=1e-9 * max(1, abs(lam)))


def test_stream_function_is_divergence_free():
    N = 16
    h = 1.0 / N
    rng = np.random.default_rng(4)
    psi = rng.standard_normal((N, N))   # psi at nodes (i h, j h), indexed [j, i]
    u = (np.roll(psi, -1, axis=0) - psi) / h         # x-face (i, j+1/2)
    v = -(np.roll(psi, -1, axis=1) - psi) / h        # y-face (i+1/2, j)
    D = mac.divergence(N)
    div = D @ np.concatenate([u.ravel(), v.ravel()])
    assert np.max(np.abs(div)) < 1e-10 * np.max(np.abs(u))


def _manufactured_errors(N, rho=1.0, mu=0.7, dt=0.1):
    h = 1.0 / N
    tp = 2 * np.pi
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    xu, yu = i * h, (j + 0.5) * h
    xv, yv = (i + 0.5) * h, j * h
    xc, yc = (i + 0.5) * h, (j + 0.5) * h

    def U(x, y):
        return np.sin(tp * x) * np.cos(tp * y)

    def V(x, y):
        return -np.cos(tp * x) * np.sin(tp * y) + 0.3 * np.sin(tp * x)

    def P(x, y):
        return np.sin(tp * x) * np.sin(2 * tp * y)

    w = np.concatenate([U(xu, yu).ravel(), V(xv, yv).ravel(), P(xc, yc).ravel()])
    A = mac.momentum(N, rho, mu, dt)
    G = mac.gradient(N)
    D = mac.divergence(N)
    n = N * N
    out_u = A @ w[:2 * n] + G @ w[2 * n:]
    # continuous: rho/dt u - mu Lap u + grad p ; Lap U = -2 tp^2 U
    lapU = -2 * tp ** 2 * U(xu, yu)
    lapV = -2 * tp ** 2 * (-np.cos(tp * xv) * np.sin(tp * yv)) - tp ** 2 * 0.3 * np.sin(tp * xv)
    px = tp * np.cos(tp * xu) * np.sin(2 * tp * yu)
    py = 2 * tp * np.sin(tp * xv) * np.cos(2 * tp * yv)
    ex_u = rho / dt * U(xu, yu) - mu * lapU + px
    ex_v = rho / dt * V(xv, yv) - mu * lapV + py
    err_mom = np.max(np.abs(out_u - np.concatenate([ex_u.ravel(), ex_v.ravel()])))
    # divergence of a non-solenoidal field (U, W), W = 0.3 sin(tp x) cos(2 tp y)
    Wv = 0.3 * np.sin(tp * xv) * np.cos(2 * tp * yv)
    ex_div = tp * np.cos(tp * xc) * np.cos(tp * yc) - 0.6 * tp * np.sin(tp * xc) * np.sin(2 * tp * yc)
    err_div = np.max(np.abs(D @ np.concatenate([U(xu, yu).ravel(), Wv.ravel()]) - ex_div.ravel()))
    return err_mom, err_div


def test_manufactured_second_order():
    e1 = _manufactured_errors(16)
    e2 = _manufactured_errors(32)
    e3 = _manufactured_errors(64)
    for k in (0, 1):
        r1 = np.log2(e1[k] / e2[k])
        r2 = np.log2(e2[k] / e3[k])
        assert 1.9 < r1 < 2.2 and 1.9 < r2 < 2.2, (k, r1, r2)


def _fft_stokes(N, rho, mu, dt, b):
    """Exact solution of the periodic MAC Stokes system mode by mode."""
    h = 1.0 / N
    n = N * N
    bu = np.fft.fft2(b[:n].reshape(N, N))
    bv = np.fft.fft2(b[n:2 * n].reshape(N, N))
    bp = np.fft.fft2(b[2 * n:].reshape(N, N))
    l, k = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")   # axis0 = j (y)
    tk = 2 * np.pi * k / N
    tl = 2 * np.pi * l / N
    a = rho / dt + mu * (4 / h ** 2) * (np.sin(tk / 2) ** 2 + np.sin(tl / 2) ** 2)
    gx = (1 - np.exp(-1j * tk)) / h     # (p_i - p_{i-1}) / h
    gy = (1 - np.exp(-1j * tl)) / h
    dx = (np.exp(1j * tk) - 1) / h      # (u_{i+1} - u_i) / h
    dy = (np.exp(1j * tl) - 1) / h
    U = np.zeros_like(bu)
    V = np.zeros_like(bu)
    Pm = np.zeros_like(bu)
    for jj in range(N):
        for ii in range(N):
            if ii == 0 and jj == 0:
                if a[0, 0] != 0:
                    U[0, 0] = bu[0, 0] / a[0, 0]
                    V[0, 0] = bv[0, 0] / a[0, 0]
                continue
            Mx = np.array([[a[jj, ii], 0, gx[jj, ii]],
                           [0, a[jj, ii], gy[jj, ii]],
                           [-dx[jj, ii], -dy[jj, ii], 0]], dtype=complex)
            s = np.linalg.solve(Mx, np.array([bu[jj, ii], bv[jj, ii], bp[jj, ii]]))
            U[jj, ii], V[jj, ii], Pm[jj, ii] = s
    return np.concatenate([np.fft.ifft2(U).real.ravel(), np.fft.ifft2(V).real.ravel(),
                           np.fft.ifft2(Pm).real.ravel()])


def test_stokes_operator_matches_fft_solution():
    for N, rho in ((16, 0.0), (16, 1.0), (24, 1.0)):
        mu, dt = 0.3, 0.05
        rng = np.random.default_rng(N)
        b = hierarchy.project_range(rng.uniform(-1, 1, 3 * N * N), N, rho)
        w = _fft_stokes(N, rho, mu, dt, b)
        A = mac.momentum(N, rho, mu, dt)
        L = mac.stokes_ib(A, mac.gradient(N), mac.divergence(N))
        res = L @ w - b
        assert np.linalg.norm(res) < 1e-10 * np.linalg.norm(b) * N * N
        # and the sparse direct solve of the bordered system agrees with the FFT
        C = hierarchy.null_space(N, rho)
        import scipy.sparse as sp
        k = C.shape[1]
        B = sp.bmat([[L, sp.csr_matrix(C)], [sp.csr_matrix(C.T), None]], format="csc")
        x = spla.spsolve(B, np.concatenate([b, np.zeros(k)]))[:3 * N * N]
        np.testing.assert_allclose(x, w, atol=1e-10 * np.max(np.abs(w)))
