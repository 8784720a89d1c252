"""Pins for the oracle's smoother options: the summed additive Schwarz
combination (plain R_k^T in place of Alg. 2's restricted R~_k^T) and
Richardson smoothing sweeps (the Sec. 6 reading of the large-box Vanka
smoother as a Richardson iteration, next to Sec. 3.3's FGMRES wrapping).

Each pin is fixed by something other than the oracle's own code:
* with L = I every local solve returns its restriction, so the summed
  smoother multiplies each unknown by the number of boxes holding it, a
  count written here from the box geometry alone (the restricted one is the
  identity: the owned sets partition the unknowns);
* for a symmetric L (L_IB is, G = -D^T) the summed smoother
  sum_k R_k^T L_k^{-1} R_k is symmetric and the restricted one is not;
* the two combinations agree on every unknown held by exactly one box;
* Richardson: the error after nu steps is (I - B A)^nu e_0 (closed form by
  matrix powers), an exact B makes one step exact, and a V-cycle with
  Richardson sweeps inside FGMRES reaches the dense direct solution.
"""
import numpy as np
import scipy.linalg as la
import scipy.sparse as sp

import workloads as W
from oracle import hierarchy, krylov, schwarz
from oracle.solver import Problem


def _cover_counts(N, box, overlap):
    """Boxes whose enlarged region holds each unknown, counted per axis from
    the geometry: box bx spans coordinates bx b - o + [0, ext) (mod N), with
    ext = m + 1 along a face's normal and m otherwise."""
    b, o = schwarz.level_box(N, box, overlap)
    m = b + 2 * o
    npd = N // b

    def along(coord, ext):
        return sum(1 for bx in range(npd) if (coord - (bx * b - o)) % N < ext)

    n = N * N
    c = np.zeros(3 * n)
    for j in range(N):
        for i in range(N):
            q = j * N + i
            c[q] = along(i, m + 1) * along(j, m)            # x-face
            c[n + q] = along(i, m) * along(j, m + 1)        # y-face
            c[2 * n + q] = along(i, m) * along(j, m)        # cell
    return c


def test_summed_schwarz_with_identity_counts_the_covering_boxes():
    rng = np.random.default_rng(41)
    for N, box, overlap in ((16, 4, 1), (32, 8, 2), (24, 6, 0), (16, 8, 3)):
        I = sp.identity(3 * N * N, format="csr")
        r = rng.standard_normal(3 * N * N)
        zs = schwarz.RAS(I, N, box, overlap, combine="sum")(r)
        np.testing.assert_allclose(zs, _cover_counts(N, box, overlap) * r, rtol=1e-14, atol=1e-14)
        zr = schwarz.RAS(I, N, box, overlap)(r)
        np.testing.assert_allclose(zr, r, rtol=1e-14, atol=1e-14)


def test_summed_schwarz_is_symmetric_and_agrees_on_single_cover():
    wl = W.plain_32(box=8, overlap=2)
    lev = hierarchy.build(wl)[-1]
    L = lev.L
    assert abs(L - L.T).max() < 1e-12 * abs(L).max()
    S = schwarz.RAS(L, lev.N, wl.box, wl.overlap, combine="sum")
    R = schwarz.RAS(L, lev.N, wl.box, wl.overlap)
    rng = np.random.default_rng(42)
    x, y = rng.standard_normal(lev.n), rng.standard_normal(lev.n)
    assert abs(x @ S(y) - y @ S(x)) <= 1e-10 * abs(x @ S(y))
    assert abs(x @ R(y) - y @ R(x)) > 1e-6 * abs(x @ R(y))
    single = _cover_counts(lev.N, wl.box, wl.overlap) == 1
    assert single.any() and not single.all()
    np.testing.assert_allclose(S(y)[single], R(y)[single], rtol=1e-12, atol=1e-12)


def test_richardson_error_propagation():
    rng = np.random.default_rng(43)
    n = 30
    A = np.diag(np.linspace(1.0, 4.0, n)) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    B = np.diag(1.0 / np.diag(A)) * 0.9
    xs = rng.standard_normal(n)
    b = A @ xs
    w0 = rng.standard_normal(n)
    for nu in (1, 2, 5):
        w = krylov.richardson_smooth(lambda v: A @ v, lambda v: B @ v, w0, b, nu)
        E = np.linalg.matrix_power(np.eye(n) - B @ A, nu)
        np.testing.assert_allclose(w - xs, E @ (w0 - xs), rtol=1e-10, atol=1e-12)
    Ainv = np.linalg.inv(A)
    w = krylov.richardson_smooth(lambda v: A @ v, lambda v: Ainv @ v, w0, b, 1)
    np.testing.assert_allclose(w, xs, rtol=1e-10, atol=1e-12)


def test_vcycle_options_reach_direct_solution():
    """Richardson sweeps with the restricted additive Schwarz and the SC
    smoothers, and the summed combination inside FGMRES sweeps.  (Undamped
    Richardson with the summed combination diverges: overlapping boxes add
    their corrections, which over-corrects.)"""
    for sm, combine, sweep in (("ras", "restricted", "richardson"), ("sc", "restricted", "richardson"),
                               ("ras", "sum", "fgmres")):
        wl = W.plain_32(smoother=sm, sweep=sweep, combine=combine)
        P = Problem(wl)
        b = W.rhs(wl.N, 0)
        x, info = P.solve(b, rtol=1e-10, max_it=100)
        assert info["converged"], (sm, combine)
        bp = P.project(b)
        C = hierarchy.null_space(wl.N, wl.rho)
        k = C.shape[1]
        Lb = np.block([[P.L.toarray(), C], [C.T, np.zeros((k, k))]])
        xd = la.solve(Lb, np.concatenate([bp, np.zeros(k)]))[:P.fine.n]
        assert np.linalg.norm(x - xd) <= 1e-8 * np.linalg.norm(xd), (sm, combine)
        # the option changes the V-cycle
        wf = W.plain_32(smoother=sm)
        Pf = Problem(wf)
        r = P.project(W.rhs(wl.N, 3))
        assert np.linalg.norm(P.mg.vcycle(r) - Pf.mg.vcycle(r)) > 1e-6 * np.linalg.norm(Pf.mg.vcycle(r))
