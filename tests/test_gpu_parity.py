"""GPU parity: every C-ABI call of libibmg against the plain FP64 oracle on the
same seeded inputs (FP64 library path).

Level vectors are compared row class by row class (IB velocity rows, other
velocity rows, pressure rows), each against its own norm (``_parity``).

Tolerances (relative, 2-norm per class) follow from the arithmetic:
* operators, transfers, spreading/interpolation: sums of <= ~60 terms of
  rounded products, so <= 1e-12 (a few hundred ulps) is a safe bound;
* solves (box inverses, the coarsest inverse, V-cycle, FGMRES): the library
  multiplies by explicit inverses while the oracle uses LU solves, so the
  difference scales with the conditioning of the local matrices; the bound is
  1e-10 relative, the figure the method is specified to.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import hierarchy, krylov, transfer
from oracle import ib as oib
from oracle.solver import Problem, spring_gradient
from _parity import assert_classes, face_classes, level_classes

pytestmark = pytest.mark.gpu

OPS_TOL = 1e-12
SOLVE_TOL = 1e-10


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lc(P, l=-1):
    lev = P.levels[l]
    return level_classes(lev.N, lev.T)


def _cases():
    # plain 32x32 Stokes membrane (3 levels)
    c1 = W.plain_32()
    # annulus at nonzero Reynolds number, ragged point count (4 rings x 150)
    X, S = W.annulus(4, 150, 0.2, 0.25)
    c2 = W.Workload("annulus_64", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4))
    # random points with random springs, odd sizes everywhere (coarse 6, N = 48)
    Xr = W.random_points(37, 21)
    rng = np.random.default_rng(5)
    Sr = np.stack([np.arange(37), (np.arange(37) + 1 + rng.integers(0, 5, 37)) % 37], 1).astype(np.int32)
    Sr = Sr[Sr[:, 0] != Sr[:, 1]]
    c3 = W.Workload("random_48", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, rng.uniform(10, 1e3, len(Sr)), box=6,
                    overlap=1)
    # large boxes (16 x 16 cells, overlap 4: 1776 unknowns per box)
    c4 = W.Workload("annulus_64_box16", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), box=16,
                    overlap=4)
    # a small membrane: most boxes are interior and share one inverse (the
    # matrix-core path), 2 tiles of 32 boxes with a ragged second tile
    Xs, Ss = W.membrane(40, 0.05, centre=(0.31, 0.62))
    c5 = W.Workload("small_64", 64, 8, 1.0, 0.1, 1e-3, Xs, Ss, np.full(len(Ss), 3e2), box=8, overlap=2)
    # Schur-complement smoother (Stokes membrane; annulus at nonzero Reynolds)
    c6 = W.plain_32(smoother="sc")
    c6.name = "plain_32_sc"
    c7 = W.Workload("annulus_64_sc", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), smoother="sc")
    # restricted multiplicative Schwarz (Alg. 3, colour-major box order): the
    # membrane, the annulus at nonzero Reynolds number, and random springs
    # whose long-range coupling needs up to 14 box colours
    c8 = W.plain_32(smoother="rms")
    c8.name = "plain_32_rms"
    c9 = W.Workload("annulus_64_rms", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), smoother="rms")
    c10 = W.Workload("random_48_rms", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, c3.kappa, box=6, overlap=1, smoother="rms")
    # tangent springs with rest lengths (2x2 blocks couple u and v): the
    # annulus with every spring stretched to 1/0.7 of its rest length, the
    # Stokes membrane with the Schur-complement smoother, and random springs
    # (rest lengths 0.3-0.9 of their lengths) with the multiplicative sweep
    def lengths(X, S):
        d = X[S[:, 1]] - X[S[:, 0]]
        d -= np.round(d)
        return np.hypot(d[:, 0], d[:, 1])
    c11 = W.Workload("annulus_64_tangent", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4),
                     spring_model="tangent", rest=0.7 * lengths(X, S))
    c12 = W.plain_32(smoother="sc", spring_model="tangent")
    c12.name, c12.rest = "plain_32_tangent_sc", 0.8 * lengths(c12.X, c12.springs)
    c13 = W.Workload("random_48_tangent_rms", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, c3.kappa, box=6, overlap=1,
                     smoother="rms", spring_model="tangent",
                     rest=lengths(Xr, Sr) * rng.uniform(0.3, 0.9, len(Sr)))
    # smoother options: the summed additive Schwarz combination (plain
    # R_k^T) and undamped Richardson sweeps (Sec. 6) with the restricted
    # additive, multiplicative and SC smoothers
    c14 = W.Workload("annulus_64_sum", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), combine="sum")
    c15 = W.plain_32(sweep="richardson")
    c15.name = "plain_32_richardson"
    c16 = W.Workload("annulus_64_sc_richardson", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4),
                     smoother="sc", sweep="richardson")
    c17 = W.Workload("random_48_rms_richardson", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, c3.kappa, box=6, overlap=1,
                     smoother="rms", sweep="richardson")
    c18 = W.Workload("random_48_sum_box16", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, c3.kappa, box=12, overlap=3,
                     combine="sum")
    return [c1, c2, c3, c4, c5, c6, c7, c8, c9, c10, c11, c12, c13, c14, c15, c16, c17, c18]


CASES = _cases()


@pytest.fixture(scope="module", params=range(len(CASES)), ids=[c.name for c in CASES])
def pair(request):
    from paper_1612_02208_amd import StokesIB
    wl = CASES[request.param]
    print(f"[case] {wl.name} N={wl.N} M={wl.M}", flush=True)
    P = Problem(wl)
    G = StokesIB(wl)
    yield wl, P, G
    G.close()


def test_apply_every_level(pair):
    wl, P, G = pair
    rng = np.random.default_rng(1)
    for l, lev in enumerate(P.levels):
        w = rng.uniform(-1, 1, lev.n)
        cl = lc(P, l)
        y = host(G.apply(dev(w), level=l))
        assert_classes(y, lev.L @ w, cl, OPS_TOL, f"apply level {l}")
        yt = host(G.apply(dev(w), level=l, transpose=True))
        assert_classes(yt, lev.L.T @ w, cl, OPS_TOL, f"apply_T level {l}")
        assert_classes(yt, y, cl, OPS_TOL, "symmetry")   # L_IB is symmetric (G = -D^T, S = J^*)


def test_spread_interp(pair):
    wl, P, G = pair
    rng = np.random.default_rng(2)
    N = wl.N
    F = rng.uniform(-1, 1, (wl.M, 2))
    f = host(G.spread(dev(F.ravel())))
    ref = np.concatenate([oib.spread_matrix(wl.X, N, c) @ F[:, c] for c in (0, 1)])
    touched = np.concatenate([np.asarray(oib.interp_pattern(wl.X, N, c).sum(0)).ravel() > 0 for c in (0, 1)])
    assert_classes(f, ref, face_classes(N, touched), OPS_TOL, "spread")
    u = rng.uniform(-1, 1, 2 * N * N)
    U = host(G.interp(dev(u))).reshape(-1, 2)
    for c in (0, 1):
        assert rel(U[:, c], oib.interp_matrix(wl.X, N, c) @ u[c * N * N:(c + 1) * N * N]) < OPS_TOL


def test_transfers(pair):
    wl, P, G = pair
    rng = np.random.default_rng(3)
    for l in range(1, len(P.levels)):
        Nc = P.levels[l - 1].N
        f = rng.uniform(-1, 1, P.levels[l].n)
        c = host(G.restrict(l, dev(f)))
        assert_classes(c, transfer.restriction(Nc) @ f, lc(P, l - 1), OPS_TOL, f"restrict {l}")
        e = rng.uniform(-1, 1, P.levels[l - 1].n)
        base = rng.uniform(-1, 1, P.levels[l].n)
        out = host(G.prolong_add(l, dev(e), dev(base)))
        assert_classes(out, base + transfer.prolongation(Nc) @ e, lc(P, l), OPS_TOL, f"prolong {l}")


def test_coarse_solve(pair):
    wl, P, G = pair
    rng = np.random.default_rng(4)
    r = rng.uniform(-1, 1, P.levels[0].n)
    x = host(G.coarse_solve(dev(r)))
    assert_classes(x, P.mg.coarse(r), lc(P, 0), SOLVE_TOL, "coarse solve")


def test_smoother_apply(pair):
    wl, P, G = pair
    rng = np.random.default_rng(6)
    for l in range(1, len(P.levels)):
        r = rng.uniform(-1, 1, P.levels[l].n)
        z = host(G.smoother_apply(l, dev(r)))
        assert_classes(z, P.mg.smoothers[l](r), lc(P, l), SOLVE_TOL, f"smoother level {l}")


def test_smooth(pair):
    wl, P, G = pair
    rng = np.random.default_rng(7)
    for l in range(1, len(P.levels)):
        lev = P.levels[l]
        w = rng.uniform(-1, 1, lev.n)
        b = rng.uniform(-1, 1, lev.n)
        out = host(G.smooth(l, dev(w), dev(b), 2))
        ref = P.mg.smooth(l, w, b, 2)   # the handle's sweep kind
        assert_classes(out, ref, lc(P, l), SOLVE_TOL, f"smooth level {l}")


def test_vcycle(pair):
    wl, P, G = pair
    r = P.project(W.rhs(wl.N, 11))
    z = host(G.vcycle(dev(r)))
    assert_classes(z, P.mg.vcycle(r), lc(P), SOLVE_TOL, "V-cycle")


def test_fgmres_fixed_iterations(pair):
    wl, P, G = pair
    b = W.rhs(wl.N, 0)
    bp = P.project(b)
    k = 4
    x, info = G.solve(dev(b), rtol=1e-300, restart=30, max_it=k)
    assert info["iters"] == k and info["status"] == "NOT_CONVERGED"
    xo, io = krylov.fgmres(P.apply, P.mg, bp, restart=30, rtol=1e-300, max_it=k)
    xo = P.project(xo)
    assert_classes(host(x), xo, lc(P), SOLVE_TOL, "FGMRES(30), 4 iterations")
    np.testing.assert_allclose(info["history"], np.array(io["history"][:k]) / np.linalg.norm(bp),
                               rtol=1e-8)


def test_fgmres_restarts_fixed_iterations(pair):
    """Restarted outer FGMRES: restart 3 for 8 iterations (cycles of 3, 3
    and 2 iterations, each from the true residual of the accumulated x)
    against the oracle's restarted FGMRES, iterate and residual history.
    Estimates that have reached the rounding floor (below 1e-11 of ||b||,
    where both sides hold noise) are only checked to lie there."""
    wl, P, G = pair
    b = W.rhs(wl.N, 0)
    bp = P.project(b)
    x, info = G.solve(dev(b), rtol=1e-300, restart=3, max_it=8)
    assert info["iters"] == 8 and info["restarts"] == 3 and info["status"] == "NOT_CONVERGED"
    xo, io = krylov.fgmres(P.apply, P.mg, bp, restart=3, rtol=1e-300, max_it=8)
    assert io["iters"] == 8
    assert_classes(host(x), P.project(xo), lc(P), SOLVE_TOL, "FGMRES(3), 8 iterations")
    hg = np.array(info["history"])
    ho = np.array(io["history"]) / np.linalg.norm(bp)
    floor = ho < 1e-11
    np.testing.assert_allclose(hg[~floor], ho[~floor], rtol=1e-8, atol=1e-14)
    assert np.all(hg[floor] < 1e-11)
    assert (~floor).sum() >= 4


def test_solve_to_tolerance(pair):
    wl, P, G = pair
    b = W.rhs(wl.N, 0)
    x, info = G.solve(dev(b), rtol=1e-8)
    assert info["converged"]
    xh = host(x)
    bp = P.project(b)
    true = np.linalg.norm(bp - P.L @ xh) / np.linalg.norm(bp)
    assert true <= 1.2e-8, true
    assert abs(info["rel_res_true"] - true) < 1e-10
    assert abs(info["rhs_null_norm"] - np.linalg.norm(b - bp)) < 1e-9 * np.linalg.norm(b)
    xo, io = P.solve(b, rtol=1e-8)
    assert abs(info["iters"] - io["iters"]) <= 1
    # both to 1e-12: the solutions agree to the conditioning of the system
    x12, i12 = G.solve(dev(b), rtol=1e-12, max_it=200)
    xo12, _ = P.solve(b, rtol=1e-12, max_it=200)
    assert_classes(host(x12), xo12, lc(P), SOLVE_TOL, "solutions at 1e-12")


def test_spring_gradient(pair):
    wl, P, G = pair
    rng = np.random.default_rng(8)
    n = P.fine.n
    w = rng.uniform(-1, 1, n)
    lam = rng.uniform(-1, 1, n)
    g = host(G.spring_gradient(dev(w), dev(lam)))
    assert rel(g, spring_gradient(wl, w, lam)) < OPS_TOL


def test_schur_setup_matches_oracle(pair):
    """Colour counts are equal and the Chebyshev bounds' Ritz values agree."""
    wl, P, G = pair
    if wl.smoother != "sc":
        pytest.skip("Schwarz smoother")
    for l in range(1, len(P.levels)):
        sm = P.mg.smoothers[l]
        info = G.sc_info(l)
        assert info["colours_u"] == int(sm.col_u.max()) + 1
        assert info["colours_p"] == int(sm.col_p.max()) + 1
        assert abs(info["lam_A"] - sm.lam_A) <= 1e-10 * abs(sm.lam_A)
        assert abs(info["lam_M"] - sm.lam_M) <= 1e-10 * abs(sm.lam_M)


def test_rms_colours_match_oracle(pair):
    """The multiplicative sweep's box colouring has the oracle's colour count
    on every level (the sweep results, compared above, need the same
    colours box by box)."""
    wl, P, G = pair
    if wl.smoother != "rms":
        pytest.skip("not the multiplicative smoother")
    st = G.stats()["levels"]
    for l in range(1, len(P.levels)):
        assert st[l]["box_colours"] == int(P.mg.smoothers[l].colour.max()) + 1, l


def test_single_kernel_timing_every_level(pair):
    """ibmg_kernel_time launches the Schwarz kernels over a level's whole box
    lists; on multiplicative-sweep levels that is more than one colour's
    range, so the interior product's slice buffer must hold it (the library
    checks this before every launch).  Algorithmic bytes and flops follow
    the box counts."""
    wl, P, G = pair
    if wl.smoother == "sc":
        pytest.skip("Schur-complement smoother")
    if wl.combine == "sum":
        with pytest.raises(Exception):
            G.kernel_time("ras_ib", len(P.levels) - 1, 1)
        pytest.skip("the restricted Schwarz kernels do not run with the summed combination")
    st = G.stats()["levels"]
    for l in range(1, len(P.levels)):
        lv = st[l]
        n_int = lv["boxes"] - lv["ib_boxes"]
        if lv["ib_boxes"]:
            t = G.kernel_time("ras_ib", l, 2)
            assert t["ms"] > 0 and t["bytes"] > 0
        if n_int:
            t = G.kernel_time("ras_interior", l, 2)
            assert t["ms"] > 0 and t["flops"] > 0
    # the handle still computes the oracle's smoother after the timing runs
    r = np.random.default_rng(12).uniform(-1, 1, P.levels[-1].n)
    z = host(G.smoother_apply(-1, dev(r)))
    assert_classes(z, P.mg.smoothers[-1](r), lc(P), SOLVE_TOL, "smoother after timing")


def test_krylov_kernel_timing(pair):
    """ibmg_kernel_time for the smoothing step's Krylov kernels (and the
    outer solve's second-pass pair) on every level: the basis at its largest
    (k = max(nu1, nu2) vectors of n = 3 N_l^2), bytes as documented; a solve
    afterwards still matches the oracle's."""
    wl, P, G = pair
    k = max(wl.nu1, wl.nu2)
    for l in range(1, len(P.levels)):
        n = P.levels[l].n
        for kind in ("apply_dots", "upd_dots", "scale_upd", "upd_norm", "combine_ls"):
            t = G.kernel_time(kind, l, 2)
            assert t["ms"] > 0 and t["bytes"] == 8.0 * (k + 2) * n, (kind, l)
        t = G.kernel_time("scale_red", l, 2)
        assert t["ms"] > 0 and t["bytes"] == 16.0 * n
    with pytest.raises(Exception):
        G.kernel_time("scale_upd", 0, 1)
    b = W.rhs(wl.N, 0)
    x, _ = G.solve(dev(b), rtol=1e-300, restart=30, max_it=4)
    xo, _ = krylov.fgmres(P.apply, P.mg, P.project(b), restart=30, rtol=1e-300, max_it=4)
    assert_classes(host(x), P.project(xo), lc(P), SOLVE_TOL, "FGMRES(30), 4 iterations after Krylov timing")


def test_transfer_and_coupling_kernel_timing(pair):
    """ibmg_kernel_time for the transfers on every level and for spreading
    and interpolation on the finest: algorithmic bytes follow the grid sizes
    and the structure's window entries, and the handle's results are
    unchanged afterwards."""
    wl, P, G = pair
    for l in range(1, len(P.levels)):
        nf, nc = P.levels[l].n, P.levels[l - 1].n
        t = G.kernel_time("restrict", l, 2)
        assert t["ms"] > 0 and t["bytes"] == 8.0 * (nf + nc)
        t = G.kernel_time("prolong", l, 2)
        assert t["ms"] > 0 and t["bytes"] == 8.0 * (nc + 2 * nf)
    N, M = wl.N, wl.M
    ents = sum(int(oib.interp_pattern(wl.X, N, c).nnz) for c in (0, 1))
    t = G.kernel_time("spread", -1, 2)
    assert t["ms"] > 0 and t["bytes"] == ents * 12.0 + 2 * (N * N + 1) * 4.0 + 2 * M * 8.0 + 2 * N * N * 8.0
    touched = sum(int((oib.interp_pattern(wl.X, N, c).sum(0) > 0).sum()) for c in (0, 1))
    t = G.kernel_time("interp", -1, 2)
    assert t["ms"] > 0 and t["bytes"] == 2 * M * 16 * 8.0 + 2 * M * 2 * 4.0 + touched * 8.0 + 2 * M * 8.0
    with pytest.raises(Exception):
        G.kernel_time("restrict", 0, 1)
    rng = np.random.default_rng(2)
    F = rng.uniform(-1, 1, (wl.M, 2))
    f = host(G.spread(dev(F.ravel())))
    ref = np.concatenate([oib.spread_matrix(wl.X, N, c) @ F[:, c] for c in (0, 1)])
    touched = np.concatenate([np.asarray(oib.interp_pattern(wl.X, N, c).sum(0)).ravel() > 0 for c in (0, 1)])
    assert_classes(f, ref, face_classes(N, touched), OPS_TOL, "spread after timing")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", ["small_64", "annulus_64_box16", "random_48_rms"])
def test_interior_product_forms_agree(name, precision, monkeypatch):
    """The interior-box product forms (pipelined 64-box tiles in XCD order,
    16- and 32-box tiles, 64 x 64 register blocks, gathered 64 x 128 tiles)
    use the same reduction slices and the same order of MFMA steps per
    output, so the smoother's result is bitwise the same whichever form a
    level runs; and it is the oracle's."""
    from paper_1612_02208_amd import StokesIB
    wl = [c for c in CASES if c.name == name][0]
    P = Problem(wl)
    r = np.random.default_rng(31).uniform(-1, 1, P.levels[-1].n)
    outs = {}
    for form in ("1", "16", "32", "64", "128"):
        monkeypatch.setenv("IBMG_INTERIOR_FORM", form)
        G = StokesIB(wl, precision=precision)
        outs[form] = host(G.smoother_apply(-1, dev(r)))
        G.close()
    for form, z in outs.items():
        assert np.array_equal(z, outs["32"]), form
    tol = SOLVE_TOL if precision == "fp64" else FP32_TOL
    assert_classes(outs["128"], P.mg.smoothers[-1](r), lc(P), tol, "interior forms")


# ---------------------------------------------------------------------------
# FP32-smoother handles (the precision form): every smoother-side call in
# FP32 against the FP64 oracle.  The FP32 path rounds its inputs, the box
# inverses, the Galerkin rows and every sum to binary32 (unit roundoff
# u = 2^-24 = 6e-8); a smoother application is a product with local inverses
# whose entries exceed the result by the local condition number, and a
# V-cycle chains those through the levels, so the bound is 1e-4 relative per
# row class (about 1700 u).  The solve itself keeps FGMRES and the residual in
# FP64, so run to 1e-12 it reaches the oracle's solution to the FP64 bound.
# ---------------------------------------------------------------------------
FP32_TOL = 1e-4
FP32_CASES = ["plain_32", "annulus_64_box16", "random_48", "plain_32_sc", "annulus_64_rms",
              "annulus_64_tangent", "annulus_64_sum", "plain_32_richardson"]


@pytest.fixture(scope="module", params=FP32_CASES)
def pair32(request):
    from paper_1612_02208_amd import StokesIB
    wl = [c for c in CASES if c.name == request.param][0]
    print(f"[case] fp32 {wl.name} N={wl.N} M={wl.M}", flush=True)
    P = Problem(wl)
    G = StokesIB(wl, precision="fp32")
    yield wl, P, G
    G.close()


def test_fp32_smoother_apply(pair32):
    wl, P, G = pair32
    rng = np.random.default_rng(6)
    for l in range(1, len(P.levels)):
        r = rng.uniform(-1, 1, P.levels[l].n)
        z = host(G.smoother_apply(l, dev(r)))
        e = assert_classes(z, P.mg.smoothers[l](r), lc(P, l), FP32_TOL, f"fp32 smoother level {l}")
        print(f"[fp32] {wl.name} smoother level {l}: {e}")


def test_fp32_smooth(pair32):
    wl, P, G = pair32
    rng = np.random.default_rng(7)
    for l in range(1, len(P.levels)):
        lev = P.levels[l]
        w = rng.uniform(-1, 1, lev.n)
        b = rng.uniform(-1, 1, lev.n)
        out = host(G.smooth(l, dev(w), dev(b), 2))
        ref = P.mg.smooth(l, w, b, 2)   # the handle's sweep kind
        e = assert_classes(out, ref, lc(P, l), FP32_TOL, f"fp32 smooth level {l}")
        print(f"[fp32] {wl.name} smooth level {l}: {e}")


def test_fp32_vcycle(pair32):
    wl, P, G = pair32
    r = P.project(W.rhs(wl.N, 11))
    z = host(G.vcycle(dev(r)))
    e = assert_classes(z, P.mg.vcycle(r), lc(P), FP32_TOL, "fp32 V-cycle")
    print(f"[fp32] {wl.name} V-cycle: {e}")


def test_fp32_solves_against_oracle(pair32):
    """To 1e-8 the FP32-smoother solve meets the tolerance by its true
    residual under the oracle's operator, and its distance to the oracle's
    1e-12 solution is recorded (bounded by the conditioning times 1e-8);
    to 1e-12 it reaches the oracle's 1e-12 solution to the FP64 bound."""
    wl, P, G = pair32
    b = W.rhs(wl.N, 0)
    bp = P.project(b)
    xo12, _ = P.solve(b, rtol=1e-12, max_it=200)
    x8, i8 = G.solve(dev(b), rtol=1e-8)
    assert i8["converged"]
    x8 = host(x8)
    assert np.linalg.norm(bp - P.L @ x8) <= 1.2e-8 * np.linalg.norm(bp)
    e8 = assert_classes(x8, xo12, lc(P), 1e-5, "fp32 solve at 1e-8 vs oracle at 1e-12")
    x12, i12 = G.solve(dev(b), rtol=1e-12, max_it=200)
    assert i12["converged"]
    e12 = assert_classes(host(x12), xo12, lc(P), SOLVE_TOL, "fp32 solve at 1e-12 vs oracle at 1e-12")
    print(f"[fp32] {wl.name} solve 1e-8 ({i8['iters']} its): {e8}; 1e-12 ({i12['iters']} its): {e12}")
