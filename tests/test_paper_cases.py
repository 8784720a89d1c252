"""Pins of the results-section test structures (Sec. 5.1 thick shell, Sec. 5.2
thin membrane) and of the parameter-study driver's host logic.

* point counts M1 = 19 N / 8, M2 = 3 N / 32 + 1 give node spacings of about
  2/3 h along and across the fibres, as the paper states;
* the spring stiffnesses reproduce the paper's force density: the nodal
  springs' force divided by the nodal weight (ds1 ds2 for the shell, ds1 for
  the membrane) converges at second order to alpha d^2X/ds1^2, which for the
  circles of Eqs. annulus and circle is -alpha (r + s2)(cos s1, sin s1), with
  alpha = gamma 3.93/0.005 (thick) and 7 gamma 3.93/0.005 (thin);
* the background flow is discretely divergence-free (the oracle's MAC
  divergence) and samples the unit-speed cell flow to O(h^2);
* dt = 0.32 h and an 8 x 8 coarsest grid.
"""
import numpy as np
import pytest

import workloads as W
from oracle.mac import divergence
from oracle.timestep import fibre_force_periodic
from paper_1612_02208_amd import sweep


@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_point_counts_and_spacing(N):
    M1, M2 = W.paper_counts(N)
    assert (M1, M2) == (19 * N // 8, 3 * N // 32 + 1)
    X, S, kap, (ds1, ds2) = W.thick_shell(N, 5.0)
    assert X.shape == (M1 * M2, 2) and S.shape == (M1 * M2, 2)
    h = 1.0 / N
    # neighbours along the inner fibre and across the shell
    along = np.linalg.norm(X[1] - X[0])
    across = np.linalg.norm(X[M1] - X[0])
    assert abs(along / h - 2 / 3) < 0.01 and abs(across / h - 2 / 3) < 1e-12
    # every fibre is closed, and no spring joins two fibres
    assert np.all(S[:, 0] // M1 == S[:, 1] // M1)
    Xt, St, kt, _ = W.thin_membrane(N, 5.0)
    assert Xt.shape == (M1, 2) and St.shape == (M1, 2)
    r = np.linalg.norm(Xt - 0.5, axis=1)
    assert np.allclose(r, 0.25, atol=1e-15)


def test_counts_need_multiples_of_32():
    with pytest.raises(ValueError):
        W.paper_counts(48)


def _force_density_error(N, structure, gamma):
    if structure == "thick":
        X, S, kap, (ds1, ds2) = W.thick_shell(N, gamma)
        weight = ds1 * ds2
        alpha = gamma * 3.93 / 0.005
    else:
        X, S, kap, ds1 = W.thin_membrane(N, gamma)
        weight = ds1
        alpha = 7 * gamma * 3.93 / 0.005
    F = fibre_force_periodic(X, S, kap) / weight
    d = X - 0.5
    exact = -alpha * d             # alpha d^2/ds1^2 of c + R (cos s1, sin s1)
    return np.abs(F - exact).max() / np.abs(exact).max(), ds1


@pytest.mark.parametrize("structure", ["thick", "thin"])
def test_spring_stiffness_reproduces_the_force_density(structure):
    e64, d64 = _force_density_error(64, structure, 50.0)
    e128, d128 = _force_density_error(128, structure, 50.0)
    # the centred second difference of cos / sin has relative error
    # 1 - 4 sin^2(ds/2) / ds^2 = ds^2 / 12 + O(ds^4)
    assert abs(e64 / (d64 ** 2 / 12) - 1) < 1e-3
    assert abs(e128 / e64 - 0.25) < 1e-3


def test_thin_is_seven_times_the_shell_per_unit_thickness():
    """The membrane's alpha is 7 gamma 3.93/0.005; the shell's per-fibre spring
    is alpha ds2 / ds1 with the same gamma."""
    N, g = 128, 5.0
    _, _, kt, (ds1, ds2) = W.thick_shell(N, g)
    _, _, km, ds1m = W.thin_membrane(N, g)
    assert ds1 == ds1m
    assert np.isclose(km[0] * ds1, 7.0 * kt[0] * ds1 / ds2, rtol=1e-14)


@pytest.mark.parametrize("N", [32, 64])
def test_background_flow_is_divergence_free(N):
    b = W.background_flow(N)
    n = N * N
    assert np.abs(divergence(N) @ b[:2 * n]).max() < 1e-12 * N
    assert np.all(b[2 * n:] == 0)
    h = 1.0 / N
    x = np.arange(N) * h
    yc = (np.arange(N) + 0.5) * h
    u = b[:n].reshape(N, N)
    exact = np.outer(np.cos(2 * np.pi * yc), np.sin(2 * np.pi * x))   # u[j, i] at (i h, (j+1/2) h)
    assert np.abs(u - exact).max() < (2 * np.pi * h) ** 2 / 24 * 1.01


def test_paper_case_parameters():
    wl = W.paper_case("thick", 128, 500.0, "mu0.01", "rms", 16, 4)
    assert wl.dt == 0.32 / 128 and wl.coarse_N == 8 and wl.levels == 5
    assert (wl.rho, wl.mu) == (1.0, 0.01)
    assert (wl.smoother, wl.box, wl.overlap) == ("rms", 16, 4)
    st = W.paper_case("thin", 64, 5.0, "stokes", "sc")
    assert (st.rho, st.mu) == (0.0, 1.0) and st.name == "thin_N64_g5_stokes_sc"
    with pytest.raises(ValueError):
        W.paper_case("disc", 64, 5.0)


def test_study_lists():
    assert len(sweep.study_cases("shell_boxes")) == 4 * 9 * 2
    assert len(sweep.study_cases("shell_refine", (64, 128))) == 2 * 2 * 4 * 3 * 2
    assert len(sweep.study_cases("membrane_refine", (64,))) == 2 * 3 * 3
    assert all(c[4] == "sc" for c in sweep.study_cases("membrane_sc"))
    for s in sweep.STUDIES:
        for c in sweep.study_cases(s, (64,)):
            W.paper_case(*c)         # every case builds
    with pytest.raises(ValueError):
        sweep.study_cases("nope")


def test_summary_tables():
    assert sweep.iters_to([1e-2, 1e-5, 1e-7, 1e-13], 1e-6) == 3
    assert sweep.iters_to([1e-2], 1e-6) is None
    recs = []
    for sm in ("rms", "ras"):
        for b in sweep.BOXES:
            for o in sweep.OVERLAPS:
                recs.append(dict(structure="thick", N=128, gamma=500.0, flow="stokes", smoother=sm, box=b,
                                 overlap=o, status="OK", converged=True, iters=b + o, it_1e6=3))
    recs[0].update(status="NOT_CONVERGED", converged=False, iters=100)
    t = sweep.summary(recs)
    assert "| stokes | 4 | 100* (3) | 6 (3) | 8 (3) | 4 (3)" in t
    ref = [dict(structure="thin", N=N, gamma=5.0, flow="mu1", smoother="ras", box=16, overlap=4, status="OK",
                converged=True, iters=N // 16, it_1e6=2) for N in (64, 128)]
    t = sweep.summary(ref)
    assert "thin, RAS 16x16 boxes, overlap 4" in t and "| mu1 | 5 | 4 (2) | 8 (2) |" in t
