"""Pins of the oracle's restricted multiplicative Schwarz smoother (Alg. 3)
against properties the algorithm and the paper fix:

* the box colouring satisfies its defining condition (no coupling of a
  box's rows to another same-colour box's owned unknowns), checked on the
  assembled operator block by block;
* within a colour the visiting order does not change the sweep, which is
  what lets a colour be updated at once;
* an exact solution is a fixed point of the sweep;
* the sweep is multiplicative: it differs from the additive sweep (the
  residual is refreshed between boxes);
* in the paper's harder regime (nonzero Reynolds number, small overlap) the
  multiplicative smoother needs no more FGMRES iterations than the additive
  one, and fewer without overlap (Sec. 5.1.1).
"""
import numpy as np
import pytest
import scipy.linalg as la

import workloads as W
from oracle import hierarchy
from oracle.schwarz import RAS, RMS, structural_pattern
from oracle.solver import Problem


def _annulus(smoother, box, overlap, N=64):
    X, S = W.annulus(4, 150, 0.2, 0.25)
    return W.Workload(f"annulus_{N}", N, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), smoother=smoother,
                      box=box, overlap=overlap)


def _random48():
    Xr = W.random_points(37, 21)
    rng = np.random.default_rng(5)
    Sr = np.stack([np.arange(37), (np.arange(37) + 1 + rng.integers(0, 5, 37)) % 37], 1).astype(np.int32)
    Sr = Sr[Sr[:, 0] != Sr[:, 1]]
    return W.Workload("random_48", 48, 6, 0.0, 0.3, 2e-2, Xr, Sr, rng.uniform(10, 1e3, len(Sr)), box=6, overlap=1,
                      smoother="rms")


@pytest.fixture(scope="module")
def levels_random():
    return hierarchy.build(_random48())


def test_colouring_condition_on_assembled_blocks(levels_random):
    wl = _random48()
    for lev in levels_random[1:]:
        P = structural_pattern(lev)
        # the pattern covers every nonzero of L
        Ld = abs(lev.L).tocsr()
        assert (Ld - Ld.multiply(P)).count_nonzero() == 0
        sm = RMS(lev.L, P, lev.N, wl.box, wl.overlap)
        Pc = P.tocsr()
        for c in range(sm.colour.max() + 1):
            boxes = np.flatnonzero(sm.colour == c)
            for i in boxes:
                for j in boxes:
                    if i == j:
                        continue
                    blk = Pc[sm.parts[j].idx][:, sm.parts[i].own_global]
                    assert blk.count_nonzero() == 0, (lev.N, c, i, j)


def test_random_springs_need_more_colours(levels_random):
    wl = _random48()
    counts = [RMS(l.L, structural_pattern(l), l.N, wl.box, wl.overlap).colour.max() + 1 for l in levels_random[1:]]
    assert max(counts) > 4   # long springs couple distant boxes


def test_order_within_a_colour_does_not_matter(levels_random):
    wl = _random48()
    lev = levels_random[-1]
    sm = RMS(lev.L, structural_pattern(lev), lev.N, wl.box, wl.overlap)
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, lev.n)
    w0 = rng.uniform(-1, 1, lev.n)
    ref = sm.sweep(w0, b)
    order = []
    for c in range(sm.colour.max() + 1):
        boxes = list(np.flatnonzero(sm.colour == c))
        rng.shuffle(boxes)
        order += boxes
    alt = sm.sweep(w0, b, order=order)
    assert np.linalg.norm(alt - ref) <= 1e-12 * np.linalg.norm(ref)
    # across colours the order does matter (the sweep is multiplicative)
    rev = sm.sweep(w0, b, order=order[::-1])
    assert np.linalg.norm(rev - ref) > 1e-6 * np.linalg.norm(ref)


def test_exact_solution_is_a_fixed_point():
    wl = W.plain_32(smoother="rms")
    P = Problem(wl)
    lev = P.fine
    sm = P.mg.smoothers[-1]
    b = P.project(W.rhs(wl.N, 4))
    C = hierarchy.null_space(lev.N, wl.rho)
    k = C.shape[1]
    B = np.block([[lev.L.toarray(), C], [C.T, np.zeros((k, k))]])
    w = la.solve(B, np.concatenate([b, np.zeros(k)]))[:lev.n]
    assert np.linalg.norm(b - lev.L @ w) < 1e-10 * np.linalg.norm(b)
    out = sm.sweep(w, b)
    assert np.linalg.norm(out - w) <= 1e-9 * np.linalg.norm(w)


def test_multiplicative_differs_from_additive():
    wl = W.plain_32(smoother="rms")
    P = Problem(wl)
    lev = P.fine
    rms = P.mg.smoothers[-1]
    ras = RAS(lev.L, lev.N, wl.box, wl.overlap)
    r = P.project(W.rhs(wl.N, 9))
    a, m = ras(r), rms(r)
    # the first colour's boxes see the plain residual in both sweeps
    first = np.concatenate([rms.parts[k].own_global for k in np.flatnonzero(rms.colour == 0)])
    assert np.allclose(a[first], m[first], rtol=1e-12, atol=1e-14)
    assert np.linalg.norm(a - m) > 1e-3 * np.linalg.norm(a)


def test_multiplicative_needs_no_more_iterations_than_additive():
    b = W.rhs(64, 0)
    its = {}
    for sm in ("ras", "rms"):
        for ov in (0, 2):
            _, info = Problem(_annulus(sm, 8, ov)).solve(b, rtol=1e-8, max_it=200)
            its[sm, ov] = info["iters"]
    assert its["rms", 2] <= its["ras", 2]
    assert its["rms", 0] < its["ras", 0]
