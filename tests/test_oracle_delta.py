"""Pins for the oracle's four-point kernel (App. A.3).

The closed-form values come from evaluating the printed piecewise formula by
hand (tests/golden/phi_values.txt).  The moment identities are the defining
properties of Peskin's four-point function: for every shift r,
sum_j phi(r - j) = 1, sum_j (r - j) phi(r - j) = 0, sum_j phi(r - j)^2 = 3/8,
and the even and odd sums are each 1/2.
"""
import os

import numpy as np
import pytest

from oracle.delta import delta_h, phi

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "phi_values.txt")


def test_phi_closed_form_values():
    data = np.loadtxt(GOLDEN)
    np.testing.assert_allclose(phi(data[:, 0]), data[:, 1], rtol=0, atol=2e-16)


def test_phi_support_and_symmetry():
    r = np.linspace(-3, 3, 6001)
    v = phi(r)
    assert np.all(v[np.abs(r) >= 2] == 0.0)
    assert np.all(v[np.abs(r) < 2] > 0.0)
    np.testing.assert_array_equal(v, phi(-r))


def test_phi_continuity_at_breakpoints():
    for r0 in (1.0, 2.0):
        eps = 1e-9
        assert abs(phi(r0 - eps) - phi(r0 + eps)) < 1e-8


@pytest.mark.parametrize("shift", np.linspace(0.0, 1.0, 37))
def test_phi_moment_conditions(shift):
    j = np.arange(-4, 5)
    w = phi(shift - j)
    assert abs(w.sum() - 1.0) < 4e-16
    assert abs(((shift - j) * w).sum()) < 4e-16
    assert abs((w * w).sum() - 3.0 / 8.0) < 4e-16
    assert abs(w[j % 2 == 0].sum() - 0.5) < 4e-16
    assert abs(w[j % 2 != 0].sum() - 0.5) < 4e-16


def test_delta_h_scaling():
    h = 1.0 / 64
    x = np.linspace(-3 * h, 3 * h, 101)
    np.testing.assert_allclose(delta_h(x, h), phi(x / h) / h)
