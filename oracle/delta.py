"""Peskin's four-point regularised delta kernel (App. A.3, definition of phi).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import numpy as np


def phi(r):
    """Basic kernel function phi(r) of App. A.3.

    phi(r) = (3 - 2|r| + sqrt(1 + 4|r| - 4 r^2)) / 8   for 0 <= |r| < 1
           = (5 - 2|r| - sqrt(-7 + 12|r| - 4 r^2)) / 8  for 1 <= |r| < 2
           = 0                                          for |r| >= 2
    """
    a = np.abs(np.asarray(r, dtype=np.float64))
    out = np.zeros_like(a)
    m1 = a < 1.0
    m2 = (a >= 1.0) & (a < 2.0)
    a1 = a[m1]
    a2 = a[m2]
    out[m1] = (3.0 - 2.0 * a1 + np.sqrt(1.0 + 4.0 * a1 - 4.0 * a1 * a1)) / 8.0
    out[m2] = (5.0 - 2.0 * a2 - np.sqrt(-7.0 + 12.0 * a2 - 4.0 * a2 * a2)) / 8.0
    return out


def delta_h(x, h):
    """One-dimensional regularised delta delta_h(x) = phi(x / h) / h (App. A.3)."""
    return phi(np.asarray(x, dtype=np.float64) / h) / h
