"""Element-honest comparison of the HIP path's vectors with the oracle's.

A level vector [u | v | p] holds three kinds of rows whose sizes differ by
orders of magnitude: velocity rows that carry an immersed-boundary term
(their diagonal holds dt kappa / h^2 on top of the stencil), the remaining
velocity rows, and the pressure rows.  A relative error over the whole vector
is set by its largest class and says little about the others, so every class
is compared here against its own norm:

    err_c = ||x_c - ref_c||_2 / ||ref_c||_2        for each class c.

A class whose reference is exactly zero is compared against the whole
reference's norm instead (its entries must vanish to that precision).
"""
import numpy as np


def level_classes(N, T=None):
    """Row classes of a level vector of an N x N level: 'ib' velocity rows
    (rows of the IB term T, a 2 N^2 square sparse matrix, with a stored
    entry), 'vel' the other velocity rows, 'p' the pressure rows."""
    n = N * N
    ib = np.zeros(3 * n, dtype=bool)
    if T is not None:
        T = T.tocsr()
        ib[:2 * n] = np.diff(T.indptr) > 0
    vel = np.zeros(3 * n, dtype=bool)
    vel[:2 * n] = True
    return {"ib": ib, "vel": vel & ~ib, "p": ~vel}


def face_classes(N, touched):
    """Classes of a face vector [u | v] (2 N^2): faces some kernel window
    touches ('touched', a boolean mask) and the rest."""
    touched = np.asarray(touched, dtype=bool)
    assert touched.size == 2 * N * N
    return {"touched": touched, "rest": ~touched}


def class_errors(x, ref, classes):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert x.shape == ref.shape, (x.shape, ref.shape)
    whole = max(float(np.linalg.norm(ref)), 1e-300)
    out = {}
    for name, m in classes.items():
        if not np.any(m):
            continue
        rn = float(np.linalg.norm(ref[m]))
        out[name] = float(np.linalg.norm(x[m] - ref[m])) / (rn if rn > 0.0 else whole)
    return out


def assert_classes(x, ref, classes, tol, what=""):
    """Assert err_c <= tol for every class; returns the errors."""
    errs = class_errors(x, ref, classes)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: class errors {errs} exceed {tol:g}"
    return errs
