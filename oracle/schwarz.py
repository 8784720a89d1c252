"""Restricted additive Schwarz smoother (Sec. 3.3.1, Alg. 2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Subdomains are boxes of cells: box k owns b x b cells and its enlarged box
adds ``overlap`` cells on every side (periodic).  The index set G_k holds the
pressures of the enlarged box's cells and all four faces of each of those
cells; the non-overlapping set G~_k holds the owned cells' pressures, left
x-faces and bottom y-faces, so the G~_k partition the unknowns.  Local
ordering: x-faces (jj-major, m x (m+1)), then y-faces ((m+1) x m), then cells.
"""
from dataclasses import dataclass
from typing import List

import numpy as np
import scipy.linalg as la


def level_box(N, box, overlap):
    """Box size and overlap used on an N x N level: b = min(box, N/2),
    o = min(overlap, (N - b - 1) // 2), so an enlarged box never wraps onto
    itself."""
    b = min(box, N // 2)
    o = min(overlap, (N - b - 1) // 2)
    if b < 1 or N % b:
        raise ValueError(f"box {b} does not tile N={N}")
    return b, max(o, 0)


@dataclass
class Patch:
    idx: np.ndarray       # global unknowns of G_k in local order
    own_local: np.ndarray  # positions (in idx) of G~_k
    own_global: np.ndarray


def patches(N, box, overlap) -> List[Patch]:
    b, o = level_box(N, box, overlap)
    m = b + 2 * o
    n = N * N
    out = []
    for pj in range(N // b):
        for pi in range(N // b):
            x0, y0 = pi * b - o, pj * b - o
            jj, ii = np.meshgrid(np.arange(m), np.arange(m + 1), indexing="ij")
            u = ((y0 + jj) % N) * N + (x0 + ii) % N
            jj, ii = np.meshgrid(np.arange(m + 1), np.arange(m), indexing="ij")
            v = n + ((y0 + jj) % N) * N + (x0 + ii) % N
            jj, ii = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
            p = 2 * n + ((y0 + jj) % N) * N + (x0 + ii) % N
            idx = np.concatenate([u.ravel(), v.ravel(), p.ravel()])
            oj, oi = np.meshgrid(np.arange(o, o + b), np.arange(o, o + b), indexing="ij")
            oj, oi = oj.ravel(), oi.ravel()
            own = np.concatenate([oj * (m + 1) + oi,
                                  m * (m + 1) + oj * m + oi,
                                  2 * m * (m + 1) + oj * m + oi])
            out.append(Patch(idx=idx, own_local=own, own_global=idx[own]))
    return out


class RAS:
    """z = sum_k R~_k^T (L_k)^{-1} R_k r with L_k = R_k L R_k^T (Alg. 2 applied
    from a zero initial guess, so r is the given right-hand side)."""

    def __init__(self, L, N, box, overlap):
        self.parts = patches(N, box, overlap)
        self.factors = []
        Lc = L.tocsr()
        for p in self.parts:
            Lk = Lc[p.idx][:, p.idx].toarray()
            self.factors.append(la.lu_factor(Lk))

    def apply(self, r):
        z = np.zeros_like(r)
        for p, f in zip(self.parts, self.factors):
            y = la.lu_solve(f, r[p.idx])
            z[p.own_global] = y[p.own_local]
        return z

    __call__ = apply
