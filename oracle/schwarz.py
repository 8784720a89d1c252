"""Restricted additive and multiplicative Schwarz smoothers (Sec. 3.3.1,
Alg. 2 and Alg. 3).

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
import scipy.sparse as sp


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
    from a zero initial guess, so r is the given right-hand side).

    combine="sum" replaces the restriction R~_k^T by R_k^T: every unknown
    of G_k receives box k's local solution, summed over the boxes holding it
    (plain additive Schwarz), boxes taken in index order."""

    def __init__(self, L, N, box, overlap, combine="restricted"):
        if combine not in ("restricted", "sum"):
            raise ValueError(combine)
        self.combine = combine
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
            if self.combine == "sum":
                z[p.idx] += y      # the indices of one box are distinct
            else:
                z[p.own_global] = y[p.own_local]
        return z

    __call__ = apply


def structural_pattern(level):
    """0/1 pattern of L_IB on a level: the five-point stencil on each velocity
    component, the IB term's structural pattern, G and -D (whose entries are
    +-1/h and never cancel); the pressure block is empty."""
    St = level.A.copy()
    St.data[:] = 1.0   # A = rho/dt I - mu Lap: diagonal + four neighbours, all nonzero
    Pv = (St + level.T_pattern).tocsr()
    Pv.data[:] = 1.0
    G = level.G.copy()
    G.data[:] = 1.0
    D = level.D.copy()
    D.data[:] = 1.0
    n = D.shape[0]
    P = sp.bmat([[Pv, G], [D, sp.csr_matrix((n, n))]], format="csr")
    P.data[:] = 1.0
    return P


def box_colours(pattern, parts):
    """Greedy colouring of the boxes for the multiplicative sweep.  Boxes i
    and j conflict when the operator couples a row of G_j to an unknown of
    G~_i, or a row of G_i to an unknown of G~_j: then the order of their two
    updates matters.  Boxes are coloured in index order with the smallest
    colour not taken by an already coloured conflicting box, so boxes of one
    colour can be updated from the same residual."""
    P = pattern.tocsr()
    owner = np.empty(P.shape[0], dtype=np.int64)
    for k, p in enumerate(parts):
        owner[p.own_global] = k
    nb = len(parts)
    reach = []
    for p in parts:
        cols = np.unique(P[p.idx].indices)
        reach.append(set(np.unique(owner[cols]).tolist()))
    adj = [set() for _ in range(nb)]
    for j in range(nb):
        for i in reach[j]:
            if i != j:
                adj[j].add(i)
                adj[i].add(j)
    colour = np.full(nb, -1, dtype=np.int64)
    for k in range(nb):
        used = {colour[q] for q in adj[k] if colour[q] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[k] = c
    return colour


class RMS:
    """w <- RMS(w, b) (Alg. 3): for each box in turn, the residual of the
    current w, a local solve with L_k = R_k L R_k^T, and the update of w on
    G~_k.  The boxes are visited in colour-major order (colour 0's boxes in
    index order, then colour 1's, ...), colours from ``box_colours``."""

    def __init__(self, L, pattern, N, box, overlap):
        self.parts = patches(N, box, overlap)
        self.L = L.tocsr()
        self.rows = [self.L[p.idx] for p in self.parts]
        self.factors = [la.lu_factor(self.L[p.idx][:, p.idx].toarray()) for p in self.parts]
        self.colour = box_colours(pattern, self.parts)
        self.order = sorted(range(len(self.parts)), key=lambda k: (self.colour[k], k))

    def sweep(self, w, b, order=None):
        w = np.array(w, dtype=np.float64, copy=True)
        for k in (self.order if order is None else order):
            p = self.parts[k]
            rk = b[p.idx] - self.rows[k] @ w          # R_k (b - L w)
            y = la.lu_solve(self.factors[k], rk)
            w[p.own_global] += y[p.own_local]
        return w

    def apply(self, r):
        """Smoother application from a zero initial guess."""
        return self.sweep(np.zeros_like(r), r)

    __call__ = apply
