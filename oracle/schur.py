"""Schur-complement (SC) smoother (Sec. 3.3.2, Eq. approx-fact-Stokes-IB).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

L~^{-1} = [I, -A~^{-1} G; 0, I] [A~^{-1}, 0; 0, M~^{-1}] [I, 0; D A~^{-1}, I]
applied to (r_u, r_p):
    y_u = A~^{-1} r_u
    y_p = M~^{-1} (r_p + D y_u)
    z_u = y_u - A~^{-1} G y_p,   z_p = y_p.
A~^{-1}: ``cheb_its`` first-kind Chebyshev iterations (Saad, Iterative Methods
for Sparse Linear Systems, 2nd ed., Alg. 12.1) from x = 0, preconditioned by
one symmetric Gauss-Seidel sweep on A_IB.  M~^{-1}: the same Chebyshev on the
positive semidefinite -D A~^{-1} G with right-hand side -(r_p + D y_u),
preconditioned by symmetric Gauss-Seidel on -M^ = -D diag(A_IB)^{-1} G
(Sec. 3.3.2).  Chebyshev intervals are [0.1 lam, 1.1 lam], lam the largest
Ritz value of 10 Arnoldi steps on the preconditioned operator.

Readings where the paper is silent: Gauss-Seidel is multicolour and
symmetric (colours forward, then backward); colours come from a greedy pass
over the rows in index order on the structural pattern of the matrix (the
five-point stencil plus the pattern of the IB term), each row taking the
smallest colour unused by its already coloured neighbours; the Arnoldi start
vector is the Weyl sequence frac(k g) - 1/2 (g = (sqrt 5 - 1)/2) with its
null-space components removed; the pressure output is projected to zero mean.
"""
import numpy as np
import scipy.sparse as sp

from . import mac
from .krylov import arnoldi_ritz_max

GOLDEN = (np.sqrt(5.0) - 1.0) / 2.0
ARNOLDI_STEPS = 10


def weyl_vector(n):
    k = np.arange(n, dtype=np.float64)
    return np.mod(k * GOLDEN, 1.0) - 0.5


def greedy_colouring(pattern):
    """Greedy colouring of a symmetric structural pattern, rows in index order."""
    P = pattern.tocsr()
    n = P.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    ip, ix = P.indptr, P.indices
    for r in range(n):
        used = set(int(col[c]) for c in ix[ip[r]:ip[r + 1]] if c != r and col[c] >= 0)
        c = 0
        while c in used:
            c += 1
        col[r] = c
    return col


class SGS:
    """One symmetric multicolour Gauss-Seidel sweep from x = 0 on A x = b:
    colours 0..C-1, then C-1..0; rows of one colour are mutually uncoupled, so
    updating them together equals updating them one after another."""

    def __init__(self, A, colours):
        A = A.tocsr()
        self.diag = A.diagonal().copy()
        self.sets = []
        for c in range(int(colours.max()) + 1):
            rows = np.nonzero(colours == c)[0]
            self.sets.append((rows, A[rows]))

    def __call__(self, b):
        x = np.zeros_like(b)
        order = list(range(len(self.sets))) + list(range(len(self.sets) - 1, -1, -1))
        for c in order:
            rows, Ar = self.sets[c]
            x[rows] += (b[rows] - Ar @ x) / self.diag[rows]
        return x


def chebyshev(apply_A, apply_Binv, b, lmin, lmax, its):
    """First-kind Chebyshev iteration for A x = b, x0 = 0, preconditioner B,
    spectrum of B^{-1}A assumed in [lmin, lmax] (Saad Alg. 12.1)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b.copy()
    d = apply_Binv(r) / theta
    x = np.zeros_like(b)
    for k in range(its):
        x = x + d
        if k == its - 1:
            break
        r = r - apply_A(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * apply_Binv(r)
        rho = rho_new
    return x


def _proj(v, blocks):
    out = v.copy()
    for a, b in blocks:
        out[a:b] -= out[a:b].mean()
    return out


class SchurSmoother:
    def __init__(self, level, rho, cheb_its=2):
        N = level.N
        n = N * N
        self.n = n
        self.its = cheb_its
        A_ib = level.A_ib
        self.A_ib = A_ib
        self.G = level.G
        self.D = level.D
        # velocity colouring on stencil + IB structure, both components in one
        # pass (rows in index order); with uncoupled components this is the
        # per-component colouring, with the tangent model it keeps coupled u
        # and v rows apart
        St = mac.stencil_pattern(N)
        P = (sp.block_diag([St, St]) + level.T_pattern).tocsr()
        self.col_u = greedy_colouring(P)
        self.sgs_A = SGS(A_ib, self.col_u)
        # approximate Schur complement -M^ = -D diag(A_IB)^{-1} G (PSD)
        dinv = sp.diags(1.0 / A_ib.diagonal())
        self.Mhat_neg = (-(self.D @ dinv @ self.G)).tocsr()
        self.col_p = greedy_colouring(self.Mhat_neg)
        self.sgs_M = SGS(self.Mhat_neg, self.col_p)
        vel_blocks = [(0, n), (n, 2 * n)] if rho == 0.0 else []
        v0 = _proj(weyl_vector(2 * n), vel_blocks)
        self.lam_A = arnoldi_ritz_max(lambda x: self.sgs_A(A_ib @ x), v0, ARNOLDI_STEPS)
        q0 = _proj(weyl_vector(n), [(0, n)])
        self.lam_M = arnoldi_ritz_max(lambda x: self.sgs_M(self.schur_op(x)), q0, ARNOLDI_STEPS)

    def A_tilde_inv(self, r):
        return chebyshev(lambda x: self.A_ib @ x, self.sgs_A, r,
                         0.1 * self.lam_A, 1.1 * self.lam_A, self.its)

    def schur_op(self, q):
        """-D A~^{-1} G q."""
        return -(self.D @ self.A_tilde_inv(self.G @ q))

    def M_tilde_inv(self, s):
        y = chebyshev(self.schur_op, self.sgs_M, -s, 0.1 * self.lam_M, 1.1 * self.lam_M, self.its)
        return y - y.mean()

    def apply(self, r):
        n = self.n
        ru, rp = r[:2 * n], r[2 * n:]
        yu = self.A_tilde_inv(ru)
        yp = self.M_tilde_inv(rp + self.D @ yu)
        zu = yu - self.A_tilde_inv(self.G @ yp)
        return np.concatenate([zu, yp])

    __call__ = apply
