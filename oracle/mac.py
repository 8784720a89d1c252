"""Staggered (MAC) grid operators on the periodic unit square (App. A.1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Grid: N x N cells, h = 1/N, cell (i, j) centred at ((i+1/2)h, (j+1/2)h).
The paper labels x1-edges (i-1/2, j) and x2-edges (i, j-1/2); here
    u[j, i] = (u_1)_{i-1/2, j}  at (i h, (j+1/2) h)
    v[j, i] = (u_2)_{i, j-1/2}  at ((i+1/2) h, j h)
    p[j, i] = p_{i, j}          at ((i+1/2) h, (j+1/2) h)
and a level vector is [u.ravel(), v.ravel(), p.ravel()] (length 3 N^2).
All indices are periodic.  The operators are the standard second-order
differences of App. A.1; the paper's block operators are
A = rho/dt I - mu Lap_h, G = grad_h, D = div_h (text after Eq. system-impib).
"""
import numpy as np
import scipy.sparse as sp


def _idx(N, i, j):
    return (np.mod(j, N) * N + np.mod(i, N)).astype(np.int64)


def scalar_laplacian(N):
    """Five-point Laplacian (u_{i+1,j} + u_{i-1,j} + u_{i,j+1} + u_{i,j-1} - 4 u_{ij}) / h^2
    on one periodic N x N staggered component."""
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    row = _idx(N, i, j)
    rows, cols, vals = [], [], []
    for di, dj, c in ((0, 0, -4.0), (1, 0, 1.0), (-1, 0, 1.0), (0, 1, 1.0), (0, -1, 1.0)):
        rows.append(row)
        cols.append(_idx(N, i + di, j + dj))
        vals.append(np.full(N * N, c / (h * h)))
    n = N * N
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n)).tocsr()


def gradient(N):
    """G = grad_h : cell pressures -> face values (2 N^2 x N^2).
    (Gp)_{i-1/2, j} = (p_{i,j} - p_{i-1,j}) / h on x-faces,
    (Gp)_{i, j-1/2} = (p_{i,j} - p_{i,j-1}) / h on y-faces."""
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    n = N * N
    face = _idx(N, i, j)
    rows = np.concatenate([face, face, n + face, n + face])
    cols = np.concatenate([_idx(N, i, j), _idx(N, i - 1, j), _idx(N, i, j), _idx(N, i, j - 1)])
    vals = np.concatenate([np.full(n, 1.0 / h), np.full(n, -1.0 / h),
                           np.full(n, 1.0 / h), np.full(n, -1.0 / h)])
    return sp.coo_matrix((vals, (rows, cols)), shape=(2 * n, n)).tocsr()


def divergence(N):
    """D = div_h : face velocities -> cells (N^2 x 2 N^2).
    (Du)_{i,j} = (u_{i+1/2,j} - u_{i-1/2,j} + v_{i,j+1/2} - v_{i,j-1/2}) / h."""
    h = 1.0 / N
    j, i = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    n = N * N
    cell = _idx(N, i, j)
    rows = np.concatenate([cell, cell, cell, cell])
    cols = np.concatenate([_idx(N, i + 1, j), _idx(N, i, j), n + _idx(N, i, j + 1), n + _idx(N, i, j)])
    vals = np.concatenate([np.full(n, 1.0 / h), np.full(n, -1.0 / h),
                           np.full(n, 1.0 / h), np.full(n, -1.0 / h)])
    return sp.coo_matrix((vals, (rows, cols)), shape=(n, 2 * n)).tocsr()


def momentum(N, rho, mu, dt):
    """A = rho/dt I - mu Lap_h acting on both velocity components (2 N^2 square)."""
    L = scalar_laplacian(N)
    n = N * N
    Ac = (rho / dt) * sp.identity(n, format="csr") - mu * L
    return sp.block_diag([Ac, Ac], format="csr")


def stokes_ib(A_ib, G, D):
    """Stokes-IB operator L_IB = [[A_IB, G], [-D, 0]] (Eq. matrix-impib)."""
    n = D.shape[0]
    Z = sp.csr_matrix((n, n))
    return sp.bmat([[A_ib, G], [-D, Z]], format="csr")


def stencil_pattern(N):
    """Structural pattern (0/1) of the five-point stencil on one component."""
    L = scalar_laplacian(N)
    P = L.copy()
    P.data[:] = 1.0
    return P
