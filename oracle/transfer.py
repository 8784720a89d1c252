"""Inter-level transfer operators (Sec. 3.2).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Refinement ratio 2: coarse cell (i, j) of an Nc x Nc grid covers fine cells
(2i..2i+1, 2j..2j+1) of the 2Nc x 2Nc grid.  Layout as in ``mac``.
"""
import numpy as np
import scipy.sparse as sp


def _lin(N, i, j):
    return (np.mod(j, N) * N + np.mod(i, N)).astype(np.int64)


def velocity_prolongation(Nc):
    """P_u: lowest-order Raviart-Thomas interpolation (Sec. 3.2): linear in the
    direction normal to a face, piecewise constant tangentially.  A fine face
    that lies on a coarse face copies it; a fine face halfway between two
    coarse faces takes their mean.  Shape (2 Nf^2, 2 Nc^2), both components."""
    Nf = 2 * Nc
    J, I = np.meshgrid(np.arange(Nf), np.arange(Nf), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    nf, nc = Nf * Nf, Nc * Nc
    rows, cols, vals = [], [], []
    # x-faces: normal direction is x
    f = _lin(Nf, I, J)
    even = I % 2 == 0
    rows += [f[even], f[~even], f[~even]]
    cols += [_lin(Nc, I[even] // 2, J[even] // 2),
             _lin(Nc, I[~even] // 2, J[~even] // 2),
             _lin(Nc, I[~even] // 2 + 1, J[~even] // 2)]
    vals += [np.ones(even.sum()), np.full((~even).sum(), 0.5), np.full((~even).sum(), 0.5)]
    # y-faces: normal direction is y
    even = J % 2 == 0
    rows += [nf + f[even], nf + f[~even], nf + f[~even]]
    cols += [nc + _lin(Nc, I[even] // 2, J[even] // 2),
             nc + _lin(Nc, I[~even] // 2, J[~even] // 2),
             nc + _lin(Nc, I[~even] // 2, J[~even] // 2 + 1)]
    vals += [np.ones(even.sum()), np.full((~even).sum(), 0.5), np.full((~even).sum(), 0.5)]
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(2 * nf, 2 * nc)).tocsr()


def velocity_restriction(Nc):
    """R_u = P_u^*, the adjoint of P_u in the grid inner products
    <a, b>_l = h_l^2 sum a b (Sec. 3.2): R_u = (h_f / h_c)^2 P_u^T."""
    return (0.25 * velocity_prolongation(Nc).T).tocsr()


def pressure_prolongation(Nc):
    """P_p: linear interpolation of cell-centred pressures (Sec. 3.2), i.e.
    bilinear in the cell centres: weights 9/16, 3/16, 3/16, 1/16 from the
    covering coarse cell and its neighbours on the fine cell's side."""
    Nf = 2 * Nc
    J, I = np.meshgrid(np.arange(Nf), np.arange(Nf), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    ic, jc = I // 2, J // 2
    di = np.where(I % 2 == 0, -1, 1)
    dj = np.where(J % 2 == 0, -1, 1)
    f = _lin(Nf, I, J)
    rows = np.concatenate([f, f, f, f])
    cols = np.concatenate([_lin(Nc, ic, jc), _lin(Nc, ic + di, jc),
                           _lin(Nc, ic, jc + dj), _lin(Nc, ic + di, jc + dj)])
    n = f.size
    vals = np.concatenate([np.full(n, 9 / 16), np.full(n, 3 / 16), np.full(n, 3 / 16), np.full(n, 1 / 16)])
    return sp.coo_matrix((vals, (rows, cols)), shape=(Nf * Nf, Nc * Nc)).tocsr()


def pressure_restriction(Nc):
    """R_p: simple averaging of the four fine cells of each coarse cell (Sec. 3.2)."""
    Nf = 2 * Nc
    J, I = np.meshgrid(np.arange(Nf), np.arange(Nf), indexing="ij")
    I = I.ravel()
    J = J.ravel()
    rows = _lin(Nc, I // 2, J // 2)
    cols = _lin(Nf, I, J)
    return sp.coo_matrix((np.full(rows.size, 0.25), (rows, cols)), shape=(Nc * Nc, Nf * Nf)).tocsr()


def restriction(Nc):
    """Full-vector restriction [R_u; R_p] (block diagonal)."""
    return sp.block_diag([velocity_restriction(Nc), pressure_restriction(Nc)], format="csr")


def prolongation(Nc):
    """Full-vector prolongation [P_u; P_p] (block diagonal)."""
    return sp.block_diag([velocity_prolongation(Nc), pressure_prolongation(Nc)], format="csr")
