"""Lagrangian-Eulerian coupling and fibre elasticity (App. A.2, A.3; Sec. 5).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Forces are nodal (each Lagrangian node carries a force, not a density), so the
quadrature weight Delta s1 Delta s2 of the spreading sum is 1 and
S_h = J_h^T / h^2; a per-spring stiffness kappa_e plays the role of
alpha Delta s2 / Delta s1 in the paper's fibre model.
"""
import numpy as np
import scipy.sparse as sp

from .delta import phi

# Offsets of the face nodes in grid units: x-faces sit at (i, j+1/2),
# y-faces at (i+1/2, j) (App. A.1 labelling).
_SHIFT = {0: (0.0, 0.5), 1: (0.5, 0.0)}


def _window(t):
    """Grid nodes k (integers) with |t - k| < 2, with r = t - k, for a vector t."""
    base = np.floor(t).astype(np.int64)
    ks, rs = [], []
    for d in range(-2, 4):
        k = base + d
        r = t - k
        ks.append(k)
        rs.append(r)
    K = np.stack(ks, 1)
    R = np.stack(rs, 1)
    keep = np.abs(R) < 2.0
    return K, R, keep


def coupling_weights(X, N, comp):
    """All (point l, face index, phi(rx) phi(ry)) triples of the discrete delta
    sums of App. A.3 for velocity component ``comp``; ``phi(rx) phi(ry)`` equals
    delta_h(x_face - X_l) h^2.  Points lie in [0, 1)^2 and the kernel support
    (4h) is shorter than the period, so the nearest periodic image is the only
    one that contributes."""
    X = np.asarray(X, dtype=np.float64)
    sx, sy = _SHIFT[comp]
    tx = X[:, 0] * N - sx
    ty = X[:, 1] * N - sy
    Kx, Rx, kx = _window(tx)
    Ky, Ry, ky = _window(ty)
    M = X.shape[0]
    rows, cols, vals = [], [], []
    for a in range(Kx.shape[1]):
        for b in range(Ky.shape[1]):
            ok = kx[:, a] & ky[:, b]
            l = np.nonzero(ok)[0]
            i = np.mod(Kx[l, a], N)
            j = np.mod(Ky[l, b], N)
            rows.append(l)
            cols.append(j * N + i)
            vals.append(phi(Rx[l, a]) * phi(Ry[l, b]))
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def interp_matrix(X, N, comp):
    """J_h for one component: (U_c)_l = sum_faces (u_c)_face delta_h(x_face - X_l) h^2
    (App. A.3, velocity interpolation).  Shape (M, N^2)."""
    r, c, v = coupling_weights(X, N, comp)
    return sp.coo_matrix((v, (r, c)), shape=(X.shape[0], N * N)).tocsr()


def spread_matrix(X, N, comp):
    """S_h for one component: (f_c)_face = sum_l (F_c)_l delta_h(x_face - X_l)
    (App. A.3, force spreading, unit nodal weights).  Shape (N^2, M)."""
    h = 1.0 / N
    r, c, v = coupling_weights(X, N, comp)
    return sp.coo_matrix((v / (h * h), (c, r)), shape=(N * N, X.shape[0])).tocsr()


def stiffness_matrix(M, springs, kappa):
    """K_h with F = K_h X for zero-rest-length linear springs (Sec. 5, App. A.2):
    the spring e = (a, b) pulls node a by kappa_e (X_b - X_a) and node b by
    kappa_e (X_a - X_b).  Acts on one coordinate; symmetric negative
    semidefinite."""
    a = np.asarray(springs[:, 0], dtype=np.int64)
    b = np.asarray(springs[:, 1], dtype=np.int64)
    k = np.asarray(kappa, dtype=np.float64)
    rows = np.concatenate([a, a, b, b])
    cols = np.concatenate([a, b, b, a])
    vals = np.concatenate([-k, k, -k, k])
    return sp.coo_matrix((vals, (rows, cols)), shape=(M, M)).tocsr()


def fibre_force(X, springs, kappa):
    """Nodal fibre force F = K_h X evaluated spring by spring (Sec. 5 linear
    fibre functional with the half-index differences of App. A.2)."""
    F = np.zeros_like(np.asarray(X, dtype=np.float64))
    for e in range(springs.shape[0]):
        a, b = int(springs[e, 0]), int(springs[e, 1])
        d = X[b] - X[a]
        F[a] += kappa[e] * d
        F[b] -= kappa[e] * d
    return F


def ib_term(X, springs, kappa, N, dt):
    """Eulerian elasticity part of A_IB on the finest grid: -dt S_h K_h J_h,
    one block per velocity component (text after Eq. matrix-impib)."""
    K = stiffness_matrix(X.shape[0], springs, kappa)
    blocks = []
    for comp in (0, 1):
        S = spread_matrix(X, N, comp)
        J = interp_matrix(X, N, comp)
        blocks.append((-dt) * (S @ (K @ J)))
    return sp.block_diag(blocks, format="csr")


# ---- structural patterns (0/1 matrices, no numerical cancellation) --------

def interp_pattern(X, N, comp):
    r, c, v = coupling_weights(X, N, comp)
    return sp.coo_matrix((np.ones_like(v), (r, c)), shape=(X.shape[0], N * N)).tocsr()


def stiffness_pattern(M, springs):
    a = np.asarray(springs[:, 0], dtype=np.int64)
    b = np.asarray(springs[:, 1], dtype=np.int64)
    rows = np.concatenate([a, a, b, b])
    cols = np.concatenate([a, b, b, a])
    P = sp.coo_matrix((np.ones(rows.size), (rows, cols)), shape=(M, M)).tocsr()
    P.data[:] = 1.0
    return P


# ---- springs with rest lengths and their tangent (Sec. 5, App. A.2, Sec. 6) --
#
# The fibre model of Sec. 5 lets the tension be any function of the strain;
# App. A.2 evaluates tension and unit tangent at half indices.  A spring
# e = (a, b) with separation d = X_b - X_a (minimum image on the periodic
# square), length l = |d|, unit vector t = d / l and tension
# T_e = kappa_e (l - L_e) pulls node a by T_e t and node b by -T_e t; with
# L_e = 0 this is the linear model above.  A Newton-Krylov treatment of the
# nonlinear model (Sec. 6) solves systems of the same form with K_h replaced
# by the force's Jacobian dF/dX at the current configuration.

def _min_image(d):
    return d - np.round(d)


def spring_force(X, springs, kappa, rest):
    """Nodal forces F(X) of springs with rest lengths (see above)."""
    X = np.asarray(X, dtype=np.float64)
    F = np.zeros_like(X)
    for e in range(springs.shape[0]):
        a, b = int(springs[e, 0]), int(springs[e, 1])
        d = _min_image(X[b] - X[a])
        L = float(rest[e])
        if L == 0.0:
            f = kappa[e] * d
        else:
            l = float(np.hypot(d[0], d[1]))
            if l == 0.0:
                raise ValueError(f"spring {e} has zero length and a nonzero rest length")
            f = kappa[e] * (l - L) / l * d
        F[a] += f
        F[b] -= f
    return F


def tangent_blocks(X, springs, kappa, rest):
    """Per spring the 2x2 block K_e = dF_a/dX_b: the derivative of
    kappa (1 - L/|d|) d in d, kappa [(1 - L/l) I + (L/l) t t^T].  [E, 2, 2]."""
    X = np.asarray(X, dtype=np.float64)
    out = np.zeros((springs.shape[0], 2, 2))
    for e in range(springs.shape[0]):
        a, b = int(springs[e, 0]), int(springs[e, 1])
        L = float(rest[e])
        if L == 0.0:
            out[e] = kappa[e] * np.eye(2)
            continue
        d = _min_image(X[b] - X[a])
        l = float(np.hypot(d[0], d[1]))
        if l == 0.0:
            raise ValueError(f"spring {e} has zero length and a nonzero rest length")
        t = d / l
        out[e] = kappa[e] * ((1.0 - L / l) * np.eye(2) + (L / l) * np.outer(t, t))
    return out


def tangent_stiffness(X, springs, kappa, rest):
    """K'_tan = -dF/dX (2M x 2M, planar order: x of every node, then y):
    spring e adds K_e to the (a, a) and (b, b) blocks and -K_e to (a, b) and
    (b, a).  Symmetric; with all L_e = 0 it is the linear stiffness
    -K_h on each coordinate."""
    M = np.asarray(X).shape[0]
    Kb = tangent_blocks(X, springs, kappa, rest)
    rows, cols, vals = [], [], []
    for e in range(springs.shape[0]):
        a, b = int(springs[e, 0]), int(springs[e, 1])
        for c in (0, 1):
            for cc in (0, 1):
                k = Kb[e, c, cc]
                rows += [c * M + a, c * M + a, c * M + b, c * M + b]
                cols += [cc * M + a, cc * M + b, cc * M + b, cc * M + a]
                vals += [k, -k, k, -k]
    return sp.coo_matrix((vals, (rows, cols)), shape=(2 * M, 2 * M)).tocsr()


def ib_term_tangent(X, springs, kappa, rest, N, dt):
    """The IB part of A_IB with the tangent stiffness, dt S_h K'_tan J_h with
    S_h = diag(S_x, S_y) and J_h = diag(J_x, J_y): 2 N^2 square, coupling the
    two velocity components through the off-diagonal entries of K_e."""
    K = tangent_stiffness(X, springs, kappa, rest)
    S = sp.block_diag([spread_matrix(X, N, 0), spread_matrix(X, N, 1)], format="csr")
    J = sp.block_diag([interp_matrix(X, N, 0), interp_matrix(X, N, 1)], format="csr")
    return (dt * (S @ (K @ J))).tocsr()


def tangent_pattern(X, springs, N):
    """Structural pattern of J^T K'_tan J: every component couples to both."""
    KP = stiffness_pattern(X.shape[0], springs)
    JP = sp.block_diag([interp_pattern(X, N, 0), interp_pattern(X, N, 1)], format="csr")
    KP2 = sp.bmat([[KP, KP], [KP, KP]], format="csr")
    P = (JP.T @ (KP2 @ JP)).tocsr()
    P.data[:] = 1.0
    return P
