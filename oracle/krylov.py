"""Flexible GMRES (Saad 1993, cited in Sec. 3.3) with classical Gram-Schmidt
applied twice, used both as the outer Krylov solver and, run for a fixed
number of iterations with the basic smoother as its preconditioner, as the
smoothing step itself (Sec. 3.3).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The small least-squares problem min || beta e1 - H y || is solved with
``numpy.linalg.lstsq`` at every step (no Givens rotations).
"""
import numpy as np


def _orthogonalise(V, w):
    """Classical Gram-Schmidt, twice: returns (h, w_perp)."""
    B = np.stack(V, 1)
    h = B.T @ w
    w = w - B @ h
    h2 = B.T @ w
    w = w - B @ h2
    return h + h2, w


def fgmres_cycle(apply_A, apply_M, r0, steps, stop_abs=None, history=None):
    """One FGMRES cycle from a zero correction: up to ``steps`` Arnoldi steps
    on A with right preconditioner M (applied afresh each step, so M may vary).
    Returns (correction, steps_taken, final residual estimate)."""
    beta = float(np.linalg.norm(r0))
    if beta == 0.0:
        return np.zeros_like(r0), 0, 0.0
    V = [r0 / beta]
    Z = []
    H = np.zeros((steps + 1, steps))
    y = np.zeros(0)
    est = beta
    k = 0
    for j in range(steps):
        z = apply_M(V[j])
        Z.append(z)
        w = apply_A(z)
        h, w = _orthogonalise(V, w)
        H[:j + 1, j] = h
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        k = j + 1
        e1 = np.zeros(k + 1)
        e1[0] = beta
        y = np.linalg.lstsq(H[:k + 1, :k], e1, rcond=None)[0]
        est = float(np.linalg.norm(e1 - H[:k + 1, :k] @ y))
        if history is not None:
            history.append(est)
        if hn == 0.0:
            break
        V.append(w / hn)
        if stop_abs is not None and est <= stop_abs:
            break
    dx = np.zeros_like(r0)
    for i in range(k):
        dx += y[i] * Z[i]
    return dx, k, est


def fgmres(apply_A, apply_M, b, restart=30, rtol=1e-8, max_it=100, x0=None):
    """Right-preconditioned restarted FGMRES from x0 (default 0); stops when the
    Arnoldi residual estimate drops to rtol ||b|| or after max_it iterations.
    Returns (x, info) with info = dict(iters, history, converged)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    bnorm = float(np.linalg.norm(b))
    hist = []
    its = 0
    if bnorm == 0.0:
        return np.zeros_like(b), dict(iters=0, history=hist, converged=True)
    target = rtol * bnorm
    while its < max_it:
        r = b - apply_A(x)
        if float(np.linalg.norm(r)) <= target:
            return x, dict(iters=its, history=hist, converged=True)
        dx, k, est = fgmres_cycle(apply_A, apply_M, r, min(restart, max_it - its),
                                  stop_abs=target, history=hist)
        x = x + dx
        its += k
        if est <= target or k == 0:
            return x, dict(iters=its, history=hist, converged=est <= target)
    return x, dict(iters=its, history=hist, converged=False)


def fgmres_smooth(apply_A, apply_B, w, b, nu):
    """Sec. 3.3 smoothing: nu FGMRES iterations on A e = b - A w from e = 0,
    right-preconditioned by the basic smoother B; returns w + e."""
    r = b - apply_A(w)
    e, _, _ = fgmres_cycle(apply_A, apply_B, r, nu)
    return w + e


def richardson_smooth(apply_A, apply_B, w, b, nu):
    """nu undamped Richardson steps w <- w + B (b - A w) with the basic
    smoother B: the reading of a smoothing sweep as a plain Richardson
    iteration (Sec. 6, on the large-box Vanka smoother)."""
    for _ in range(nu):
        w = w + apply_B(b - apply_A(w))
    return w


def arnoldi_ritz_max(apply_op, v0, steps):
    """Largest real part among the Ritz values (eigenvalues of the square
    Hessenberg matrix) after ``steps`` Arnoldi steps from v0."""
    V = [v0 / np.linalg.norm(v0)]
    H = np.zeros((steps + 1, steps))
    k = 0
    for j in range(steps):
        w = apply_op(V[j])
        h, w = _orthogonalise(V, w)
        H[:j + 1, j] = h
        hn = float(np.linalg.norm(w))
        H[j + 1, j] = hn
        k = j + 1
        if hn == 0.0:
            break
        V.append(w / hn)
    ev = np.linalg.eigvals(H[:k, :k])
    return float(np.max(ev.real))
