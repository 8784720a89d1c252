"""Python binding of libibmg: one ``StokesIB`` object per Stokes-IB system,
or one ``StokesIBBatch`` for many independent systems solved together.

Only argument marshalling happens here: torch supplies every byte of device
memory (each handle's workspace is one torch tensor, sized by the library's
sizing call) and the current HIP stream; every computation runs in the
library's kernels.  Vectors are float64 CUDA tensors laid out [u | v | p]
(see include/ibmg.h).
"""
import ctypes

import numpy as np
import torch

from . import _lib

_STATUS = {0: "OK", 1: "NOT_CONVERGED", -1: "ERR_ARG", -2: "ERR_HIP", -3: "ERR_WORKSPACE",
           -4: "ERR_BREAKDOWN", -5: "ERR_NONFINITE", -6: "ERR_STATE"}

# Extra workspace beyond the set-up's exact size: a rebuild at moved
# positions (time steps) may touch more boxes than the first set-up.
WORKSPACE_HEADROOM = 0.125
WORKSPACE_EXTRA = 64 << 20


class IbmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _dev_vec(t, n, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if t.numel() != n or not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous with {n} elements")
    return t


def _make_desc(system, precision):
    """ibmg_desc of a system description; returns it with the host arrays it
    points into (keep them alive while the descriptor is in use)."""
    X = np.ascontiguousarray(system.X, dtype=np.float64)
    springs = np.ascontiguousarray(system.springs, dtype=np.int32)
    kappa = np.ascontiguousarray(system.kappa, dtype=np.float64)
    d = _lib.Desc()
    d.N = int(system.N)
    d.coarse_N = int(system.coarse_N)
    d.rho, d.mu, d.dt = float(system.rho), float(system.mu), float(system.dt)
    d.M = int(X.shape[0])
    d.X = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.n_springs = int(springs.shape[0])
    d.ends = springs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    d.kappa = kappa.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    d.smoother = {"ras": _lib.RAS, "sc": _lib.SC, "rms": _lib.RMS}[getattr(system, "smoother", "ras")]
    d.box = int(getattr(system, "box", 8))
    d.overlap = int(getattr(system, "overlap", 2))
    d.nu1 = int(getattr(system, "nu1", 2))
    d.nu2 = int(getattr(system, "nu2", 2))
    d.cheb_its = int(getattr(system, "cheb_its", 2))
    d.precision = {"fp64": _lib.FP64, "fp32": _lib.FP32_SMOOTHER}[precision]
    d.spring_model = {"linear": _lib.SPRING_LINEAR, "tangent": _lib.SPRING_TANGENT}[
        getattr(system, "spring_model", "linear")]
    d.combine = {"restricted": _lib.COMBINE_RESTRICTED, "sum": _lib.COMBINE_SUM}[
        getattr(system, "combine", "restricted")]
    d.sweep_kind = {"fgmres": _lib.SWEEP_FGMRES, "richardson": _lib.SWEEP_RICHARDSON}[
        getattr(system, "sweep", "fgmres")]
    d.max_restart = int(getattr(system, "max_restart", 30))
    rest = getattr(system, "rest", None)
    if rest is not None:
        rest = np.ascontiguousarray(rest, dtype=np.float64)
        if rest.shape != (springs.shape[0],):
            raise ValueError("rest must hold one length per spring")
        d.rest = rest.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d, (X, springs, kappa, rest)


def _ptr_array(ts):
    return (ctypes.c_void_p * len(ts))(*[t.data_ptr() for t in ts])


def _workspace(lib, nbytes, headroom):
    """The handle's device workspace: one uint8 torch tensor (torch's caching
    allocator aligns it to at least 256 bytes)."""
    total = int(nbytes * (1.0 + headroom)) + (WORKSPACE_EXTRA if headroom > 0 else 0)
    ws = torch.empty(max(total, 256), dtype=torch.uint8, device="cuda")
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace tensor is not 256-byte aligned")
    return ws


class StokesIB:
    """Multigrid-preconditioned solver for one periodic Stokes-IB system.

    ``system`` is any object with the attributes N, coarse_N, rho, mu, dt,
    X [M,2], springs [E,2], kappa [E], smoother ("ras"|"sc"), box, overlap,
    nu1, nu2, cheb_its (e.g. ``workloads.Workload``)."""

    def __init__(self, system, precision="fp64", workspace_headroom=WORKSPACE_HEADROOM):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("StokesIB needs a HIP device")
        d, keep = _make_desc(system, precision)
        self.N = d.N
        self.X, self.springs, self.kappa, self.rest = keep
        self.M = d.M
        self.E = d.n_springs
        self.rho = d.rho
        self.precision = precision
        self.desc = d
        nb = ctypes.c_size_t()
        st = self.lib.ibmg_workspace_bytes(ctypes.byref(d), ctypes.byref(nb))
        if st != 0:
            raise IbmgError(st, self.lib.ibmg_last_error(None).decode())
        self.workspace_bytes = nb.value
        self.workspace = _workspace(self.lib, nb.value, workspace_headroom)
        h = ctypes.c_void_p()
        st = self.lib.ibmg_create(ctypes.byref(d), _ptr(self.workspace), self.workspace.numel(), _stream(),
                                  ctypes.byref(h))
        if st != 0:
            raise IbmgError(st, self.lib.ibmg_last_error(None).decode())
        self.h = h
        nl = ctypes.c_int32()
        self._check(self.lib.ibmg_levels(self.h, ctypes.byref(nl)))
        self.n_levels = nl.value
        self.level_sizes = []
        for l in range(self.n_levels):
            n = ctypes.c_int32()
            self._check(self.lib.ibmg_level_n(self.h, l, ctypes.byref(n)))
            self.level_sizes.append(n.value)

    def _check(self, st, ok=(0,)):
        if st not in ok:
            raise IbmgError(st, self.lib.ibmg_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.ibmg_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_used(self):
        """(bytes in use now, most bytes ever in use) of the handle's workspace."""
        a, b = ctypes.c_size_t(), ctypes.c_size_t()
        self._check(self.lib.ibmg_workspace_used(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def n(self, level=-1):
        N = self.level_sizes[level]
        return 3 * N * N

    def _new(self, n):
        return torch.empty(n, dtype=torch.float64, device="cuda")

    # ---- operators ---------------------------------------------------------
    def apply(self, w, level=-1, transpose=False, out=None):
        level = level % self.n_levels
        n = self.n(level)
        _dev_vec(w, n, "w")
        y = self._new(n) if out is None else _dev_vec(out, n, "out")
        fn = self.lib.ibmg_apply_A_IB_T if transpose else self.lib.ibmg_apply_A_IB
        self._check(fn(self.h, level, _ptr(w), _ptr(y), _stream()))
        return y

    def spread(self, F):
        F = _dev_vec(F, 2 * self.M, "F") if self.M else F
        f = self._new(2 * self.N * self.N)
        self._check(self.lib.ibmg_spread(self.h, _ptr(F) if self.M else None, _ptr(f), _stream()))
        return f

    def interp(self, u):
        _dev_vec(u, 2 * self.N * self.N, "u")
        U = self._new(max(2 * self.M, 1))
        self._check(self.lib.ibmg_interp(self.h, _ptr(u), _ptr(U), _stream()))
        return U[:2 * self.M]

    def restrict(self, level, fine):
        level = level % self.n_levels
        _dev_vec(fine, self.n(level), "fine")
        c = self._new(self.n(level - 1))
        self._check(self.lib.ibmg_restrict(self.h, level, _ptr(fine), _ptr(c), _stream()))
        return c

    def prolong_add(self, level, coarse, fine):
        level = level % self.n_levels
        _dev_vec(coarse, self.n(level - 1), "coarse")
        _dev_vec(fine, self.n(level), "fine")
        self._check(self.lib.ibmg_prolong_add(self.h, level, _ptr(coarse), _ptr(fine), _stream()))
        return fine

    def smoother_apply(self, level, r):
        level = level % self.n_levels
        _dev_vec(r, self.n(level), "r")
        z = self._new(self.n(level))
        self._check(self.lib.ibmg_smoother_apply(self.h, level, _ptr(r), _ptr(z), _stream()))
        return z

    def smooth(self, level, w, b, nu):
        level = level % self.n_levels
        _dev_vec(w, self.n(level), "w")
        _dev_vec(b, self.n(level), "b")
        self._check(self.lib.ibmg_smooth(self.h, level, _ptr(w), _ptr(b), int(nu), _stream()))
        return w

    def coarse_solve(self, r):
        _dev_vec(r, self.n(0), "r")
        x = self._new(self.n(0))
        self._check(self.lib.ibmg_coarse_solve(self.h, _ptr(r), _ptr(x), _stream()))
        return x

    def vcycle(self, r, out=None):
        _dev_vec(r, self.n(), "r")
        z = self._new(self.n()) if out is None else _dev_vec(out, self.n(), "out")
        self._check(self.lib.ibmg_vcycle(self.h, _ptr(r), _ptr(z), _stream()))
        return z

    def solve(self, b, rtol=1e-8, restart=30, max_it=100, x0=None, out=None, history=128,
              transpose=False):
        _dev_vec(b, self.n(), "b")
        if x0 is not None:
            x = x0.clone() if out is None else out.copy_(x0)
        else:
            x = self._new(self.n()) if out is None else out
        o = _lib.SolveOpts(float(rtol), int(restart), int(max_it), 1 if x0 is not None else 0,
                           1 if transpose else 0)
        hist = (ctypes.c_double * history)()
        info = _lib.SolveInfo()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = history
        st = self._check(self.lib.ibmg_fgmres_solve(self.h, _ptr(b), _ptr(x), ctypes.byref(o),
                                                    ctypes.byref(info), _stream()), ok=(0, 1))
        k = min(info.iters, history)
        return x, dict(status=_STATUS[st], converged=st == 0, iters=info.iters,
                       restarts=info.restarts, rel_res_est=info.rel_res_est,
                       rel_res_true=info.rel_res_true, rhs_null_norm=info.rhs_null_norm,
                       setup_ms=info.setup_ms, solve_ms=info.solve_ms, vcycles=info.vcycles,
                       history=list(hist[:k]))

    # ---- semi-implicit time step (Sec. 2.2) --------------------------------
    def step_rhs(self, w):
        """[(rho/dt) u + S_h K_h X; 0] for w = [u | v | p] at the current positions."""
        _dev_vec(w, self.n(), "w")
        rhs = self._new(self.n())
        self._check(self.lib.ibmg_step_rhs(self.h, _ptr(w), _ptr(rhs), _stream()))
        return rhs

    def time_step(self, w, rtol=1e-8, restart=30, max_it=100, history=128):
        """Advance one step: returns (u, p)^{n+1} (a new tensor) and the solve
        info; the handle's structure moves to X^{n+1} and is rebuilt there."""
        _dev_vec(w, self.n(), "w")
        x = w.clone()
        o = _lib.SolveOpts(float(rtol), int(restart), int(max_it), 0, 0)
        hist = (ctypes.c_double * history)()
        info = _lib.SolveInfo()
        info.history = ctypes.cast(hist, ctypes.POINTER(ctypes.c_double))
        info.history_cap = history
        st = self._check(self.lib.ibmg_time_step(self.h, _ptr(x), ctypes.byref(o), ctypes.byref(info), _stream()),
                         ok=(0, 1))
        return x, dict(status=_STATUS[st], converged=st == 0, iters=info.iters, rel_res_true=info.rel_res_true,
                       rhs_null_norm=info.rhs_null_norm, solve_ms=info.solve_ms, rebuild_ms=info.setup_ms)

    def positions(self):
        X = np.empty((self.M, 2), dtype=np.float64)
        self._check(self.lib.ibmg_positions(self.h, X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
        return X

    def spring_gradient(self, w, lam):
        _dev_vec(w, self.n(), "w")
        _dev_vec(lam, self.n(), "lam")
        g = self._new(max(self.E, 1))
        self._check(self.lib.ibmg_spring_gradient(self.h, _ptr(w), _ptr(lam), _ptr(g), _stream()))
        return g[:self.E]

    def set_kappa(self, kappa):
        k = np.ascontiguousarray(kappa, dtype=np.float64)
        if k.shape != (self.E,):
            raise ValueError("kappa has the wrong length")
        self.kappa = k
        self._check(self.lib.ibmg_set_kappa(self.h, k.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            _stream()))

    def sc_info(self, level):
        """Schur-complement smoother data of a level: Ritz-value bounds and
        Gauss-Seidel colour counts."""
        lam = (ctypes.c_double * 2)()
        col = (ctypes.c_int32 * 2)()
        self._check(self.lib.ibmg_sc_info(self.h, level % self.n_levels, lam, col))
        return dict(lam_A=lam[0], lam_M=lam[1], colours_u=col[0], colours_p=col[1])

    def kernel_time(self, kernel, level=-1, reps=50):
        """Average duration (ms) of one launch of a single library kernel on
        this handle's stream, with its algorithmic bytes and flops per launch.
        kernel: "ras_ib", "ras_interior", "stencil", "restrict", "prolong",
        "spread", "interp", the smoothing step's Krylov kernels "apply_dots",
        "upd_dots", "scale_upd", "combine_ls", the outer solve's second-pass
        kernels "upd_norm", "scale_red" (single handles) or "ras_batch"
        (batch handles)."""
        k = {"ras_ib": _lib.KERNEL_RAS_IB, "ras_interior": _lib.KERNEL_RAS_INTERIOR,
             "stencil": _lib.KERNEL_STENCIL, "ras_batch": _lib.KERNEL_RAS_BATCH,
             "restrict": _lib.KERNEL_RESTRICT, "prolong": _lib.KERNEL_PROLONG,
             "spread": _lib.KERNEL_SPREAD, "interp": _lib.KERNEL_INTERP,
             "apply_dots": _lib.KERNEL_APPLY_DOTS, "upd_dots": _lib.KERNEL_UPD_DOTS,
             "upd_norm": _lib.KERNEL_UPD_NORM, "scale_red": _lib.KERNEL_SCALE_RED,
             "combine_ls": _lib.KERNEL_COMBINE_LS, "scale_upd": _lib.KERNEL_SCALE_UPD}[kernel]
        ms, by, fl = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.ibmg_kernel_time(self.h, k, level % self.n_levels, int(reps), _stream(),
                                              ctypes.byref(ms), ctypes.byref(by), ctypes.byref(fl)))
        return dict(ms=ms.value, bytes=by.value, flops=fl.value)

    def stats(self):
        buf = (ctypes.c_int64 * 256)()
        wr = ctypes.c_int32()
        self._check(self.lib.ibmg_stats(self.h, buf, 256, ctypes.byref(wr)))
        v = list(buf[:wr.value])
        out = {"levels": []}
        for l in range(v[0]):
            N, boxes, uniq, ib, tnnz, ncol = v[1 + 6 * l:7 + 6 * l]
            out["levels"].append(dict(N=N, boxes=boxes, unique_boxes=uniq, ib_boxes=ib, ib_nnz=tnnz,
                                      box_colours=ncol))
        return out


class StokesIBBatch:
    """Many independent periodic Stokes-IB systems solved together (one
    persistent launch per smoother sweep across all of them).  ``systems`` is
    a list of system descriptions as for ``StokesIB``; they may differ in N,
    structure and stiffness but must share the fluid and box parameters."""

    def __init__(self, systems, precision="fp32", workspace_headroom=0.0):
        self.lib = _lib.load()
        if not torch.cuda.is_available():
            raise RuntimeError("StokesIBBatch needs a HIP device")
        descs = (_lib.Desc * len(systems))()
        keep = []
        for i, sy in enumerate(systems):
            d, k = _make_desc(sy, precision)
            descs[i] = d
            keep.append(k)
        self.nsys = len(systems)
        self.sizes = [int(sy.N) for sy in systems]
        self.precision = precision
        nb = ctypes.c_size_t()
        st = self.lib.ibmg_batch_workspace_bytes(self.nsys, descs, ctypes.byref(nb))
        if st != 0:
            raise IbmgError(st, self.lib.ibmg_last_error(None).decode())
        self.workspace_bytes = nb.value
        self.workspace = _workspace(self.lib, nb.value, workspace_headroom)
        h = ctypes.c_void_p()
        st = self.lib.ibmg_batch_create(self.nsys, descs, _ptr(self.workspace), self.workspace.numel(), _stream(),
                                        ctypes.byref(h))
        if st != 0:
            raise IbmgError(st, self.lib.ibmg_last_error(None).decode())
        self.h = h
        self.n_levels = len(self.stats()["levels"])

    def _check(self, st, ok=(0,)):
        if st not in ok:
            raise IbmgError(st, self.lib.ibmg_last_error(self.h).decode())
        return st

    def close(self):
        if getattr(self, "h", None):
            self.lib.ibmg_destroy(self.h)
            self.h = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    kernel_time = StokesIB.kernel_time
    workspace_used = StokesIB.workspace_used

    def _vecs(self, ts, name):
        if len(ts) != self.nsys:
            raise ValueError(f"{name} must hold {self.nsys} vectors")
        for i, t in enumerate(ts):
            _dev_vec(t, 3 * self.sizes[i] ** 2, f"{name}[{i}]")
        return ts

    def vcycle(self, rs):
        self._vecs(rs, "r")
        zs = [torch.empty(3 * N * N, dtype=torch.float64, device="cuda") for N in self.sizes]
        self._check(self.lib.ibmg_batch_vcycle(self.h, _ptr_array(rs), _ptr_array(zs), _stream()))
        return zs

    def solve(self, bs, rtol=1e-8, restart=30, max_it=100, x0=None, history=128):
        self._vecs(bs, "b")
        if x0 is not None:
            xs = [x.clone() for x in self._vecs(x0, "x0")]
        else:
            xs = [torch.empty(3 * N * N, dtype=torch.float64, device="cuda") for N in self.sizes]
        o = _lib.SolveOpts(float(rtol), int(restart), int(max_it), 1 if x0 is not None else 0, 0)
        infos = (_lib.SolveInfo * self.nsys)()
        hists = []
        for i in range(self.nsys):
            hb = (ctypes.c_double * history)()
            hists.append(hb)
            infos[i].history = ctypes.cast(hb, ctypes.POINTER(ctypes.c_double))
            infos[i].history_cap = history
        st = self._check(self.lib.ibmg_batch_fgmres_solve(self.h, _ptr_array(bs), _ptr_array(xs),
                                                          ctypes.byref(o), infos, _stream()), ok=(0, 1))
        out = []
        for i in range(self.nsys):
            inf = infos[i]
            k = min(inf.iters, history)
            out.append(dict(converged=inf.rel_res_est <= rtol, iters=inf.iters, restarts=inf.restarts,
                            rel_res_est=inf.rel_res_est, rel_res_true=inf.rel_res_true,
                            rhs_null_norm=inf.rhs_null_norm, setup_ms=inf.setup_ms, solve_ms=inf.solve_ms,
                            vcycles=inf.vcycles,
                            history=list(hists[i][:k])))
        return xs, dict(status=_STATUS[st], converged=st == 0, systems=out)

    def stats(self):
        buf = (ctypes.c_int64 * 1024)()
        wr = ctypes.c_int32()
        self._check(self.lib.ibmg_batch_stats(self.h, buf, 1024, ctypes.byref(wr)))
        v = list(buf[:wr.value])
        out = dict(nsys=v[0], levels=[])
        for l in range(v[1]):
            N, nact, n_int, n_ib, rows, tb, grid, ns = v[2 + 8 * l:10 + 8 * l]
            out["levels"].append(dict(N=N, systems=nact, interior_boxes=n_int, ib_boxes=n_ib, ib_rows=rows,
                                      tile=tb, grid=grid, sweep_us=ns / 1e3))
        return out
