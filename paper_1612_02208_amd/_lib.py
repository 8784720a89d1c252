"""ctypes declarations of libibmg (include/ibmg.h).  Argument marshalling only."""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libibmg.so")

IBMG_OK = 0
IBMG_NOT_CONVERGED = 1
IBMG_ERR_ARG = -1
IBMG_ERR_HIP = -2
IBMG_ERR_WORKSPACE = -3
IBMG_ERR_BREAKDOWN = -4
IBMG_ERR_NONFINITE = -5
IBMG_ERR_STATE = -6

RAS, SC, RMS = 0, 1, 2
SPRING_LINEAR, SPRING_TANGENT = 0, 1
FP64, FP32_SMOOTHER = 0, 1
COMBINE_RESTRICTED, COMBINE_SUM = 0, 1
SWEEP_FGMRES, SWEEP_RICHARDSON = 0, 1

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


class Desc(ctypes.Structure):
    _fields_ = [
        ("N", ctypes.c_int32), ("coarse_N", ctypes.c_int32),
        ("rho", ctypes.c_double), ("mu", ctypes.c_double), ("dt", ctypes.c_double),
        ("M", ctypes.c_int32), ("X", _dp),
        ("n_springs", ctypes.c_int32), ("ends", _ip), ("kappa", _dp),
        ("smoother", ctypes.c_int32), ("box", ctypes.c_int32), ("overlap", ctypes.c_int32),
        ("nu1", ctypes.c_int32), ("nu2", ctypes.c_int32), ("cheb_its", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("spring_model", ctypes.c_int32), ("rest", _dp),
        ("combine", ctypes.c_int32), ("sweep_kind", ctypes.c_int32), ("max_restart", ctypes.c_int32),
    ]


class SolveOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("restart", ctypes.c_int32),
                ("max_it", ctypes.c_int32), ("use_x0", ctypes.c_int32),
                ("transpose", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("restarts", ctypes.c_int32),
                ("rel_res_est", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("rhs_null_norm", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double),
                ("history", _dp), ("history_cap", ctypes.c_int32), ("vcycles", ctypes.c_int32)]


EXPORTS = [
    "ibmg_workspace_bytes", "ibmg_create", "ibmg_workspace_used", "ibmg_destroy", "ibmg_last_error", "ibmg_levels", "ibmg_level_n",
    "ibmg_apply_A_IB", "ibmg_apply_A_IB_T", "ibmg_spread", "ibmg_interp", "ibmg_restrict",
    "ibmg_prolong_add", "ibmg_smoother_apply", "ibmg_smooth", "ibmg_coarse_solve", "ibmg_vcycle",
    "ibmg_fgmres_solve", "ibmg_spring_gradient", "ibmg_spring_gradient_static", "ibmg_set_kappa", "ibmg_stats", "ibmg_sc_info",
    "ibmg_batch_workspace_bytes", "ibmg_batch_create", "ibmg_batch_size", "ibmg_batch_vcycle", "ibmg_batch_fgmres_solve",
    "ibmg_batch_stats", "ibmg_kernel_time", "ibmg_step_rhs", "ibmg_time_step", "ibmg_positions",
]

KERNEL_RAS_IB, KERNEL_RAS_INTERIOR, KERNEL_STENCIL, KERNEL_RAS_BATCH = 0, 1, 2, 3
KERNEL_RESTRICT, KERNEL_PROLONG, KERNEL_SPREAD, KERNEL_INTERP = 4, 5, 6, 7
KERNEL_APPLY_DOTS, KERNEL_UPD_DOTS, KERNEL_UPD_NORM, KERNEL_SCALE_RED, KERNEL_COMBINE_LS = 8, 9, 10, 11, 12
KERNEL_SCALE_UPD = 13

_lib = None


def load():
    """Load libibmg.so from the package directory; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libibmg.so is not built ({LIB_PATH}); run paper_1612_02208_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    sz = ctypes.c_size_t
    lib.ibmg_workspace_bytes.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(sz)]
    lib.ibmg_create.argtypes = [ctypes.POINTER(Desc), vp, sz, vp, ctypes.POINTER(vp)]
    lib.ibmg_workspace_used.argtypes = [vp, ctypes.POINTER(sz), ctypes.POINTER(sz)]
    lib.ibmg_destroy.argtypes = [vp]
    lib.ibmg_last_error.argtypes = [vp]
    lib.ibmg_last_error.restype = ctypes.c_char_p
    lib.ibmg_levels.argtypes = [vp, _ip]
    lib.ibmg_level_n.argtypes = [vp, ctypes.c_int32, _ip]
    for name in ("ibmg_apply_A_IB", "ibmg_apply_A_IB_T", "ibmg_restrict", "ibmg_prolong_add",
                 "ibmg_smoother_apply"):
        getattr(lib, name).argtypes = [vp, ctypes.c_int32, vp, vp, vp]
    lib.ibmg_smooth.argtypes = [vp, ctypes.c_int32, vp, vp, ctypes.c_int32, vp]
    for name in ("ibmg_spread", "ibmg_interp", "ibmg_coarse_solve", "ibmg_vcycle"):
        getattr(lib, name).argtypes = [vp, vp, vp, vp]
    lib.ibmg_fgmres_solve.argtypes = [vp, vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    lib.ibmg_spring_gradient.argtypes = [vp, vp, vp, vp, vp]
    lib.ibmg_spring_gradient_static.argtypes = [vp, vp, vp, vp, vp]
    lib.ibmg_set_kappa.argtypes = [vp, _dp, vp]
    lib.ibmg_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, _ip]
    lib.ibmg_sc_info.argtypes = [vp, ctypes.c_int32, _dp, _ip]
    lib.ibmg_batch_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc), ctypes.POINTER(sz)]
    lib.ibmg_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Desc), vp, sz, vp, ctypes.POINTER(vp)]
    lib.ibmg_batch_size.argtypes = [vp, _ip]
    vpp = ctypes.POINTER(vp)
    lib.ibmg_batch_vcycle.argtypes = [vp, vpp, vpp, vp]
    lib.ibmg_batch_fgmres_solve.argtypes = [vp, vpp, vpp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    lib.ibmg_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, _ip]
    lib.ibmg_kernel_time.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, _dp, _dp, _dp]
    lib.ibmg_step_rhs.argtypes = [vp, vp, vp, vp]
    lib.ibmg_time_step.argtypes = [vp, vp, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo), vp]
    lib.ibmg_positions.argtypes = [vp, _dp]
    for name in EXPORTS:
        if name != "ibmg_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib
