"""CPU checks of the C ABI boundary: the library is built, loads, and exports
every entry point that include/ibmg.h declares; the binding declares the same
set.  No compute call is made (there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ibmg.h")
LIB = os.path.join(ROOT, "paper_1612_02208_amd", "libibmg.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibmg_[a-z_A-Z0-9]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("ibmg_apply_A_IB", "ibmg_spread", "ibmg_interp", "ibmg_vcycle", "ibmg_fgmres_solve"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_matches_header():
    from paper_1612_02208_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_create_rejects_bad_descriptors_without_a_device():
    """Argument validation runs on the host before any device work."""
    import numpy as np
    from paper_1612_02208_amd import _lib
    lib = _lib.load()
    X = np.array([[0.5, 0.5], [0.6, 0.5]])
    ends = np.array([[0, 1]], dtype=np.int32)
    kap = np.array([1.0])

    def desc(**kw):
        d = _lib.Desc()
        d.N, d.coarse_N, d.rho, d.mu, d.dt = 32, 8, 0.0, 1.0, 1e-2
        d.M, d.n_springs = 2, 1
        d.X = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.ends = ends.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        d.kappa = kap.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        d.smoother, d.box, d.overlap, d.nu1, d.nu2, d.cheb_its, d.precision = 0, 8, 2, 2, 2, 2, 0
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    h = ctypes.c_void_p()
    for bad in (dict(N=48), dict(N=33), dict(coarse_N=2), dict(coarse_N=32), dict(mu=0.0), dict(dt=-1.0),
                dict(rho=float("nan")), dict(nu1=0), dict(box=5), dict(precision=7), dict(smoother=3),
                dict(M=-1), dict(combine=2), dict(combine=1, smoother=2), dict(combine=1, smoother=1),
                dict(sweep_kind=2), dict(max_restart=65), dict(max_restart=-1)):
        st = lib.ibmg_create(ctypes.byref(desc(**bad)), None, 0, None, ctypes.byref(h))
        assert st == _lib.IBMG_ERR_ARG, (bad, st)
        assert lib.ibmg_last_error(None)
    Xbad = np.array([[0.5, 1.5], [0.6, 0.5]])
    d = desc()
    d.X = Xbad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ibmg_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    e2 = np.array([[0, 5]], dtype=np.int32)
    d = desc()
    d.ends = e2.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.ibmg_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    # spring model: unknown model, rest lengths without the tangent model, a
    # negative rest length, and a zero-length spring with a rest length
    rest = np.array([0.05])
    neg = np.array([-0.05])
    rp = rest.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for bad in (dict(spring_model=2), dict(rest=rp),
                dict(spring_model=1, rest=neg.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))):
        assert lib.ibmg_create(ctypes.byref(desc(**bad)), None, 0, None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG, bad
    Xz = np.array([[0.5, 0.5], [0.5, 0.5]])
    d = desc(spring_model=1, rest=rp)
    d.X = Xz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ibmg_create(ctypes.byref(d), None, 0, None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    assert b"zero length" in lib.ibmg_last_error(None)
    assert lib.ibmg_destroy(None) == _lib.IBMG_ERR_STATE


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_batch_create_rejects_mismatched_systems_without_a_device():
    """The batched form checks every descriptor and the shared parameters on
    the host; single-system calls on no handle report a state error."""
    import numpy as np
    from paper_1612_02208_amd import _lib
    lib = _lib.load()
    X = np.array([[0.5, 0.5], [0.6, 0.5]])
    ends = np.array([[0, 1]], dtype=np.int32)
    kap = np.array([1.0])

    def descs(n, changes=None):
        arr = (_lib.Desc * n)()
        for i in range(n):
            d = arr[i]
            d.N, d.coarse_N, d.rho, d.mu, d.dt = 32 if i % 2 == 0 else 64, 8, 0.0, 1.0, 1e-3
            d.M, d.n_springs = 2, 1
            d.X = X.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.ends = ends.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.kappa = kap.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            d.smoother, d.box, d.overlap, d.nu1, d.nu2, d.cheb_its, d.precision = 0, 8, 2, 2, 2, 2, 1
        for (i, k), v in (changes or {}).items():
            setattr(arr[i], k, v)
        return arr

    h = ctypes.c_void_p()
    for bad in ({(1, "mu"): 0.5}, {(1, "box"): 4}, {(0, "smoother"): 1}, {(1, "precision"): 0},
                {(1, "rho"): 1.0}, {(1, "N"): 40}, {(0, "dt"): 2e-3}, {(2, "spring_model"): 1},
                {(1, "combine"): 1}, {(0, "sweep_kind"): 1}):
        st = lib.ibmg_batch_create(3, descs(3, bad), None, 0, None, ctypes.byref(h))
        assert st == _lib.IBMG_ERR_ARG, (bad, st)
        assert lib.ibmg_last_error(None)
    assert lib.ibmg_batch_create(0, descs(1), None, 0, None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    n = ctypes.c_int32()
    assert lib.ibmg_batch_size(None, ctypes.byref(n)) == _lib.IBMG_ERR_STATE
    assert lib.ibmg_batch_vcycle(None, None, None, None) == _lib.IBMG_ERR_STATE


def _desc_of(wl, precision="fp64", max_restart=30):
    from paper_1612_02208_amd.solver import _make_desc
    wl.max_restart = max_restart
    return _make_desc(wl, precision)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_workspace_sizing_runs_without_a_device():
    """ibmg_workspace_bytes runs the set-up's planning with no device work:
    it answers here, with no GPU, and the same descriptor always gets the
    same size.  The size holds at least the outer FGMRES basis of
    max_restart, and the FP32-smoother form needs less than the FP64 one
    (its box inverses are half the size)."""
    import workloads as W
    from paper_1612_02208_amd import _lib
    lib = _lib.load()
    X, S = W.annulus(4, 150, 0.2, 0.25)
    import numpy as np
    cases = [W.plain_32(), W.plain_32(smoother="sc"), W.plain_32(smoother="rms"),
             W.plain_32(combine="sum"), W.plain_32(sweep="richardson"),
             W.Workload("annulus_64_box16", 64, 8, 1.0, 1e-2, 5e-4, X, S, np.full(len(S), 1e4), box=16, overlap=4)]
    for wl in cases:
        sizes = {}
        for prec in ("fp64", "fp32"):
            d, keep = _desc_of(wl, prec)
            nb = ctypes.c_size_t()
            assert lib.ibmg_workspace_bytes(ctypes.byref(d), ctypes.byref(nb)) == _lib.IBMG_OK, \
                lib.ibmg_last_error(None)
            nb2 = ctypes.c_size_t()
            assert lib.ibmg_workspace_bytes(ctypes.byref(d), ctypes.byref(nb2)) == _lib.IBMG_OK
            assert nb.value == nb2.value and nb.value % 256 == 0
            n = 3 * wl.N * wl.N
            assert nb.value >= (2 * 30 + 1) * n * 8
            sizes[prec] = nb.value
        assert sizes["fp32"] < sizes["fp64"], wl.name
        d, keep = _desc_of(wl, "fp64", max_restart=60)
        nb = ctypes.c_size_t()
        assert lib.ibmg_workspace_bytes(ctypes.byref(d), ctypes.byref(nb)) == _lib.IBMG_OK
        assert nb.value >= sizes["fp64"] + 60 * 3 * wl.N * wl.N * 8
    # the summed combination keeps whole box inverses: more than the owned rows
    d1, k1 = _desc_of(W.plain_32(), "fp64")
    d2, k2 = _desc_of(W.plain_32(combine="sum"), "fp64")
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    lib.ibmg_workspace_bytes(ctypes.byref(d1), ctypes.byref(a))
    lib.ibmg_workspace_bytes(ctypes.byref(d2), ctypes.byref(b))
    assert b.value > a.value
    # a bad descriptor fails the sizing call as it fails create
    d, keep = _desc_of(W.plain_32(), "fp64")
    d.mu = -1.0
    assert lib.ibmg_workspace_bytes(ctypes.byref(d), ctypes.byref(a)) == _lib.IBMG_ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_batch_workspace_sizing_runs_without_a_device():
    import workloads as W
    from paper_1612_02208_amd import _lib
    lib = _lib.load()
    systems = W.batch_systems(6)
    arr = (_lib.Desc * len(systems))()
    keep = []
    for i, sy in enumerate(systems):
        d, k = _desc_of(sy, "fp32")
        arr[i] = d
        keep.append(k)
    nb = ctypes.c_size_t()
    assert lib.ibmg_batch_workspace_bytes(len(systems), arr, ctypes.byref(nb)) == _lib.IBMG_OK, \
        lib.ibmg_last_error(None)
    tot = sum(3 * s.N * s.N for s in systems)
    assert nb.value >= 61 * tot * 8


@pytest.mark.skipif(not os.path.exists(LIB), reason="libibmg.so not built")
def test_create_rejects_missing_or_misaligned_workspace():
    """The workspace is checked on the host before any device work."""
    import workloads as W
    from paper_1612_02208_amd import _lib
    lib = _lib.load()
    d, keep = _desc_of(W.plain_32(), "fp64")
    h = ctypes.c_void_p()
    assert lib.ibmg_create(ctypes.byref(d), None, 1 << 30, None, ctypes.byref(h)) == _lib.IBMG_ERR_WORKSPACE
    assert lib.ibmg_create(ctypes.byref(d), ctypes.c_void_p(4096 + 8), 1 << 30, None,
                           ctypes.byref(h)) == _lib.IBMG_ERR_WORKSPACE
    assert b"aligned" in lib.ibmg_last_error(None)
    u, p = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.ibmg_workspace_used(None, ctypes.byref(u), ctypes.byref(p)) == _lib.IBMG_ERR_STATE
