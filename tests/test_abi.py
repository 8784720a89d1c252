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
    for bad in (dict(N=48), dict(N=33), dict(coarse_N=2), dict(mu=0.0), dict(dt=-1.0),
                dict(rho=float("nan")), dict(nu1=0), dict(box=5), dict(precision=7), dict(smoother=3),
                dict(M=-1)):
        st = lib.ibmg_create(ctypes.byref(desc(**bad)), None, ctypes.byref(h))
        assert st == _lib.IBMG_ERR_ARG, (bad, st)
        assert lib.ibmg_last_error(None)
    Xbad = np.array([[0.5, 1.5], [0.6, 0.5]])
    d = desc()
    d.X = Xbad.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ibmg_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    e2 = np.array([[0, 5]], dtype=np.int32)
    d = desc()
    d.ends = e2.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    assert lib.ibmg_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    # spring model: unknown model, rest lengths without the tangent model, a
    # negative rest length, and a zero-length spring with a rest length
    rest = np.array([0.05])
    neg = np.array([-0.05])
    rp = rest.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    for bad in (dict(spring_model=2), dict(rest=rp),
                dict(spring_model=1, rest=neg.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))):
        assert lib.ibmg_create(ctypes.byref(desc(**bad)), None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG, bad
    Xz = np.array([[0.5, 0.5], [0.5, 0.5]])
    d = desc(spring_model=1, rest=rp)
    d.X = Xz.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.ibmg_create(ctypes.byref(d), None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
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
                {(1, "rho"): 1.0}, {(1, "N"): 40}, {(0, "dt"): 2e-3}, {(2, "spring_model"): 1}):
        st = lib.ibmg_batch_create(3, descs(3, bad), None, ctypes.byref(h))
        assert st == _lib.IBMG_ERR_ARG, (bad, st)
        assert lib.ibmg_last_error(None)
    assert lib.ibmg_batch_create(0, descs(1), None, ctypes.byref(h)) == _lib.IBMG_ERR_ARG
    n = ctypes.c_int32()
    assert lib.ibmg_batch_size(None, ctypes.byref(n)) == _lib.IBMG_ERR_STATE
    assert lib.ibmg_batch_vcycle(None, None, None, None) == _lib.IBMG_ERR_STATE
