"""The allocation-free spring gradient (ibmg_spring_gradient_static) against
the workspace entry point ibmg_spring_gradient, both called through the C
ABI: two structures in a row on one GPU (the second smaller, with tangent
springs), each result equal bit for bit to the workspace entry point's (the
same kernels on the same inputs) and to the oracle's gradient within the
operator bound; a structure beyond the scratch's 2^18 points is rejected.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from oracle.solver import spring_gradient

pytestmark = pytest.mark.gpu


def _call(lib, fn, G, w, lam):
    from paper_1612_02208_amd.solver import _stream
    out = torch.full((max(G.E, 1),), float("nan"), dtype=torch.float64, device="cuda")
    st = fn(G.h, ctypes.c_void_p(w.data_ptr()), ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(out.data_ptr()),
            _stream())
    assert st == 0, lib.ibmg_last_error(G.h)
    torch.cuda.synchronize()
    return out[:G.E].cpu().numpy()


def _tangent_32():
    wl = W.plain_32(spring_model="tangent")
    d = wl.X[wl.springs[:, 1]] - wl.X[wl.springs[:, 0]]
    d -= np.round(d)
    wl.rest = 0.8 * np.hypot(d[:, 0], d[:, 1])
    return wl


def test_static_gradient_matches_workspace_gradient():
    from paper_1612_02208_amd import StokesIB, _lib
    lib = _lib.load()
    for k, wl in enumerate((W.diff_256(), _tangent_32())):
        print(f"[case] static gradient {wl.name} N={wl.N} M={wl.M} springs={len(wl.springs)}", flush=True)
        G = StokesIB(wl)
        rng = np.random.default_rng(60 + k)
        n = 3 * wl.N * wl.N
        wh, lh = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
        w = torch.from_numpy(wh).cuda()
        lam = torch.from_numpy(lh).cuda()
        g_ws = _call(lib, lib.ibmg_spring_gradient, G, w, lam)
        g_st = _call(lib, lib.ibmg_spring_gradient_static, G, w, lam)
        assert np.array_equal(g_st, g_ws), k
        go = spring_gradient(wl, wh, lh)
        assert np.linalg.norm(g_st - go) <= 1e-12 * np.linalg.norm(go), k
        # a second call on the same structure gives the same bits
        assert np.array_equal(_call(lib, lib.ibmg_spring_gradient_static, G, w, lam), g_ws)
        G.close()


def test_static_gradient_rejects_structures_beyond_its_scratch():
    from paper_1612_02208_amd import IbmgError, StokesIB, _lib
    lib = _lib.load()
    M = (1 << 18) + 1
    X = np.random.default_rng(61).uniform(0.0, 1.0, (M, 2))
    wl = W.Workload("points_beyond_scratch", 32, 8, 0.0, 1.0, 1e-2, X, np.zeros((0, 2), dtype=np.int32),
                    np.zeros(0))
    G = StokesIB(wl)
    z = torch.zeros(3 * 32 * 32, dtype=torch.float64, device="cuda")
    from paper_1612_02208_amd.solver import _stream
    st = lib.ibmg_spring_gradient_static(G.h, ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                         None, _stream())
    assert st == _lib.IBMG_ERR_ARG
    assert b"allocation-free gradient holds" in lib.ibmg_last_error(G.h)
    G.close()
