"""Benchmark: solve time to 1e-8 relative residual and V-cycles/s at N = 512,
FP32 smoother against FP64, on one MI355X.

Workload: 512 x 512 periodic grid, rho = 1, mu = 1e-2, dt = 5e-4; elastic
annulus between radii 0.2 and 0.25 (4 rings x 2048 points, ring and radial
springs, kappa = 1e4); 7-level V-cycle (512 -> 8), restricted additive Schwarz
on 16 x 16 boxes with overlap 4 (--box/--overlap), 2 + 2 FGMRES smoothing
iterations, outer FGMRES(30) to 1e-8; seeded uniform[-1, 1] right-hand side.

One step = one FP64 solve plus one FP32-smoother solve of the same
right-hand side, both to 1e-8 (set-up excluded; inputs resident in HBM).
``value`` = V-cycles applied in the timed steps / timed wall time.

Also reported: the roofline of the dominant kernel (k_ras_ib_sym<double>
with its sums: the finest level's Schwarz boxes with their own inverse,
streamed from the symmetric storage of their owned rows), timed alone with HIP
events on the stream it runs on; the other hot kernels, the smoothing step's
Krylov kernels among them; each solve's true residual under the oracle's
operator, and at 128^2 (the same structure) the distance of both precisions'
solutions to the oracle's; the plain 32^2 system and the 256^2 smoother
comparison (four stiffnesses, additive Schwarz and the Schur-complement
smoother) against the oracle; the differentiation workload (forward and
adjoint solves, gradient kernel, gradient against the oracle's); the batched
form on 64 independent systems (N in {64, 128, 256}, FP32 smoother); and the
FP64 CPU oracle on a bounded sample, its complete V-cycles and solves timed
with set-up apart.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-baseline sample|off]
                    [--batch on|off] [--rms on|off] [--step on|off] [--configs on|off]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solve time to 1e-8 rel-res & V-cycles/s at N=512; FP32 smoother vs FP64"
HBM_PEAK_GBS = 8000.0
FP64_MFMA_PEAK_TFS = 78.6
FP32_MFMA_PEAK_TFS = 157.3
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_ras_ib_annulus512.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1612_02208_amd", "csrc", "dense_kernels.hip")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--N", type=int, default=512)
    p.add_argument("--cpu-baseline", default="sample", choices=["sample", "off"])
    p.add_argument("--cpu-boxes", type=int, default=128)
    p.add_argument("--roofline-reps", type=int, default=50)
    # 16 x 16 boxes with overlap 4: at mu = 1e-2 the paper finds that only the
    # largest boxes and overlaps give an effective smoother (Sec. 5.1.1, 5.2.1);
    # here they need 30 iterations against 76 for 8 x 8 / 2 and solve faster
    p.add_argument("--box", type=int, default=16)
    p.add_argument("--overlap", type=int, default=4)
    p.add_argument("--batch", default="on", choices=["on", "off"])
    p.add_argument("--rms", default="on", choices=["on", "off"])
    p.add_argument("--step", default="on", choices=["on", "off"])
    p.add_argument("--tangent", default="on", choices=["on", "off"])
    p.add_argument("--large", default="on", choices=["on", "off"])
    p.add_argument("--configs", default="on", choices=["on", "off"])
    return p.parse_args()


def measured_traffic(alg_bytes):
    """HBM bytes per launch of the IB-box sweep (k_ras_ib_sym and its sums) from the committed
    rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE passes, each scaled by what the
    same counter reads for a plain copy of known size; None when no
    counters are recorded or the kernel source changed since they were."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    rec = json.load(open(TRAFFIC_FILE))
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if rec.get("kernel_source_sha256") != sha:
        return None
    f_fetch = rec["copy_bytes_read"] / (rec["copy_fetch_kib"] * 1024.0)
    f_write = rec["copy_bytes_written"] / (rec["copy_write_kib"] * 1024.0)
    return rec["fetch_kib"] * 1024.0 * f_fetch + rec["write_kib"] * 1024.0 * f_write


def smoother_bench(wl, b, smoother, box, overlap, reps=3):
    """FP64 solve of the same workload and right-hand side with another
    smoother: iterations, solve time and V-cycle rate."""
    import copy
    import torch
    from paper_1612_02208_amd import StokesIB
    w2 = copy.copy(wl)
    w2.smoother, w2.box, w2.overlap = smoother, box, overlap
    t0 = time.perf_counter()
    g = StokesIB(w2, precision="fp64")
    setup = time.perf_counter() - t0
    x = torch.empty_like(b)
    g.solve(b, rtol=1e-8, out=x)
    ms, info = [], None
    for _ in range(reps):
        _, info = g.solve(b, rtol=1e-8, out=x)
        ms.append(info["solve_ms"])
    st = g.stats()["levels"]
    g.close()
    return {"smoother": smoother, "box": box, "overlap": overlap, "iters": info["iters"],
            "solve_ms": float(np.median(ms)), "vcycles_per_s": info["vcycles"] / (float(np.median(ms)) / 1e3),
            "rel_res_true": info["rel_res_true"], "setup_s": setup,
            "box_colours": [lv["box_colours"] for lv in st[1:]]}


def step_bench(wl, b):
    """One semi-implicit time step of the same workload (FP64): right-hand
    side, solve to 1e-8, position update and the rebuild of every level at
    the moved structure (box inverses included)."""
    import copy
    import torch
    from paper_1612_02208_amd import StokesIB
    g = StokesIB(copy.copy(wl), precision="fp64")
    w = torch.zeros_like(b)
    g.time_step(w, rtol=1e-8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    w2, info = g.time_step(w, rtol=1e-8)
    torch.cuda.synchronize()
    total = 1e3 * (time.perf_counter() - t0)
    X = g.positions()
    g.close()
    return {"step_ms": total, "solve_ms": info["solve_ms"], "rebuild_ms": info["rebuild_ms"],
            "rest_ms": total - info["solve_ms"] - info["rebuild_ms"],
            "iters": info["iters"], "rel_res_true": info["rel_res_true"],
            "max_displacement": float(np.abs(X - wl.X).max())}


def tangent_bench(wl, b, reps=3):
    """The same workload with tangent springs (rest lengths 0.7 of the
    springs' lengths, so every spring is stretched): FP64 and FP32-smoother
    solves to 1e-8, the explicit IB-row entries against the linear model's,
    and one FP64 time step (right-hand side with the nonlinear force, solve,
    position update, rebuild with the tangent blocks at X^{n+1})."""
    import copy
    import torch
    from paper_1612_02208_amd import StokesIB
    d = wl.X[wl.springs[:, 1]] - wl.X[wl.springs[:, 0]]
    d -= np.round(d)
    w2 = copy.copy(wl)
    w2.spring_model, w2.rest = "tangent", 0.7 * np.hypot(d[:, 0], d[:, 1])
    out = {"rest": "0.7 x spring length"}
    for prec in ("fp64", "fp32"):
        t0 = time.perf_counter()
        g = StokesIB(w2, precision=prec)
        setup = time.perf_counter() - t0
        x = torch.empty_like(b)
        g.solve(b, rtol=1e-8, out=x)
        ms, info = [], None
        for _ in range(reps):
            _, info = g.solve(b, rtol=1e-8, out=x)
            ms.append(info["solve_ms"])
        med = float(np.median(ms))
        out[prec] = {"iters": info["iters"], "solve_ms": med, "vcycles_per_s": info["vcycles"] / (med / 1e3),
                     "rel_res_true": info["rel_res_true"], "setup_s": setup}
        if prec == "fp64":
            out["ib_row_entries"] = sum(lv["ib_nnz"] for lv in g.stats()["levels"])
            w = torch.zeros_like(b)
            g.time_step(w, rtol=1e-8)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, si = g.time_step(w, rtol=1e-8)
            torch.cuda.synchronize()
            tot = 1e3 * (time.perf_counter() - t0)
            out["time_step"] = {"step_ms": tot, "solve_ms": si["solve_ms"], "rebuild_ms": si["rebuild_ms"],
                                "iters": si["iters"]}
        g.close()
    g = StokesIB(wl, precision="fp64")
    out["ib_row_entries_linear"] = sum(lv["ib_nnz"] for lv in g.stats()["levels"])
    g.close()
    return out


def large_bench(reps=20):
    """The grid and coupling kernels where their data cannot stay in the
    caches: a 4096^2 periodic grid (fields of 400 MB), FP64, with 2^20 points
    and no springs, in two layouts: a suspension of 32 x 32 membranes of
    1024 points each (radius 0.35/32, points in fibre order, as the paper's
    structures come) and the same count scattered uniformly (seed 7, no
    spatial order: the worst case for the point gathers).  Stencil,
    restriction and prolongation on the finest level, spreading and
    interpolation of all points; algorithmic bytes as for the main
    workload."""
    import torch
    import workloads as W
    from paper_1612_02208_amd import StokesIB
    N, M = 4096, 1 << 20
    out = {}
    layouts = (("suspension", W.suspension_points(32, 0.35 / 32, 1024)), ("uniform_random", W.random_points(M, 7)))
    for tag, X in layouts:
        wl = W.Workload(f"grid_{N}_{tag}", N, 8, 1.0, 1e-2, 5e-4, X, np.zeros((0, 2), dtype=np.int32),
                        np.zeros(0), box=8, overlap=2)
        t0 = time.perf_counter()
        g = StokesIB(wl, precision="fp64")
        rec = {"workload": f"{N}x{N} periodic grid, {X.shape[0]} points ({tag.replace('_', ' ')}), "
                           f"no springs, FP64", "setup_s": time.perf_counter() - t0}
        kinds = (("stencil", "k_apply<double>"), ("restrict", "k_restrict<double>"),
                 ("prolong", "k_prolong_add<double>"), ("spread", "k_spread"), ("interp", "k_interp_lanes<double>"))
        for kind, name in kinds:
            if tag != "suspension" and kind in ("stencil", "restrict", "prolong"):
                continue   # the grid kernels do not see the points
            t = g.kernel_time(kind, -1, reps)
            rec[name] = {"bound": "hbm", "avg_ms": t["ms"], "alg_bytes": t["bytes"],
                         "gbs": t["bytes"] / t["ms"] / 1e6, "frac": t["bytes"] / t["ms"] / 1e6 / HBM_PEAK_GBS}
        g.close()
        out[tag] = rec
    torch.cuda.synchronize()
    return out


def batch_bench(dev, reps=3):
    """The batched form: 64 independent systems (N in {64, 128, 256}, kappa
    log-uniform in [1e1, 1e5], membranes of 4N points), FP32 smoother, each
    solved to 1e-8; set-up (with the tile autotuner) timed separately."""
    import torch
    import workloads as W
    from paper_1612_02208_amd import StokesIBBatch
    systems = W.batch_systems(64)
    t0 = time.perf_counter()
    B = StokesIBBatch(systems, precision="fp32")
    setup = time.perf_counter() - t0
    bs = [torch.from_numpy(W.rhs(s.N, s.rhs_seed)).to(dev) for s in systems]
    B.solve(bs, rtol=1e-8)
    torch.cuda.synchronize()
    times, info = [], None
    for _ in range(reps):
        t0 = time.perf_counter()
        _, info = B.solve(bs, rtol=1e-8)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    its = [si["iters"] for si in info["systems"]]
    st = B.stats()
    top = st["levels"][-1]
    kt = B.kernel_time("ras_batch", -1, 20)
    out = {"workload": "64 systems, N in {64,128,256} (counts %s), Stokes mu=1 dt=1e-3, membranes r~U[0.15,0.3] "
                       "with 4N points, kappa log-uniform [1e1,1e5], RAS 8x8/2, FP32 smoother, FGMRES to 1e-8"
                       % {n: sum(1 for s in systems if s.N == n) for n in (64, 128, 256)},
           "converged": info["converged"], "solve_ms": 1e3 * t, "systems_per_s": 64 / t,
           "vcycles_per_s": sum(its) / t, "iters_min": min(its), "iters_max": max(its),
           "max_rel_res_true": max(si["rel_res_true"] for si in info["systems"]), "setup_s": setup,
           "tuned_plans": [dict(N=lv["N"], systems=lv["systems"], tile=lv["tile"], grid=lv["grid"],
                                sweep_us=lv["sweep_us"]) for lv in st["levels"][1:]],
           "ras_batch_finest": {"kernel": "k_ras_batch<float>", "N": top["N"], "systems": top["systems"],
                                "avg_ms": kt["ms"], "alg_bytes": kt["bytes"],
                                "achieved_gbs": kt["bytes"] / kt["ms"] / 1e6,
                                "frac_hbm": kt["bytes"] / kt["ms"] / 1e6 / HBM_PEAK_GBS}}
    B.close()
    return out


def oracle_operator(wl):
    """The oracle's finest-level L_IB (assembled sparse, FP64) and the
    projection of the right-hand side onto its range."""
    from oracle import hierarchy, ib as oib, mac
    N = wl.N
    if getattr(wl, "spring_model", "linear") == "tangent":
        IB = oib.ib_term_tangent(wl.X, wl.springs, wl.kappa, wl.rest, N, wl.dt)
    else:
        IB = oib.ib_term(wl.X, wl.springs, wl.kappa, N, wl.dt)
    L = mac.stokes_ib((mac.momentum(N, wl.rho, wl.mu, wl.dt) + IB).tocsr(), mac.gradient(N), mac.divergence(N))
    return L.tocsr(), (lambda v: hierarchy.project_range(v, N, wl.rho))


def true_residual(L, proj, b, x):
    bp = proj(b)
    return float(np.linalg.norm(bp - L @ x) / np.linalg.norm(bp))


def rel_err(x, ref):
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def gpu_solve(g, b, rtol=1e-8, reps=3, max_it=100):
    """Median solve time of ``reps`` solves after one warm-up; the last
    solution and info."""
    import torch
    x = torch.empty_like(b)
    g.solve(b, rtol=rtol, out=x, max_it=max_it)
    ms, info = [], None
    for _ in range(reps):
        _, info = g.solve(b, rtol=rtol, out=x, max_it=max_it)
        ms.append(info["solve_ms"])
    torch.cuda.synchronize()
    return x.cpu().numpy(), info, float(np.median(ms))


def c3_oracle_128(dev):
    """The benchmark's structure (4 x 2048-point annulus, kappa = 1e4, rho = 1,
    mu = 1e-2, RAS 16/4) on a 128^2 grid, where the whole oracle runs: both
    precisions' solutions to 1e-8 against the oracle's 1e-12 solution, with
    the oracle's set-up, V-cycle and solve timed."""
    import torch
    import workloads as W
    from oracle.solver import Problem
    from paper_1612_02208_amd import StokesIB
    wl = W.annulus_512(N=128, box=16, overlap=4)
    b_h = W.rhs(wl.N, 0)
    b = torch.from_numpy(b_h).to(dev)
    t0 = time.perf_counter()
    P = Problem(wl)
    t_setup = time.perf_counter() - t0
    r = P.project(b_h)
    t0 = time.perf_counter()
    P.mg.vcycle(r)
    t_vc = time.perf_counter() - t0
    t0 = time.perf_counter()
    xo, io = P.solve(b_h, rtol=1e-8)
    t_solve = time.perf_counter() - t0
    xo12, _ = P.solve(b_h, rtol=1e-12, max_it=200)
    out = {"workload": "annulus 4x2048 points, kappa=1e4, rho=1 mu=1e-2 dt=5e-4, 128x128, 5 levels, RAS 16x16/4",
           "oracle": {"setup_s": t_setup, "vcycle_s": t_vc, "solve_s": t_solve, "iters": io["iters"]}}
    for prec in ("fp64", "fp32"):
        g = StokesIB(wl, precision=prec)
        x, info, ms = gpu_solve(g, b)
        g.close()
        out[prec] = {"iters": info["iters"], "solve_ms": ms, "rel_res_true": true_residual(P.L, P.project, b_h, x),
                     "rel_err_vs_oracle_1e-12": rel_err(x, xo12), "rel_err_vs_oracle_1e-8": rel_err(x, xo)}
    return out


def c1_bench(dev):
    """Plain FP64 solve (32^2 Stokes membrane, 128 points, kappa = 1e2, 3
    levels, RAS 8/2) against the oracle."""
    import torch
    import workloads as W
    from oracle.solver import Problem
    from paper_1612_02208_amd import StokesIB
    wl = W.plain_32()
    b_h = W.rhs(wl.N, 0)
    b = torch.from_numpy(b_h).to(dev)
    g = StokesIB(wl)
    x, info, ms = gpu_solve(g, b, reps=5)
    g.close()
    P = Problem(wl)
    t0 = time.perf_counter()
    xo, io = P.solve(b_h, rtol=1e-8)
    t_solve = time.perf_counter() - t0
    return {"workload": "32x32 Stokes, membrane r=0.25 of 128 points, kappa=1e2, 3 levels, RAS 8x8/2, FP64",
            "iters": info["iters"], "oracle_iters": io["iters"], "solve_ms": ms, "oracle_solve_s": t_solve,
            "rel_res_true": true_residual(P.L, P.project, b_h, x), "rel_err_vs_oracle": rel_err(x, xo)}


def c2_bench(dev):
    """Smoother comparison: 256^2 Stokes membrane of 1024 points, kappa in
    {1, 1e2, 1e4, 1e6}, additive Schwarz 8/2 and the Schur-complement
    smoother, 6 levels, FP64, each to 1e-8.  Every solve's true residual is
    taken under the oracle's operator; the oracle solves too for every SC
    case and for RAS at kappa = 1e4 (its RAS set-up factors 1360 boxes per
    stiffness), and the distance of the solutions is reported."""
    import torch
    import workloads as W
    from oracle.solver import Problem
    from paper_1612_02208_amd import StokesIB
    b_h = W.rhs(256, 0)
    b = torch.from_numpy(b_h).to(dev)
    out = []
    for kappa in (1e0, 1e2, 1e4, 1e6):
        for sm in ("ras", "sc"):
            wl = W.smoother_256(kappa, sm)
            t0 = time.perf_counter()
            g = StokesIB(wl)
            setup = time.perf_counter() - t0
            x, info, ms = gpu_solve(g, b)
            st = g.stats()["levels"]
            g.close()
            rec = {"kappa": kappa, "smoother": sm, "box": "8x8/2" if sm == "ras" else None, "iters": info["iters"],
                   "solve_ms": ms, "vcycles_per_s": info["vcycles"] / (ms / 1e3), "setup_s": setup}
            if sm == "sc" or kappa == 1e4:
                t0 = time.perf_counter()
                P = Problem(wl)
                t_set = time.perf_counter() - t0
                t0 = time.perf_counter()
                xo, io = P.solve(b_h, rtol=1e-8)
                rec.update(oracle_iters=io["iters"], oracle_setup_s=t_set, oracle_solve_s=time.perf_counter() - t0,
                           rel_err_vs_oracle=rel_err(x, xo), rel_res_true=true_residual(P.L, P.project, b_h, x))
            else:
                L, proj = oracle_operator(wl)
                rec["rel_res_true"] = true_residual(L, proj, b_h, x)
            out.append(rec)
            print(f"[bench] C2 kappa={kappa:g} {sm}: {rec['iters']} its, {ms:.1f} ms", file=sys.stderr, flush=True)
    return out


def c5_bench(dev, reps=3):
    """Differentiation form: 256^2 Stokes membrane of 1024 points,
    kappa_i = 1e3 (1 + 0.5 u_i); loss 0.5 ||u - u_t||^2 with u_t from a
    second stiffness field.  Forward solve, adjoint solve (transposed
    operator path) to 1e-12 and the gradient kernel timed apart; the gradient
    against the oracle's (tests/golden/c5_oracle_gradient.txt)."""
    import torch
    import workloads as W
    from paper_1612_02208_amd import StokesIB
    wl, wt = W.diff_256(field_seed=1), W.diff_256(field_seed=2)
    b = torch.from_numpy(W.rhs(256, 0)).to(dev)
    G, Gt = StokesIB(wl), StokesIB(wt)
    ut, _ = Gt.solve(b, rtol=1e-12, max_it=400)
    n2 = 2 * 256 * 256
    fw, aw, gk = [], [], []
    for _ in range(reps + 1):
        w, iw = G.solve(b, rtol=1e-12, max_it=400)
        rhs = torch.zeros_like(w)
        rhs[:n2] = w[:n2] - ut[:n2]
        lam, il = G.solve(rhs, rtol=1e-12, max_it=400, transpose=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(20):
            g = G.spring_gradient(w, lam)
        e1.record()
        torch.cuda.synchronize()
        fw.append(iw["solve_ms"])
        aw.append(il["solve_ms"])
        gk.append(e0.elapsed_time(e1) / 20)
    gh = g.cpu().numpy()
    G.close()
    Gt.close()
    golden = os.path.join(ROOT, "tests", "golden", "c5_oracle_gradient.txt")
    go = np.loadtxt(golden)
    return {"workload": "256x256 Stokes, membrane of 1024 points, kappa_i = 1e3 (1 + 0.5 u_i), loss 0.5|u - u_t|^2",
            "forward_ms": float(np.median(fw[1:])), "forward_iters": iw["iters"],
            "adjoint_ms": float(np.median(aw[1:])), "adjoint_iters": il["iters"],
            "gradient_kernel_ms": float(np.median(gk[1:])), "springs": int(len(wl.springs)),
            "rel_err_vs_oracle_gradient": rel_err(gh, go)}


def cpu_baseline(wl, nboxes):
    """The plain FP64 oracle on the host cores, on a bounded sample of the
    workload.  (1) Complete oracle V-cycles (Alg. 1: FGMRES-wrapped RAS
    smoothing on every level, transfers, the coarsest direct solve) of the
    same structure, fluid, boxes and smoothing on a 128^2 grid, set-up timed
    apart, with all BLAS threads and with one.  (2) The 512^2 finest level's
    box solves (gather, LU solve, owned-set scatter) on ``nboxes`` boxes.
    ``value`` scales (1) to 512^2 by the ratio of box solves per V-cycle
    (every level's boxes, each level at its own box size); the per-box cost
    of (2) checks that the boxes cost the same at both sizes."""
    import scipy.linalg as la
    from threadpoolctl import threadpool_info, threadpool_limits
    import workloads as W
    from oracle import hierarchy, schwarz
    from oracle.solver import Problem

    def box_solves(N):
        sizes = hierarchy.level_sizes(N, wl.coarse_N)[1:]
        return (wl.nu1 + wl.nu2) * sum(len(schwarz.patches(n, wl.box, wl.overlap)) for n in sizes)

    small = W.annulus_512(N=128, box=wl.box, overlap=wl.overlap)
    t0 = time.perf_counter()
    P = Problem(small)
    t_setup = time.perf_counter() - t0
    r = P.project(W.rhs(small.N, 0))

    def vcycle_s(reps=2):
        P.mg.vcycle(r)
        t0 = time.perf_counter()
        for _ in range(reps):
            P.mg.vcycle(r)
        return (time.perf_counter() - t0) / reps

    t_vc128 = vcycle_s()
    with threadpool_limits(limits=1, user_api="blas"):
        t_vc128_1 = vcycle_s(1)
    ratio = box_solves(wl.N) / box_solves(small.N)
    # the 512^2 finest level's box solves on a sample
    fine = hierarchy.build(wl)[-1]
    parts = schwarz.patches(fine.N, wl.box, wl.overlap)
    step = max(1, len(parts) // nboxes)
    sample = parts[::step][:nboxes]
    Lc = fine.L.tocsr()
    facs = [la.lu_factor(Lc[p.idx][:, p.idx].toarray()) for p in sample]
    rr = np.random.default_rng(0).uniform(-1, 1, fine.n)
    z = np.zeros_like(rr)
    t0 = time.perf_counter()
    for p, f in zip(sample, facs):
        y = la.lu_solve(f, rr[p.idx])
        z[p.own_global] = y[p.own_local]
    t_box512 = (time.perf_counter() - t0) / len(sample)
    parts128 = schwarz.patches(small.N, wl.box, wl.overlap)
    L128 = P.levels[-1].L.tocsr()
    f128 = [la.lu_factor(L128[p.idx][:, p.idx].toarray()) for p in parts128[:16]]
    r128 = np.random.default_rng(1).uniform(-1, 1, P.levels[-1].n)
    t0 = time.perf_counter()
    for p, f in zip(parts128[:16], f128):
        la.lu_solve(f, r128[p.idx])
    t_box128 = (time.perf_counter() - t0) / 16
    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    t_vc = t_vc128 * ratio
    return {"value": 1.0 / t_vc, "unit": "V-cycles/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle: complete V-cycles of the same structure, fluid, boxes and smoothing on "
                       f"128x128 ({t_vc128:.2f} s each, set-up {t_setup:.1f} s apart), scaled by the ratio "
                       f"of box solves per V-cycle at {wl.N}x{wl.N} and 128x128 ({ratio:.2f}); box solves "
                       f"cost {t_box512 * 1e3:.2f} ms at {wl.N} ({len(sample)} sampled) and "
                       f"{t_box128 * 1e3:.2f} ms at 128; cores = BLAS threads"),
            "vcycle_s": t_vc, "vcycle_128_s": t_vc128, "setup_128_s": t_setup, "box_solve_ratio": ratio,
            "box_solve_ms_512": 1e3 * t_box512, "box_solve_ms_128": 1e3 * t_box128,
            "cpu_model": model, "host_cpus": os.cpu_count(),
            "single_thread": {"value": 1.0 / (t_vc128_1 * ratio), "vcycle_128_s": t_vc128_1}}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_1612_02208_amd import StokesIB

    wl = W.annulus_512(N=a.N)
    wl.N = a.N
    wl.box, wl.overlap = a.box, a.overlap
    b_h = W.rhs(wl.N, 0)
    torch.cuda.init()
    dev = torch.device("cuda:0")
    b = torch.from_numpy(b_h).to(dev)
    t0 = time.perf_counter()
    g64 = StokesIB(wl, precision="fp64")
    t_setup64 = time.perf_counter() - t0
    t0 = time.perf_counter()
    g32 = StokesIB(wl, precision="fp32")
    t_setup32 = time.perf_counter() - t0
    print(f"[bench] set-up fp64 {t_setup64:.2f}s fp32 {t_setup32:.2f}s", file=sys.stderr, flush=True)

    x64 = torch.empty_like(b)
    x32 = torch.empty_like(b)

    def step():
        _, i64 = g64.solve(b, rtol=1e-8, out=x64)
        _, i32 = g32.solve(b, rtol=1e-8, out=x32)
        return i64, i32

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    recs = []
    t0 = time.perf_counter()
    for k in range(a.steps):
        recs.append(step())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"[bench] {a.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)
    vcycles = sum(r[0]["vcycles"] + r[1]["vcycles"] for r in recs)
    s64 = [r[0]["solve_ms"] for r in recs]
    s32 = [r[1]["solve_ms"] for r in recs]
    i64, i32 = recs[-1]
    diff = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))

    # standalone V-cycle throughput (100 back-to-back calls on a fixed r, FP64
    # and FP32 smoother, graph-replayed; and FP64 launched kernel by kernel
    # from a handle made with IBMG_GRAPH=0)
    def vc_rate(g, reps=100):
        r = torch.from_numpy(b_h).to(dev)
        z = torch.empty_like(r)
        g.vcycle(r, out=z)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            g.vcycle(r, out=z)
        torch.cuda.synchronize()
        return reps / (time.perf_counter() - t)

    vc64, vc32 = vc_rate(g64), vc_rate(g32)
    prev = os.environ.get("IBMG_GRAPH")
    os.environ["IBMG_GRAPH"] = "0"
    try:
        g64e = StokesIB(wl, precision="fp64")
    finally:
        if prev is None:
            del os.environ["IBMG_GRAPH"]
        else:
            os.environ["IBMG_GRAPH"] = prev
    vc64e = vc_rate(g64e)
    g64e.close()

    # roofline of the dominant kernel: the finest level's Schwarz boxes with
    # their own inverse (HBM streaming of the stored owned rows: the lower
    # owned tiles and every non-owned column, k_ras_ib_sym, with the launch
    # that adds its row and column sums), launched alone by the library with
    # HIP events on this stream; the other hot kernels for reference
    kt = g64.kernel_time("ras_ib", -1, a.roofline_reps)
    ras_ms, alg_bytes = kt["ms"], kt["bytes"]
    achieved = alg_bytes / (ras_ms * 1e-3) / 1e9
    traffic = measured_traffic(alg_bytes)
    kernels = {}
    for g, tag, peak in ((g64, "double", FP64_MFMA_PEAK_TFS), (g32, "float", FP32_MFMA_PEAK_TFS)):
        ib = g.kernel_time("ras_ib", -1, a.roofline_reps)
        it = g.kernel_time("ras_interior", -1, a.roofline_reps)
        sc = g.kernel_time("stencil", -1, a.roofline_reps)
        # the finest level's IB boxes run in symmetric storage on both handles
        kernels[f"k_ras_ib_sym<{tag}> + k_ras_sum"] = {"bound": "hbm", "avg_ms": ib["ms"], "alg_bytes": ib["bytes"],
                                                       "gbs": ib["bytes"] / ib["ms"] / 1e6,
                                                       "frac": ib["bytes"] / ib["ms"] / 1e6 / HBM_PEAK_GBS}
        kernels[f"k_ras_interior<{tag}>"] = {"bound": "mfma", "avg_ms": it["ms"], "alg_flops": it["flops"],
                                             "tflops": it["flops"] / it["ms"] / 1e9,
                                             "frac": it["flops"] / it["ms"] / 1e9 / peak}
        kernels[f"k_apply<{tag}>"] = {"bound": "hbm", "avg_ms": sc["ms"], "alg_bytes": sc["bytes"],
                                      "gbs": sc["bytes"] / sc["ms"] / 1e6,
                                      "frac": sc["bytes"] / sc["ms"] / 1e6 / HBM_PEAK_GBS}
        # grid transfers on the finest level; spreading and interpolation (FP64
        # on both handles, so timed once)
        names = [("restrict", f"k_restrict<{tag}>"), ("prolong", f"k_prolong_add<{tag}>")]
        if tag == "double":
            names += [("spread", "k_spread"), ("interp", "k_interp_lanes<double>")]
        for kind, name in names:
            t = g.kernel_time(kind, -1, a.roofline_reps)
            kernels[name] = {"bound": "hbm", "avg_ms": t["ms"], "alg_bytes": t["bytes"],
                             "gbs": t["bytes"] / t["ms"] / 1e6, "frac": t["bytes"] / t["ms"] / 1e6 / HBM_PEAK_GBS}
        # the smoothing step's Krylov kernels on the finest level (basis of
        # nu = 2 vectors); at 512^2 their vectors fit the Infinity Cache, so
        # the rates are against HBM peak but the data may come from cache
        for kind, name in (("apply_dots", f"k_apply_dots<{tag}>"), ("upd_dots", f"k_upd_dots<{tag}>"),
                           ("scale_upd", f"k_scale_upd<{tag}>"), ("combine_ls", f"k_combine_ls<{tag}>")):
            t = g.kernel_time(kind, -1, a.roofline_reps)
            kernels[name] = {"bound": "hbm", "avg_ms": t["ms"], "alg_bytes": t["bytes"],
                             "gbs": t["bytes"] / t["ms"] / 1e6, "frac": t["bytes"] / t["ms"] / 1e6 / HBM_PEAK_GBS}

    out = {
        "metric": METRIC,
        "value": vcycles / elapsed,
        "unit": "V-cycles/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * elapsed / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 + f32-smoother",
        "data": "synthetic",
        "config": {"workload": f"annulus_{wl.N}: {wl.N}x{wl.N} periodic, rho=1 mu=1e-2 dt=5e-4, "
                               f"4x2048-point annulus r=0.2..0.25, kappa=1e4, 7-level V-cycle, "
                               f"RAS {wl.box}x{wl.box}/{wl.overlap}, nu=2+2, FGMRES(30) to 1e-8",
                   "N": wl.N, "points": wl.M, "springs": int(len(wl.springs)),
                   "box": wl.box, "overlap": wl.overlap},
        "solve_ms_fp64": float(np.median(s64)),
        "solve_ms_fp32": float(np.median(s32)),
        "fp32_speedup": float(np.median(s64) / np.median(s32)),
        "iters_fp64": i64["iters"], "iters_fp32": i32["iters"],
        "rel_res_true_fp64": i64["rel_res_true"], "rel_res_true_fp32": i32["rel_res_true"],
        "fp32_vs_fp64_rel_diff": diff,
        "vcycles_per_s_fp64": vc64, "vcycles_per_s_fp32": vc32, "vcycles_per_s_fp64_no_graph": vc64e,
        "setup_s_fp64": t_setup64, "setup_s_fp32": t_setup32,
        "roofline": {"bound": "hbm", "kernel": "k_ras_ib_sym<double> + k_ras_sum (finest level IB boxes, "
                                               "symmetric storage of their owned rows)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launch_ms": ras_ms, "alg_bytes_per_launch": alg_bytes},
        "kernels": kernels,
    }
    # each solve's true residual under the oracle's operator (the whole
    # oracle does not set up at this size in bench time; the same structure
    # at 128^2 is compared with the oracle's solutions below)
    L_or, proj = oracle_operator(wl)
    out["oracle_rel_res_true_fp64"] = true_residual(L_or, proj, b_h, x64.cpu().numpy())
    out["oracle_rel_res_true_fp32"] = true_residual(L_or, proj, b_h, x32.cpu().numpy())
    del L_or
    if a.configs == "on":
        for key, fn in (("c3_structure_128_vs_oracle", c3_oracle_128), ("c1_plain_32", c1_bench),
                        ("c2_smoothers_256", c2_bench), ("c5_gradient_256", c5_bench)):
            t0 = time.perf_counter()
            out[key] = fn(dev)
            print(f"[bench] {key} {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.rms == "on":
        t0 = time.perf_counter()
        out["smoothers_fp64"] = [smoother_bench(wl, b, "rms", a.box, a.overlap),
                                 smoother_bench(wl, b, "ras", 8, 2), smoother_bench(wl, b, "rms", 8, 2)]
        print(f"[bench] smoother comparison {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.step == "on":
        t0 = time.perf_counter()
        out["time_step_fp64"] = step_bench(wl, b)
        print(f"[bench] time step {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.tangent == "on":
        t0 = time.perf_counter()
        out["tangent_fp64_fp32"] = tangent_bench(wl, b)
        print(f"[bench] tangent springs {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.large == "on":
        t0 = time.perf_counter()
        out["kernels_large_grid"] = large_bench()
        print(f"[bench] large-grid kernels {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.batch == "on":
        t0 = time.perf_counter()
        out["batch"] = batch_bench(dev)
        print(f"[bench] batch form {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    if a.cpu_baseline != "off":
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_boxes)
        print(f"[bench] cpu baseline {time.perf_counter() - t0:.1f}s", file=sys.stderr, flush=True)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
