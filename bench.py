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

Also reported: the roofline of the dominant kernel (k_ras_ib<double>, the
finest level's Schwarz boxes with their own inverse), timed alone with HIP
events on the stream it runs on; the other hot kernels; the batched form on
64 independent systems (N in {64, 128, 256}, FP32 smoother); and the FP64 CPU
oracle on a bounded sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--cpu-baseline sample|off]
                    [--batch on|off] [--rms on|off] [--step on|off]
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
    p.add_argument("--cpu-boxes", type=int, default=1024)
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
    return p.parse_args()


def measured_traffic(alg_bytes):
    """HBM bytes per launch of k_ras_ib<double> from the committed
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
    return {"step_ms": total, "solve_ms": info["solve_ms"], "rebuild_ms": total - info["solve_ms"],
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
            out["time_step"] = {"step_ms": tot, "solve_ms": si["solve_ms"], "rebuild_ms": tot - si["solve_ms"],
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


def cpu_baseline(wl, nboxes):
    """Time the plain FP64 oracle on a bounded sample of the same workload and
    scale it to V-cycles/s: the box solves of the finest level (gather,
    LU solve, owned-set scatter) on ``nboxes`` of its boxes, and one
    L_IB apply per level; a V-cycle performs (nu1 + nu2) box solves per box of
    every level >= 1 and six operator applies per level."""
    import scipy.linalg as la
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import hierarchy, schwarz

    levels = hierarchy.build(wl)
    fine = levels[-1]
    parts = schwarz.patches(fine.N, wl.box, wl.overlap)
    step = max(1, len(parts) // nboxes)
    sample = parts[::step][:nboxes]
    Lc = fine.L.tocsr()
    facs = [la.lu_factor(Lc[p.idx][:, p.idx].toarray()) for p in sample]
    box_solves = (wl.nu1 + wl.nu2) * sum(len(schwarz.patches(l.N, wl.box, wl.overlap)) for l in levels[1:])

    def timed():
        rng = np.random.default_rng(0)
        r = rng.uniform(-1, 1, fine.n)
        z = np.zeros_like(r)
        t0 = time.perf_counter()
        for p, f in zip(sample, facs):
            y = la.lu_solve(f, r[p.idx])
            z[p.own_global] = y[p.own_local]
        t_box = (time.perf_counter() - t0) / len(sample)
        t_ops = 0.0
        for lev in levels:
            w = rng.uniform(-1, 1, lev.n)
            t0 = time.perf_counter()
            for _ in range(3):
                lev.L @ w
            t_ops += 6 * (time.perf_counter() - t0) / 3
        return t_box, t_ops, box_solves * t_box + t_ops

    threads = max([d.get("num_threads", 1) for d in threadpool_info() if d.get("user_api") == "blas"] or [1])
    t_box, t_ops, t_vc = timed()
    with threadpool_limits(limits=1, user_api="blas"):
        _, _, t_vc1 = timed()
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / t_vc, "unit": "V-cycles/s", "cores": threads, "kind": "oracle",
            "sample": (f"FP64 oracle on the N={wl.N} annulus: {len(sample)} of {len(parts)} finest boxes "
                       f"(LU solve + scatter, {t_box * 1e3:.3f} ms/box) scaled to the {box_solves} box "
                       f"solves of one V-cycle, plus 6 sparse L_IB applies per level "
                       f"({t_ops * 1e3:.1f} ms); factorisation and set-up excluded; cores = BLAS threads"),
            "vcycle_s": t_vc, "cpu_model": model, "host_cpus": os.cpu_count(),
            "single_thread": {"value": 1.0 / t_vc1, "vcycle_s": t_vc1}}


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

    # roofline of the dominant kernel: k_ras_ib<double>, the finest level's
    # Schwarz boxes with their own inverse (HBM streaming of the owned
    # inverse rows), launched alone by the library with HIP events on this
    # stream; the other hot kernels for reference
    kt = g64.kernel_time("ras_ib", -1, a.roofline_reps)
    ras_ms, alg_bytes = kt["ms"], kt["bytes"]
    achieved = alg_bytes / (ras_ms * 1e-3) / 1e9
    traffic = measured_traffic(alg_bytes)
    kernels = {}
    for g, tag, peak in ((g64, "double", FP64_MFMA_PEAK_TFS), (g32, "float", FP32_MFMA_PEAK_TFS)):
        ib = g.kernel_time("ras_ib", -1, a.roofline_reps)
        it = g.kernel_time("ras_interior", -1, a.roofline_reps)
        sc = g.kernel_time("stencil", -1, a.roofline_reps)
        kernels[f"k_ras_ib<{tag}>"] = {"bound": "hbm", "avg_ms": ib["ms"], "alg_bytes": ib["bytes"],
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
        "roofline": {"bound": "hbm", "kernel": "k_ras_ib<double> (finest level)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "launch_ms": ras_ms, "alg_bytes_per_launch": alg_bytes},
        "kernels": kernels,
    }
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
