"""Single-kernel timings of the N = 512 annulus workload, and one plain copy
of known size, for profilers (HIP-event averages, algorithmic bytes and the
resulting rates; run it under ``rocprofv3 --pmc`` to read hardware counters
per dispatch, the copy calibrating the counters' units):

    python -m paper_1612_02208_amd.profile_kernels [--N 512] [--box 16]
        [--overlap 4] [--precision fp64] [--reps 5] [--copy-mib 1024]

With ``--solve membrane256`` it instead runs whole FGMRES solves to 1e-8 (a
warm-up, then ``--reps`` timed) of the 256^2 Stokes membrane (1024 points,
``--kappa``, ``--smoother ras|sc``), so that a kernel trace attributes a
solve's time to its kernels.

With ``--step`` it runs ``--reps`` semi-implicit time steps of the annulus
and prints each step's solve and rebuild times, the rebuild's phases going
to stderr (IBMG_SETUP_TIMES).

With ``--interior-forms`` it times the interior product in each of its
forms at the finest level: 1 = pipelined 64-box tiles in XCD order, 16 and
32 boxes per narrow tile, 64 = register-blocked tiles, 128 = gathered
operand.

With ``--large`` it times the grid and coupling kernels on a 4096^2 grid
with 2^20 points instead (fields of 400 MB, beyond the caches): a
suspension of 32 x 32 membranes in fibre order for the stencil, the
transfers, spreading and interpolation, then the same count of uniformly
scattered points for spreading and interpolation.

Prints one JSON line per kernel.
"""
import argparse
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--N", type=int, default=512)
    p.add_argument("--box", type=int, default=16)
    p.add_argument("--overlap", type=int, default=4)
    p.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    p.add_argument("--reps", type=int, default=5)
    p.add_argument("--copy-mib", type=int, default=1024)
    p.add_argument("--large", action="store_true")
    p.add_argument("--solve", default="", choices=["", "membrane256"])
    p.add_argument("--kappa", type=float, default=1e4)
    p.add_argument("--smoother", default="sc", choices=["ras", "sc", "rms"])
    p.add_argument("--interior-forms", action="store_true")
    p.add_argument("--step", action="store_true")
    a = p.parse_args()
    import numpy as np
    import torch
    import workloads as W
    from paper_1612_02208_amd import StokesIB

    if a.solve:
        wl = W.smoother_256(a.kappa, a.smoother)
        g = StokesIB(wl, precision=a.precision)
        b = torch.from_numpy(W.rhs(wl.N, 0)).cuda()
        x, info = g.solve(b, rtol=1e-8)
        st = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(a.reps):
            x, info = g.solve(b, rtol=1e-8)
        e1.record(st)
        torch.cuda.synchronize()
        print(json.dumps(dict(workload=wl.name, precision=a.precision, reps=a.reps, iters=info["iters"],
                              converged=info["converged"], solve_ms=e0.elapsed_time(e1) / a.reps,
                              vcycles=info["vcycles"])), flush=True)
        g.close()
        copy_calibration(a.copy_mib, a.reps)
        return

    if a.large:
        N, M = 4096, 1 << 20
        for tag, X in (("suspension", W.suspension_points(32, 0.35 / 32, 1024)),
                       ("uniform_random", W.random_points(M, 7))):
            wl = W.Workload(f"grid_{N}_{tag}", N, 8, 1.0, 1e-2, 5e-4, X, np.zeros((0, 2), dtype=np.int32),
                            np.zeros(0), box=8, overlap=2)
            g = StokesIB(wl, precision="fp64")
            kinds = [("spread", "k_spread"), ("interp", "k_interp_lanes<double>")]
            if tag == "suspension":
                kinds = [("stencil", "k_apply<double>"), ("restrict", "k_restrict<double>"),
                         ("prolong", "k_prolong_add<double>")] + kinds
            for kern, name in kinds:
                t = g.kernel_time(kern, -1, a.reps)
                print(json.dumps(dict(kernel=name, layout=tag, N=N, points=int(X.shape[0]), reps=a.reps,
                                      avg_ms=t["ms"], alg_bytes=t["bytes"], gbs=t["bytes"] / t["ms"] / 1e6)),
                      flush=True)
            g.close()
        copy_calibration(a.copy_mib, a.reps)
        return

    wl = W.annulus_512(N=a.N)
    wl.box, wl.overlap = a.box, a.overlap
    if a.step:
        # semi-implicit time steps of the annulus (FP64): the set-up's phase
        # times go to stderr for every rebuild (IBMG_SETUP_TIMES)
        import time
        os.environ["IBMG_SETUP_TIMES"] = "1"
        g = StokesIB(wl, precision=a.precision)
        w = torch.zeros(3 * a.N * a.N, dtype=torch.float64, device="cuda")
        for k in range(a.reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w, info = g.time_step(w, rtol=1e-8)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            print(json.dumps(dict(kind="time_step", step=k, step_ms=ms, solve_ms=info["solve_ms"],
                                  rebuild_ms=ms - info["solve_ms"], iters=info["iters"])), flush=True)
        g.close()
        del os.environ["IBMG_SETUP_TIMES"]
        return
    if a.interior_forms:
        # each tile form of the interior product, forced through the set-up
        # tuner's override, one handle per form
        for form in (1, 16, 32, 64, 128):
            os.environ["IBMG_INTERIOR_FORM"] = str(form)
            g = StokesIB(wl, precision=a.precision)
            t = g.kernel_time("ras_interior", -1, a.reps)
            print(json.dumps(dict(kernel="k_ras_interior", form=form, precision=a.precision, N=a.N, reps=a.reps,
                                  avg_ms=t["ms"], alg_flops=t["flops"], tflops=t["flops"] / t["ms"] / 1e9)),
                  flush=True)
            g.close()
        del os.environ["IBMG_INTERIOR_FORM"]
        return
    g = StokesIB(wl, precision=a.precision)
    suffix = "<double>" if a.precision == "fp64" else "<float>"
    kinds = [("ras_ib", "k_ras_ib"), ("ras_interior", "k_ras_interior"), ("stencil", "k_apply"),
             ("restrict", "k_restrict"), ("prolong", "k_prolong_add")]
    if a.precision == "fp64":
        kinds += [("spread", "k_spread"), ("interp", "k_interp_lanes")]
    for kern, name in kinds:
        t = g.kernel_time(kern, -1, a.reps)
        rec = dict(kernel=name + ("" if kern == "spread" else suffix), level=g.n_levels - 1, N=a.N, reps=a.reps, avg_ms=t["ms"],
                   alg_bytes=t["bytes"], alg_flops=t["flops"], gbs=t["bytes"] / t["ms"] / 1e6,
                   tflops=t["flops"] / t["ms"] / 1e9)
        print(json.dumps(rec), flush=True)
    g.close()
    copy_calibration(a.copy_mib, a.reps)


def copy_calibration(copy_mib, reps):
    """A plain device copy of known size (reads and writes copy_mib MiB once
    per repetition), which calibrates the units of the HBM byte counters."""
    import torch
    if copy_mib <= 0:
        return
    n = copy_mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(st)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    print(json.dumps(dict(kernel="copy", bytes_read=n * 8, bytes_written=n * 8, avg_ms=ms,
                          gbs=2 * n * 8 / ms / 1e6)), flush=True)


if __name__ == "__main__":
    main()
