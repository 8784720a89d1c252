"""Parameter studies of the results section (Sec. 5.1, 5.2) on the GPU path.

Each case is the linear solve of one semi-implicit time step without
convection: the paper's thick shell or thin membrane at resolution N,
stiffness ratio gamma and a flow condition (Stokes, or rho = 1 with mu = 1,
0.1, 0.01, 0.001), dt = 0.32 h, from the fluid state u^n of
``workloads.background_flow`` and the structure in its initial configuration.
The step's right-hand side [(rho/dt) u^n + S_h K_h X^n; 0] is formed by the
library and solved by FGMRES preconditioned by the V-cycle from a zero guess,
until the residual falls by ``rtol`` (1e-12 in the paper) or ``max_it`` (100)
iterations have run, with nu FGMRES smoothing sweeps before and after each
coarse correction (the paper does not state nu).  One record per case: iterations, whether the tolerance
was reached, the iterations needed for a 1e-6 reduction, the true final
relative residual and the setup and solve times.

Studies (the paper's figures they follow):
  shell_boxes      thick, N=128, gamma=500: box {4,8,16} x overlap {0,2,4},
                   RMS and RAS, Stokes and mu in {1, 0.1, 0.01}
                   (Figs. 5.1.1-1, 5.1.1-2)
  shell_refine     thick, N in sizes, gamma in {5, 50, 500}, Stokes and
                   mu in {1, 0.1, 0.01}, boxes 8/2 and 16/4, RMS and RAS
                   (Figs. 5.1.1-3, 5.1.1-4)
  shell_sc         thick, Schur-complement smoother, Stokes and
                   mu in {1, 0.1, 0.01, 0.001} (Fig. 5.1.2-1)
  membrane_boxes   thin, as shell_boxes (Figs. 5.2.1-1, 5.2.1-2)
  membrane_refine  thin, boxes 16/4, mu in {1, 0.1, 0.01} (Fig. 5.2.1-3)
  membrane_sc      thin, Schur-complement smoother (Fig. 5.2.2-1)

Usage:
  python -m paper_1612_02208_amd.sweep --study shell_boxes --out runs.jsonl
  python -m paper_1612_02208_amd.sweep --summary runs.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import workloads as W

GAMMAS = (5.0, 50.0, 500.0)
BOXES = (4, 8, 16)
OVERLAPS = (0, 2, 4)
SCHWARZ_FLOWS = ("stokes", "mu1", "mu0.1", "mu0.01")
SC_FLOWS = ("stokes", "mu1", "mu0.1", "mu0.01", "mu0.001")


def study_cases(study: str, sizes=(64, 128, 256, 512)):
    """The list of (structure, N, gamma, flow, smoother, box, overlap) of a study."""
    out = []
    if study in ("shell_boxes", "membrane_boxes"):
        st = "thick" if study.startswith("shell") else "thin"
        for flow in SCHWARZ_FLOWS:
            for b in BOXES:
                for o in OVERLAPS:
                    for sm in ("rms", "ras"):
                        out.append((st, 128, 500.0, flow, sm, b, o))
    elif study == "shell_refine":
        for b, o in ((8, 2), (16, 4)):
            for sm in ("rms", "ras"):
                for flow in SCHWARZ_FLOWS:
                    for g in GAMMAS:
                        for N in sizes:
                            out.append(("thick", N, g, flow, sm, b, o))
    elif study == "membrane_refine":
        for sm in ("rms", "ras"):
            for flow in ("mu1", "mu0.1", "mu0.01"):
                for g in GAMMAS:
                    for N in sizes:
                        out.append(("thin", N, g, flow, sm, 16, 4))
    elif study in ("shell_sc", "membrane_sc"):
        st = "thick" if study.startswith("shell") else "thin"
        for flow in SC_FLOWS:
            for g in GAMMAS:
                for N in sizes:
                    out.append((st, N, g, flow, "sc", 8, 2))
    else:
        raise ValueError(f"unknown study {study!r}")
    return out


STUDIES = ("shell_boxes", "shell_refine", "shell_sc", "membrane_boxes", "membrane_refine", "membrane_sc")


def iters_to(history, level):
    """First iteration whose relative residual estimate is <= level (None if never)."""
    for k, v in enumerate(history):
        if v <= level:
            return k + 1
    return None


def run_case(case, rtol=1e-12, max_it=100, restart=30, nu=2):
    """Solve one case on the GPU path (nu pre- and post-smoothing sweeps)
    and return its record."""
    import torch
    from .solver import IbmgError, StokesIB
    st, N, g, flow, sm, b, o = case
    wl = W.paper_case(st, N, g, flow, sm, b, o, nu1=nu, nu2=nu)
    rec = dict(structure=st, N=N, gamma=g, flow=flow, smoother=sm, box=b, overlap=o, nu=nu, name=wl.name,
               M=wl.M, dt=wl.dt, kappa=float(wl.kappa[0]))
    t0 = time.perf_counter()
    try:
        G = StokesIB(wl)
    except IbmgError as e:
        rec.update(status="setup_error", error=str(e))
        return rec
    torch.cuda.synchronize()
    rec["setup_ms"] = 1e3 * (time.perf_counter() - t0)
    try:
        u = torch.from_numpy(W.background_flow(N)).cuda()
        rhs = G.step_rhs(u)
        _, info = G.solve(rhs, rtol=rtol, restart=restart, max_it=max_it, history=max_it + 1)
        h = info["history"]
        rec.update(status=info["status"], converged=info["converged"], iters=info["iters"],
                   it_1e6=iters_to(h, 1e-6), rel_res_true=info["rel_res_true"],
                   rel_res_est=info["rel_res_est"], solve_ms=info["solve_ms"],
                   reduction_per_it=(h[-1] ** (1.0 / len(h)) if h and h[-1] > 0 else None),
                   levels=G.n_levels)
    except IbmgError as e:
        rec.update(status="solve_error", error=str(e))
    finally:
        G.close()
    return rec


def _fmt_it(r):
    if r.get("status") not in ("OK", "NOT_CONVERGED"):
        return "err"
    return f"{r['iters']}" if r["converged"] else f"{r['iters']}*"


def _cell(r, metric):
    if r is None:
        return ""
    if metric == "ms":
        return "err" if "solve_ms" not in r else f"{r['solve_ms']:.1f}" + ("" if r.get("converged") else "*")
    return f"{_fmt_it(r)} ({r.get('it_1e6')})"


def summary(records, metric="iters") -> str:
    """Markdown tables of a study's records: iterations to rtol ('*' = not
    reached within max_it), with iterations to 1e-6 in parentheses, or
    (metric "ms") the solve's wall-clock milliseconds."""
    what = "solve ms" if metric == "ms" else "iterations (iterations to 1e-6)"
    lines = []
    by = {}
    for r in records:
        key = (r["structure"], r["smoother"], r["box"] if r["smoother"] != "sc" else None,
               r["overlap"] if r["smoother"] != "sc" else None)
        by.setdefault(key, []).append(r)
    boxes_mode = len({r["N"] for r in records}) == 1 and len({(r["box"], r["overlap"]) for r in records}) > 1
    if boxes_mode:
        # rows: flow x box; columns: overlap, per smoother
        flows = list(dict.fromkeys(r["flow"] for r in records))
        sms = list(dict.fromkeys(r["smoother"] for r in records))
        st = records[0]["structure"]
        lines.append(f"{st}, N={records[0]['N']}, gamma={records[0]['gamma']:g}: {what}")
        lines.append("")
        hdr = "| flow | box | " + " | ".join(f"{sm.upper()} o={o}" for sm in sms for o in OVERLAPS) + " |"
        lines.append(hdr)
        lines.append("|" + "---|" * (2 + len(sms) * len(OVERLAPS)))
        idx = {(r["flow"], r["smoother"], r["box"], r["overlap"]): r for r in records}
        for f in flows:
            for b in BOXES:
                cells = []
                for sm in sms:
                    for o in OVERLAPS:
                        r = idx.get((f, sm, b, o))
                        cells.append(_cell(r, metric))
                lines.append(f"| {f} | {b} | " + " | ".join(cells) + " |")
        return "\n".join(lines)
    for key, rs in by.items():
        st, sm, b, o = key
        head = f"{st}, {sm.upper()}" + (f" {b}x{b} boxes, overlap {o}" if b is not None else "")
        lines.append(head + ": " + what)
        lines.append("")
        Ns = sorted({r["N"] for r in rs})
        lines.append("| flow | gamma | " + " | ".join(f"N={N}" for N in Ns) + " |")
        lines.append("|" + "---|" * (2 + len(Ns)))
        idx = {(r["flow"], r["gamma"], r["N"]): r for r in rs}
        for f in dict.fromkeys(r["flow"] for r in rs):
            for g in sorted({r["gamma"] for r in rs}):
                cells = []
                for N in Ns:
                    r = idx.get((f, g, N))
                    cells.append(_cell(r, metric))
                lines.append(f"| {f} | {g:g} | " + " | ".join(cells) + " |")
        lines.append("")
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--study", action="append", choices=STUDIES)
    ap.add_argument("--sizes", default="64,128,256,512")
    ap.add_argument("--rtol", type=float, default=1e-12)
    ap.add_argument("--max-it", type=int, default=100)
    ap.add_argument("--nu", type=int, default=2, help="pre- and post-smoothing sweeps per level")
    ap.add_argument("--out", default=None, help="append one JSON record per case to this file")
    ap.add_argument("--summary", default=None, help="print markdown tables of a records file")
    ap.add_argument("--metric", choices=("iters", "ms"), default="iters", help="what --summary tabulates")
    a = ap.parse_args(argv)
    if a.summary:
        recs = [json.loads(l) for l in open(a.summary) if l.strip()]
        if a.study:
            recs = [r for r in recs if r["study"] in a.study]
        for s in dict.fromkeys(r["study"] for r in recs):
            for nu in sorted({r.get("nu", 2) for r in recs if r["study"] == s}):
                print(f"### {s}, nu = {nu}\n")
                print(summary([r for r in recs if r["study"] == s and r.get("nu", 2) == nu], a.metric))
                print()
        return 0
    if not a.study:
        ap.error("--study or --summary is required")
    sizes = tuple(int(s) for s in a.sizes.split(","))
    fh = open(a.out, "a") if a.out else None
    for study in a.study:
        cases = study_cases(study, sizes)
        t0 = time.perf_counter()
        for i, c in enumerate(cases):
            rec = run_case(c, a.rtol, a.max_it, nu=a.nu)
            rec["study"] = study
            print(f"[{study} nu={a.nu} {i + 1}/{len(cases)}] {rec['name']}: {rec.get('status')} "
                  f"iters={rec.get('iters')} 1e-6@{rec.get('it_1e6')} "
                  f"res={rec.get('rel_res_true', float('nan')):.2e} "
                  f"setup={rec.get('setup_ms', 0):.0f}ms solve={rec.get('solve_ms', 0):.1f}ms",
                  flush=True)
            if fh:
                fh.write(json.dumps(rec) + "\n")
                fh.flush()
        print(f"[{study}] {len(cases)} cases in {time.perf_counter() - t0:.1f} s", flush=True)
    if fh:
        fh.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
