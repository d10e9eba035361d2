#!/usr/bin/env python3
"""Throughput of the CC-MSAV vesicle time step on one MI355X.

One "step" is one full CC-MSAV-BDF2 time step (stencil terms, SAV inner
products, 5x5 solve, DCT elliptic solves) of the named synthetic workload; the
inputs are resident in device memory before the timed region starts. By
default the mixed-precision path (FP32 transforms, FP64 state and scalars) is
timed on the N = 4096 vesicle, and the FP64 path is then run for the same
number of steps to report its throughput and the mixed path's error against
it. Prints one JSON line: the throughput in Mcell-steps/s, a roofline entry
for the dominant kernel (algorithmic bytes per launch over its mean duration
from HIP events on the library's stream), and the FP64 CPU oracle timed on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mcell-steps/s at N=2048/4096, mixed-prec & batched vs FP64, rel err ≤1e-6"
HBM_PEAK_GBS = 8000.0

# Algorithmic HBM bytes per cell for one launch of each kernel of the step.
# State fields are FP64; the eight stencil fields, the eight x-transformed
# intermediates and the two solved fields are FP64 (fp64) or FP32 (mixed).
# The stencil pass reads phi, psi at levels n, n-1 (and n-2 for the lagged
# ||d||^2) and writes eight fields; the row DCT reads and writes eight; the
# column pass reads eight; the column solve reads seven and writes two; the
# row inverse reads two and writes the two new state fields. The mixed path
# solves for increments, so its row inverse also reads phi^n, psi^n.
def gemm_flops(members):
    """Matrix-core flops per launch of each phase of the DCT-as-GEMM variant:
    three bf16 products (hi hi, hi lo, lo hi) of 2 m n k flops each, for the
    row products of 8 (forward) and 2 (inverse) fields against the nx x nx DCT
    matrix and the column products against the ny x ny one."""
    f = {"row_dct": 0.0, "col_gram": 0.0, "col_solve": 0.0, "row_idct": 0.0}
    for mb in members:
        nx, ny = mb.params["nx"], mb.params["ny"]
        f["row_dct"] += 3 * 2.0 * (8 * ny) * nx * nx
        f["col_gram"] += 3 * 2.0 * 8 * nx * ny * ny
        f["col_solve"] += 3 * 2.0 * 2 * nx * ny * ny
        f["row_idct"] += 3 * 2.0 * (2 * ny) * nx * nx
    return f


BF16_PEAK_TFLOPS = 2500.0


def kernel_bytes_per_cell(precision: str, scheme: str = "bdf2"):
    m = 8 if precision == "fp64" else 4
    # The BDF1 scheme's stencil pass reads level n only (phi*, psi* = phi^n, psi^n).
    levels = 3 if scheme == "bdf2" else 1
    return {
        "stencil": 2 * levels * 8 + 8 * m,
        "row_dct": 16 * m,
        "col_gram": 8 * m,
        "solve5": 0,
        "col_solve": 7 * m + 2 * m,
        "row_idct": 2 * m + 2 * 8 + (2 * 8 if precision != "fp64" else 0),
    }


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def source_digest() -> str:
    """Hash of the code of the HIP sources, to tell whether stored counters are
    stale. Comments and whitespace are left out: they compile to nothing."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_10057_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if not name.endswith((".hip", ".hpp")):
            continue
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            code = " ".join(_COMMENT.sub(" ", f.read()).split())
        h.update(name.encode())
        h.update(code.encode())
    return h.hexdigest()[:16]


def stored_traffic(workload: str, precision: str, kernel: str, cells: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_digest():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(members, budget_s: float = 12.0):
    """FP64 oracle timed on this host over a bounded sample of the workload:
    the first two steps (one BDF1, one BDF2) of as many members as fit in
    about ``budget_s`` seconds (at least one)."""
    from oracle import ccmsav_ref as R
    cells = 0
    taken = 0
    used = 0.0
    for m in members:
        st = R.initial_state(m.phi0, m.psi0, m.params)
        t0 = time.perf_counter()
        R.step(st)
        R.step(st)
        used += time.perf_counter() - t0
        cells += m.phi0.size * 2
        taken += 1
        if used > budget_s:
            break
    sizes = sorted({m.params["nx"] for m in members[:taken]})
    return {"value": cells / used / 1e6, "unit": "Mcell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"the first 2 steps (one BDF1, one BDF2) of {taken} of {len(members)} "
                      f"member(s) (N={sizes}): {used:.2f} s, single-threaded numpy/scipy"}


def timed_run(C, torch, members, precision, steps, warmup, profile_steps, dev, graph,
              bdf1=False):
    """Warm up, time ``steps`` steps between two synchronisations, then take
    ``profile_steps`` more with per-kernel events. Returns timings and the
    final states (after warmup + steps + profile_steps steps)."""
    phi0 = [torch.from_numpy(m.phi0).to(dev) for m in members]
    psi0 = [torch.from_numpy(m.psi0).to(dev) for m in members]
    stream = torch.cuda.current_stream(dev)
    ctx = C.Context.ensemble([m.params for m in members], phi0, psi0, precision,
                             stream=stream.cuda_stream, graph=graph, bdf1=bdf1)
    nm = len(members)
    mass0 = [ctx.mass(i)[0] for i in range(nm)]
    ctx.step(warmup)
    ctx.sync()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.sync()                       # raises on any device-side error of the run
    prof = ctx.profile_steps(profile_steps) if profile_steps > 0 else {}
    tuning = ctx.tuning()
    mass = [ctx.mass(i)[0] for i in range(nm)]
    out = dict(wall=wall, ev_ms=ev0.elapsed_time(ev1), prof=prof, tuning=tuning,
               drift=max(abs(a - b) / abs(b) for a, b in zip(mass, mass0)),
               energy=[None if bdf1 else ctx.energy(member=i) for i in range(nm)],
               fields=[ctx.fields(i) for i in range(nm)],
               savs=[ctx.savs(i)[0] for i in range(nm)])
    ctx.close()
    return out


# HBM bytes per cell of one relaxation step with FP64 transforms: right-hand
# side (read phi, write rhs), row DCT (read rhs, write one field), column solve
# (read one, write two), row inverse (read two, write two FP64 fields).
SMOOTH_BYTES_PER_CELL_FP64 = 16 + 16 + 24 + 32


def smooth_bench(C, torch, np, member, args, dev):
    """Time ccmsav_smooth_ic (App. F: M = 0.01, dt = 1e-6, ten steps per call)."""
    nsub = 10
    sharp = torch.from_numpy(np.where(member.phi0 > 0.0, 1.0, -1.0)).to(dev)
    out = torch.empty_like(sharp)
    ctx = C.Context(member.params, member.phi0, member.psi0, args.precision)
    lib = C.load()
    call = lambda: C._check(lib.ccmsav_smooth_ic(ctx._h, 0.01, 1e-6, nsub, sharp.data_ptr(),  # noqa: E731
                                                 out.data_ptr()), "ccmsav_smooth_ic")
    for _ in range(max(1, args.warmup)):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        call()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    cells = member.phi0.size
    value = cells * nsub * args.steps / wall / 1e6
    ms_call = 1e3 * wall / args.steps
    frac = None
    if args.precision == "fp64":
        frac = SMOOTH_BYTES_PER_CELL_FP64 * value * 1e6 / 1e9 / HBM_PEAK_GBS
    print(json.dumps({"metric": "App. F smoothing, Mcell-steps/s", "value": value,
                      "unit": "Mcell-steps/s", "n_gpus": 1, "calls": args.steps,
                      "steps_per_call": nsub, "ms_per_call": ms_call,
                      "higher_is_better": True, "dtype": {"fp64": "f64", "mixed": "f32+f64"}.get(
                          args.precision, args.precision),
                      "data": "synthetic", "config": {"workload": args.workload,
                                                      "nx": member.params["nx"],
                                                      "ny": member.params["ny"],
                                                      "precision": args.precision},
                      "hbm_frac_of_step_model": frac}), flush=True)


def elliptic_bench(C, torch, np, member, args, dev):
    """Time ccmsav_elliptic_solve_bc (both outputs) on the workload's grid."""
    ny, nx = member.phi0.shape
    rhs = torch.from_numpy(np.random.default_rng(1).standard_normal((ny, nx))).to(dev)
    oc, oz = torch.empty_like(rhs), torch.empty_like(rhs)
    ctx = C.Context(member.params, member.phi0, member.psi0, args.precision)
    for _ in range(max(1, args.warmup)):
        ctx.elliptic_solve(rhs, oc, oz, bc=args.elliptic)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.elliptic_solve(rhs, oc, oz, bc=args.elliptic)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    value = nx * ny * args.steps / wall / 1e6
    print(json.dumps({"metric": "fast direct solve (chi and zeta), Mcell-solves/s", "value": value,
                      "unit": "Mcell-solves/s", "n_gpus": 1, "calls": args.steps,
                      "ms_per_call": 1e3 * wall / args.steps, "higher_is_better": True,
                      "dtype": "f64" if args.elliptic == "periodic" or args.precision == "fp64"
                      else "f32+f64", "data": "synthetic",
                      "config": {"workload": args.workload, "nx": nx, "ny": ny,
                                 "boundaries": args.elliptic, "precision": args.precision}}),
          flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="vesicle4096")
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed", "gemm"])
    ap.add_argument("--graph", action="store_true",
                    help="replay the steady-state steps from a captured HIP graph")
    ap.add_argument("--profile-steps", type=int, default=50,
                    help="steps of the per-kernel event pass that feeds the roofline")
    ap.add_argument("--scheme", default="bdf2", choices=["bdf2", "bdf1"],
                    help="time-stepping scheme: CC-MSAV-BDF2 (the default), or the "
                         "first-order CC-MSAV-BDF1 scheme at every step")
    ap.add_argument("--smooth-ic", action="store_true",
                    help="instead of the step, time the App. F initial-condition relaxation "
                         "(ccmsav_smooth_ic, ten steps per call) on the workload's first grid")
    ap.add_argument("--elliptic", choices=["neumann", "dirichlet", "periodic"], default=None,
                    help="instead of the step, time the standalone fast direct solver "
                         "(chi^{-1} and zeta^{-1} of one field) with these boundaries")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64 run that the mixed path is checked and compared against")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="after timing, copy this many MiB with a plain torch copy "
                         "(a known-size kernel that calibrates rocprofv3 byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the single-grid step is run on one MI355X).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2601_10057_amd import ccmsav as C
    from workloads import make_workload

    members = make_workload(args.workload)
    cells = sum(m.phi0.size for m in members)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.smooth_ic:
        smooth_bench(C, torch, np, members[0], args, dev)
        return
    if args.elliptic:
        elliptic_bench(C, torch, np, members[0], args, dev)
        return

    bdf1 = args.scheme == "bdf1"
    run = timed_run(C, torch, members, args.precision, args.steps, args.warmup,
                    args.profile_steps, dev, args.graph, bdf1)
    wall = run["wall"]
    ms_per_step = 1e3 * wall / args.steps
    value = cells * args.steps / wall / 1e6
    print(f"[bench] {args.workload} {args.precision}: {ms_per_step:.4f} ms/step (wall), "
          f"{run['ev_ms'] / args.steps:.4f} ms/step (events), {value:.1f} Mcell-steps/s",
          file=sys.stderr, flush=True)

    prof = run["prof"]
    per_cell = kernel_bytes_per_cell(args.precision, args.scheme)
    for k, ms in prof.items():
        gbs = per_cell[k] * cells / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        print(f"[bench] kernel {k}: {ms * 1e3:.1f} us/launch, {per_cell[k]} B/cell, "
              f"{gbs:.0f} GB/s", file=sys.stderr, flush=True)
    roofline = None
    if prof and args.precision == "gemm":
        fl = gemm_flops(members)
        for k, v in fl.items():
            print(f"[bench] phase {k}: {prof[k] * 1e3:.1f} us, "
                  f"{v / (prof[k] * 1e-3) / 1e12:.1f} TFLOP/s (bf16 matrix cores, incl. splits)",
                  file=sys.stderr, flush=True)
        dom = max(fl, key=lambda k: prof[k])
        achieved = fl[dom] / (prof[dom] * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": dom, "achieved": achieved,
                    "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS,
                    "traffic": None, "flops_per_launch": fl[dom], "us_per_launch": prof[dom] * 1e3,
                    "step_flops": sum(fl.values()),
                    "step_frac": sum(fl.values()) / (ms_per_step * 1e-3) / 1e12 / BF16_PEAK_TFLOPS}
    elif prof:
        dom = max(prof, key=prof.get)
        dom_bytes = per_cell[dom] * cells
        achieved = dom_bytes / (prof[dom] * 1e-3) / 1e9
        traffic = stored_traffic(args.workload, args.precision, dom, cells)
        roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "bytes_per_launch": dom_bytes, "us_per_launch": prof[dom] * 1e3,
                    "step_bytes_per_cell": sum(per_cell.values()),
                    "step_frac": sum(per_cell.values()) * value * 1e6 / 1e9 / HBM_PEAK_GBS}

    finite = all(bool(np.all(np.isfinite(f[0]))) for f in run["fields"])
    if not bdf1:
        finite = finite and bool(np.all(np.isfinite(run["energy"])))
    check = {"mass_drift": run["drift"], "E_mod": run["energy"][0], "finite": finite}
    compare = None
    if args.precision != "fp64" and not args.no_compare:
        ref = timed_run(C, torch, members, "fp64", args.steps, args.warmup, args.profile_steps,
                        dev, args.graph, bdf1)
        rel = lambda a, b: float(np.abs(a - b).max() / np.abs(b).max())  # noqa: E731
        check.update(
            rel_linf_phi_vs_fp64=max(rel(a[0], b[0]) for a, b in zip(run["fields"], ref["fields"])),
            rel_linf_psi_vs_fp64=max(rel(a[1], b[1]) for a, b in zip(run["fields"], ref["fields"])),
            rel_sav_vs_fp64=max(rel(a, b) for a, b in zip(run["savs"], ref["savs"])),
            steps_compared=args.warmup + args.steps + args.profile_steps)
        fp64_value = cells * args.steps / ref["wall"] / 1e6
        compare = {"fp64_value": fp64_value, "fp64_ms_per_step": 1e3 * ref["wall"] / args.steps,
                   "speedup_vs_fp64": value / fp64_value}
        print(f"[bench] fp64 path: {compare['fp64_ms_per_step']:.4f} ms/step, "
              f"{fp64_value:.1f} Mcell-steps/s; mixed/fp64 = {compare['speedup_vs_fp64']:.3f}; "
              f"rel err phi {check['rel_linf_phi_vs_fp64']:.2e}", file=sys.stderr, flush=True)

    if args.copy_probe_mib > 0:
        a = torch.empty(args.copy_probe_mib * 2 ** 18, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()

    cpu = None if args.no_cpu_baseline else cpu_baseline(members)
    m0 = members[0]
    config = {"workload": args.workload, "members": len(members), "cells": cells,
              "grids": sorted({(m.params["nx"], m.params["ny"]) for m in members}),
              "precision": args.precision, "graph": args.graph, "scheme": args.scheme,
              "dt": sorted({m.params["dt"] for m in members}),
              "eps_cells": sorted({m.meta.get("eps_cells", 4.0) for m in members})}
    if len(members) == 1:
        config.update(nx=m0.params["nx"], ny=m0.params["ny"])
    config["autotune"] = [dict(grid=[t["nx"], t["ny"]], **t["variants"]) for t in run["tuning"]]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Mcell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "gemm": "bf16x3+f32+f64"}[args.precision],
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "vs_fp64": compare,
        "check": check,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
