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
def fs_n1(n):
    """First factor N1 of the factored (four-step) transform of n points, 0 for
    the dense product with the n x n DCT matrix (the library's choice)."""
    return 64 if n >= 4096 else (32 if n == 2048 else 0)


def line_flops(n, inverse):
    """Matrix-core flops of one DCT of n points: six bf16 products of
    three-part operands, 2 m n k flops each. Dense: the n x n matrix, 12 n^2.
    Factored (n = N1 N2, real and imaginary parts stacked): forward 2 N1 x N1
    and N2 x 2 N2 matrices, 24 (N1 + N2) n; inverse 2 N1 x 2 N1 and N2 x 2 N2,
    48 N1 n + 24 N2 n."""
    n1 = fs_n1(n)
    if n1 == 0:
        return 6 * 2.0 * n * n
    n2 = n // n1
    return 6 * 2.0 * n * ((4 * n1 + 2 * n2) if inverse else (2 * n1 + 2 * n2))


def gemm_flops(members):
    """Matrix-core flops per launch of each phase of the DCT-as-GEMM variant:
    the row transforms of 8 (forward) and 2 (inverse) fields along x, the
    column transforms along y."""
    f = {"row_dct": 0.0, "col_gram": 0.0, "col_solve": 0.0, "row_idct": 0.0}
    for mb in members:
        nx, ny = mb.params["nx"], mb.params["ny"]
        f["row_dct"] += 8 * ny * line_flops(nx, False)
        f["col_gram"] += 8 * nx * line_flops(ny, False)
        f["col_solve"] += 2 * nx * line_flops(ny, True)
        f["row_idct"] += 2 * ny * line_flops(nx, True)
    return f


BF16_PEAK_TFLOPS = 2500.0


# Algorithmic bytes per cell of the step's four passes in the pipeline model
# of the measurement plan (FP64 state; FP64 or FP32 intermediates):
#   P1 stencil terms + row DCT-II, one pass: reads phi, psi at levels n and
#      n-1 (level n only in the BDF1 scheme), writes the 8 x-transformed fields;
#   P2 column DCT-II + Parseval sums: reads 8;
#   P3 combine, divide, column DCT-III: reads 7, writes 2;
#   P4 row DCT-III: reads 2 (+ phi^n, psi^n in the increment form), writes the
#      2 new state fields.
# FP64: 96 + 64 + 72 + 32 = 264 B; mixed: 64 + 32 + 36 + 40 = 172 B. This build
# runs P1 as two launches (k_stencil, then k_row_dct8) with the 8 stencil
# fields in HBM between them, and its stencil reads level n-2 as well for the
# lagged ||d||^2, and its FP32 intermediates come in pairs of fields, so that
# the column solve's Allen-Cahn group reads f_lin next to the unused P~:
# kernel_bytes_per_cell below counts those extra bytes (256 B mixed, 408 B
# FP64), this model does not.
PASSES = {"P1": ("stencil", "row_dct"), "P2": ("col_gram",), "P3": ("col_solve",),
          "P4": ("row_idct",)}


def pass_bytes_per_cell(precision: str, scheme: str = "bdf2"):
    m = 8 if precision == "fp64" else 4
    levels = 2 if scheme == "bdf2" else 1
    inc = precision != "fp64"
    return {"P1": 2 * levels * 8 + 8 * m, "P2": 8 * m, "P3": 9 * m,
            "P4": 2 * m + 2 * 8 + (2 * 8 if inc else 0)}


def kernel_bytes_per_cell(precision: str, scheme: str = "bdf2"):
    m = 8 if precision == "fp64" else 4
    # The BDF1 scheme's stencil pass reads level n only (phi*, psi* = phi^n, psi^n).
    levels = 3 if scheme == "bdf2" else 1
    return {
        "stencil": 2 * levels * 8 + 8 * m,
        "row_dct": 16 * m,
        "col_gram": 8 * m,
        "solve5": 0,
        "col_solve": (7 if precision == "fp64" else 8) * m + 2 * m,
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


def _traffic_record(workload: str, precision: str):
    """key: value lines of profiles/traffic_<workload>_<precision>.txt, or None
    when absent or taken on other kernel sources than these."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha") != source_digest():
        return None
    return kv


def stored_traffic(workload: str, precision: str, pass_name: str, cells: int):
    """HBM bytes of one run of a pass (the sum over its launches) from the
    committed rocprofv3 counter summary, or None."""
    kv = _traffic_record(workload, precision)
    try:
        return float(kv[f"{pass_name}_bytes_per_cell"]) * cells if kv else None
    except (KeyError, ValueError):
        return None


def stored_step_traffic(workload: str, precision: str):
    """HBM bytes per cell of one step from the committed counter summary, or None."""
    kv = _traffic_record(workload, precision)
    try:
        return float(kv["step_bytes_per_cell"]) if kv else None
    except (KeyError, ValueError):
        return None


# ---- digests of rocprofv3 output into the summaries under profiles/ ----------

def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(path, newline="") as f:
            rows.extend(csv.DictReader(f))
    if not rows:
        raise SystemExit(f"no *{suffix} under {directory}")
    return rows


def _short(name: str) -> str:
    """Kernel name without the return type and the argument list."""
    if name.startswith("void "):
        name = name[5:]
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i]
    return name


def digest_trace(directory: str, name: str, command: str):
    """profiles/kernel_trace_<name>.md from a rocprofv3 --kernel-trace --stats run."""
    rows = _csv_rows(directory, "kernel_stats.csv")
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = [f"# rocprofv3 kernel trace: {name}", "",
             "Command (on one MI355X; $REPO is the repository root):", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | share % |",
             "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{100.0 * float(r['TotalDurationNs']) / total:.1f} |")
    path = os.path.join(ROOT, "profiles", f"kernel_trace_{name}.md")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def _counter_means(directory: str, counter: str):
    """{kernel: (dispatches, mean KiB per dispatch)} and the largest copy-kernel value."""
    acc = {}
    copy = 0.0
    for r in _csv_rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = _short(r["Kernel_Name"])
        v = float(r["Counter_Value"])
        n, t = acc.get(k, (0, 0.0))
        acc[k] = (n + 1, t + v)
        if "copyBuffer" in k:
            copy = max(copy, v)
    return {k: (n, t / n) for k, (n, t) in acc.items()}, copy


def digest_pmc(directory: str, name: str, command: str, cus: int = 256):
    """profiles/counters_<name>.md: the mean per dispatch of every counter of
    a rocprofv3 --pmc run, per kernel, with the derived figures the summary
    uses: MFMA busy share = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE x CUs),
    matrix-core TFLOP/s = 512 x SQ_INSTS_VALU_MFMA_MOPS_BF16 / kernel time,
    LDS bank-conflict share = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS, mean
    resident waves = SQ_WAVE_CYCLES / SQ_BUSY_CYCLES."""
    rows = _csv_rows(directory, "counter_collection.csv")
    acc = {}
    for r in rows:
        k = _short(r["Kernel_Name"])
        d = acc.setdefault(k, {})
        cn = r["Counter_Name"]
        n, t = d.get(cn, (0, 0.0))
        d[cn] = (n + 1, t + float(r["Counter_Value"]))
        if cn == next(iter(d)):          # one duration sample per dispatch
            n2, t2 = d.get("_ns", (0, 0.0))
            d["_ns"] = (n2 + 1, t2 + float(r["End_Timestamp"]) - float(r["Start_Timestamp"]))
    names = sorted({c for d in acc.values() for c in d if c != "_ns"})
    lines = [f"# rocprofv3 counters: {name}", "",
             "Command (on one MI355X; $REPO is the repository root):", "", "```", command, "```",
             "", "Mean per dispatch. Derived: MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / "
             f"(GRBM_GUI_ACTIVE x {cus} CUs); MFMA TFLOP/s = 512 x SQ_INSTS_VALU_MFMA_MOPS_BF16 / "
             "dispatch time; LDS conflict = SQ_LDS_BANK_CONFLICT / SQ_ACTIVE_INST_LDS; waves = "
             "SQ_WAVE_CYCLES / SQ_BUSY_CYCLES (mean resident waves per busy SQ cycle, summed over "
             "the SQs).", "",
             "| kernel | dispatches | us | " + " | ".join(names) + " | derived |",
             "|---|---|---|" + "---|" * len(names) + "---|"]
    for k in sorted(acc):
        d = acc[k]
        mean = {c: t / n for c, (n, t) in d.items()}
        der = []
        us = mean.get("_ns", 0.0) / 1e3
        if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and mean.get("GRBM_GUI_ACTIVE"):
            der.append(f"MFMA busy {mean['SQ_VALU_MFMA_BUSY_CYCLES'] / (mean['GRBM_GUI_ACTIVE'] * cus):.2f}")
        if "SQ_INSTS_VALU_MFMA_MOPS_BF16" in mean and us > 0:
            der.append(f"MFMA {512 * mean['SQ_INSTS_VALU_MFMA_MOPS_BF16'] / (us * 1e-6) / 1e12:.0f} TFLOP/s")
        if mean.get("SQ_ACTIVE_INST_LDS"):
            der.append(f"LDS conflict {mean.get('SQ_LDS_BANK_CONFLICT', 0.0) / mean['SQ_ACTIVE_INST_LDS']:.3f}")
        if mean.get("SQ_BUSY_CYCLES") and "SQ_WAVE_CYCLES" in mean:
            der.append(f"waves {mean['SQ_WAVE_CYCLES'] / mean['SQ_BUSY_CYCLES']:.1f}")
        vals = " | ".join(f"{mean[c]:.4g}" if c in mean else "" for c in names)
        lines.append(f"| `{k}` | {d['_ns'][0]} | {us:.1f} | {vals} | {'; '.join(der)} |")
    path = os.path.join(ROOT, "profiles", f"counters_{name}.md")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(path)


def digest_counters(fetch_dir: str, write_dir: str, workload: str, precision: str,
                    probe_mib: int, commands: str, autotuned: str):
    """profiles/traffic_<workload>_<precision>.{md,txt} from one FETCH_SIZE and
    one WRITE_SIZE run of the same command ending with a plain device copy of
    probe_mib MiB: each counter is scaled so that the copy reads and writes
    its size, and per-dispatch bytes are divided by the cells of the grid.
    ``autotuned`` names the launch variant of each tuned kernel that the timed
    steps used, as `row_dct=1,col_solve=1,row_idct=0` (the first step runs
    both variants)."""
    from workloads import make_workload
    cells = sum(m.phi0.size for m in make_workload(workload))
    fetch, copy_f = _counter_means(fetch_dir, "FETCH_SIZE")
    write, copy_w = _counter_means(write_dir, "WRITE_SIZE")
    kib = probe_mib * 1024.0
    if copy_f <= 0 or copy_w <= 0:
        raise SystemExit("no copy-kernel dispatch found for the calibration")
    sf, sw = kib / copy_f, kib / copy_w
    per_cell = lambda v, s: v * s * 1024.0 / cells  # noqa: E731
    var = dict(kv.split("=") for kv in autotuned.split(",")) if autotuned else {}
    names = {"stencil": "k_stencil", "row_dct": "k_row_dct8", "col_gram": "k_col_gram",
             "solve5": "k_solve", "col_solve": "k_col_solve", "row_idct": "k_row_idct"}
    algo = kernel_bytes_per_cell(precision)
    rows, used = [], {}
    for k in sorted(set(fetch) | set(write)):
        nf, f = fetch.get(k, (0, 0.0))
        nw, w = write.get(k, (0, 0.0))
        bf, bw = per_cell(f, sf), per_cell(w, sw)
        # (the 5x5 kernel of large grids is k_solve_sliced)
        phase = next((ph for ph, kn in names.items()
                      if re.match(rf"ccm::{kn}(_sliced)?(<|$)", k)), None)
        chosen = phase is not None and (phase not in var or k.rstrip(">").endswith(f", {var[phase]}"))
        if chosen:
            # launches of several grid shapes (an ensemble) add up
            used[phase] = (used.get(phase, (0.0, ""))[0] + bf + bw, k)
        rows.append(f"| `{k}` | {max(nf, nw)} | {bf:.2f} | {bw:.2f} | {bf + bw:.2f} | "
                    f"{algo.get(phase, '') if phase else ''} | {'yes' if chosen else ''} |")
    step = sum(b for b, _ in used.values())
    passes = {ps: sum(used[k][0] for k in ks if k in used) for ps, ks in PASSES.items()}
    digest = source_digest()
    md = [f"# HBM traffic per kernel launch: {workload}, {precision}", "",
          "Two rocprofv3 counter runs on one MI355X ($REPO is the repository root):", "", "```",
          commands, "```", "",
          f"Calibration: each run ends with a plain {probe_mib} MiB device copy. For that copy "
          f"FETCH_SIZE reads {copy_f:.1f} KiB and WRITE_SIZE {copy_w:.1f} KiB of {kib:.0f} KiB moved, "
          f"so FETCH_SIZE is scaled by {sf:.4f} and WRITE_SIZE by {sw:.4f}. Bytes per cell = scaled "
          f"KiB per dispatch x 1024 / {cells} cells. Kernel sources hashed `{digest}` (code only, "
          "as bench.py's source_digest). The first step runs both launch variants of the "
          "autotuned kernels; 'step' marks the ones the timed steps use.", "",
          "| kernel | dispatches | fetch B/cell | write B/cell | total B/cell | algorithmic B/cell "
          "(this build's kernels) | step |", "|---|---|---|---|---|---|---|", *rows, "",
          f"Per step (the kernels marked 'step'): {step:.2f} B/cell. Per pass of the pipeline "
          f"model (algorithmic {pass_bytes_per_cell(precision)}): " +
          ", ".join(f"{ps} {b:.2f}" for ps, b in passes.items()) + " B/cell."]
    if precision == "gemm":
        # the matrix-core variant has its own kernels: the table only, no
        # per-pass record for the roofline line
        md = md[:md.index("| kernel | dispatches | fetch B/cell | write B/cell | total B/cell | "
                          "algorithmic B/cell (this build's kernels) | step |")]
        md = [ln.replace(" The first step runs both launch variants of the autotuned kernels; "
                         "'step' marks the ones the timed steps use.", "") for ln in md]
        md += ["| kernel | dispatches | fetch B/cell | write B/cell | total B/cell |",
               "|---|---|---|---|---|"]
        md += ["|".join(r.split("|")[:6]) + "|" for r in rows]
    base = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}")
    with open(base + ".md", "w") as f:
        f.write("\n".join(md) + "\n")
    if precision == "gemm":
        print(base + ".md")
        return
    txt = [f"# counter bytes per cell, {workload} {precision}; see traffic_{workload}_{precision}.md",
           f"workload: {workload}", f"precision: {precision}", f"source_sha: {digest}",
           f"fetch_scale: {sf:.6f}", f"write_scale: {sw:.6f}",
           f"step_bytes_per_cell: {step:.4f}"]
    txt += [f"{ps}_bytes_per_cell: {b:.4f}" for ps, b in passes.items()]
    txt += [f"{ph}_bytes_per_cell: {b:.4f}" for ph, (b, _) in sorted(used.items())]
    with open(base + ".txt", "w") as f:
        f.write("\n".join(txt) + "\n")
    print(base + ".md")


def host_cores() -> int:
    """Cores this process may run on (the affinity mask), else os.cpu_count()."""
    try:
        return len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        return os.cpu_count() or 1


def _oracle_leg(members, budget_s: float, workers: int):
    """The FP64 oracle as it stands over the first two steps (one BDF1, one
    BDF2) of as many members as fit in about ``budget_s`` seconds (at least
    one), with scipy's transforms on ``workers`` threads."""
    import scipy.fft
    from oracle import ccmsav_ref as R
    cells = 0
    taken = 0
    used = 0.0
    with scipy.fft.set_workers(workers):
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
    return cells / used / 1e6, taken, used


def cpu_baseline(members, budget_s: float = 12.0):
    """FP64 oracle timed on this host over a bounded sample of the workload:
    once with scipy's transforms (the oracle's DCTs above N = 512) on every
    core of the host, once on one thread. The all-core leg is the reported
    value; numpy's pointwise and stencil arithmetic stays on one thread in
    both, as the oracle is written."""
    cores = host_cores()
    v_all, taken, used_all = _oracle_leg(members, budget_s, cores)
    v_one, _, used_one = _oracle_leg(members[:taken], budget_s, 1)
    sizes = sorted({m.params["nx"] for m in members[:taken]})
    return {"value": v_all, "unit": "Mcell-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"the first 2 steps (one BDF1, one BDF2) of {taken} of {len(members)} "
                      f"member(s) (N={sizes}), numpy/scipy FP64: {used_all:.2f} s with scipy.fft "
                      f"on {cores} threads; {used_one:.2f} s on one thread",
            "single_thread_value": v_one, "host_cpu_count": os.cpu_count()}


def timed_run(C, torch, members, precision, steps, warmup, profile_steps, dev, graph,
              bdf1=False, classical=False, periodic=False, persistent=False):
    """Warm up, time ``steps`` steps between two synchronisations, then take
    ``profile_steps`` more with per-kernel events. Returns timings and the
    final states (after warmup + steps + profile_steps steps)."""
    phi0 = [torch.from_numpy(m.phi0).to(dev) for m in members]
    psi0 = [torch.from_numpy(m.psi0).to(dev) for m in members]
    stream = torch.cuda.current_stream(dev)
    ctx = C.Context.ensemble([m.params for m in members], phi0, psi0, precision,
                             stream=stream.cuda_stream, graph=graph, bdf1=bdf1,
                             classical=classical, periodic=periodic, persistent=persistent)
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
               pcg=ctx.pcg_stats() if classical else None,
               energy=[None if (bdf1 or classical) else ctx.energy(member=i) for i in range(nm)],
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
    ap.add_argument("--scheme", default="bdf2", choices=["bdf2", "bdf1", "classical"],
                    help="time-stepping scheme: CC-MSAV-BDF2 (the default), the "
                         "first-order CC-MSAV-BDF1 scheme at every step, or the classical "
                         "MSAV scheme with its PCG solves (FP64)")
    ap.add_argument("--persistent", action="store_true",
                    help="every step as one persistent kernel launch (mixed precision, grids "
                         "of 64 to 512)")
    ap.add_argument("--compare-persistent", action="store_true",
                    help="also time the persistent launch on the same workload and check that "
                         "its states equal the timed run's bit for bit")
    ap.add_argument("--periodic", action="store_true",
                    help="periodic boundaries (FP64 step with FFT solves)")
    ap.add_argument("--compare-classical", action="store_true",
                    help="also time the classical MSAV scheme (FP64, PCG) on the same workload "
                         "and report the CC-MSAV speedup on this GPU")
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
    ap.add_argument("--digest-trace", nargs=2, metavar=("DIR", "NAME"),
                    help="write profiles/kernel_trace_NAME.md from a rocprofv3 --stats output "
                         "directory (no GPU work); --digest-command gives the command text")
    ap.add_argument("--digest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic_<workload>_<precision>.{md,txt} from a "
                         "FETCH_SIZE and a WRITE_SIZE rocprofv3 run (no GPU work)")
    ap.add_argument("--digest-pmc", nargs=2, metavar=("DIR", "NAME"),
                    help="write profiles/counters_NAME.md from a rocprofv3 --pmc run (no GPU work)")
    ap.add_argument("--digest-command", default="", help="command text for the digests")
    ap.add_argument("--digest-autotuned", default="",
                    help="launch variants of the timed steps, e.g. row_dct=1,col_solve=1,row_idct=0")
    args = ap.parse_args()
    if args.digest_trace:
        digest_trace(args.digest_trace[0], args.digest_trace[1], args.digest_command)
        return
    if args.digest_pmc:
        digest_pmc(args.digest_pmc[0], args.digest_pmc[1], args.digest_command)
        return
    if args.digest_counters:
        digest_counters(args.digest_counters[0], args.digest_counters[1], args.workload,
                        args.precision, args.copy_probe_mib or 256, args.digest_command,
                        args.digest_autotuned)
        return
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
    classical = args.scheme == "classical"
    if classical or args.periodic:
        args.precision = "fp64"
    run = timed_run(C, torch, members, args.precision, args.steps, args.warmup,
                    args.profile_steps, dev, args.graph, bdf1, classical, args.periodic,
                    args.persistent)
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
    elif prof and not (classical or args.periodic or args.persistent):
        # The dominant pass of the pipeline model, by its launches' mean
        # durations on the library's stream (HIP events); P1 is the stencil
        # launch plus the row DCT launch.
        pb = pass_bytes_per_cell(args.precision, args.scheme)
        pass_ms = {ps: sum(prof[k] for k in ks) for ps, ks in PASSES.items()}
        for ps, ms in pass_ms.items():
            print(f"[bench] pass {ps} ({'+'.join(PASSES[ps])}): {ms * 1e3:.1f} us, {pb[ps]} B/cell "
                  f"(pipeline model), {pb[ps] * cells / (ms * 1e-3) / 1e9:.0f} GB/s",
                  file=sys.stderr, flush=True)
        dom = max(pass_ms, key=pass_ms.get)
        dom_bytes = pb[dom] * cells
        achieved = dom_bytes / (pass_ms[dom] * 1e-3) / 1e9
        traffic = stored_traffic(args.workload, args.precision, dom, cells)
        roofline = {"bound": "hbm", "kernel": f"{dom}: " + " + ".join(PASSES[dom]),
                    "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "bytes_per_launch": dom_bytes, "us_per_launch": pass_ms[dom] * 1e3,
                    "pass_us": {ps: ms * 1e3 for ps, ms in pass_ms.items()},
                    "step_bytes_per_cell": sum(pb.values()),
                    "step_frac": sum(pb.values()) * value * 1e6 / 1e9 / HBM_PEAK_GBS,
                    "kernel_bytes_per_cell": per_cell,
                    "kernel_step_frac": sum(per_cell.values()) * value * 1e6 / 1e9 / HBM_PEAK_GBS,
                    "counter_bytes_per_cell_step": stored_step_traffic(args.workload,
                                                                       args.precision)}

    finite = all(bool(np.all(np.isfinite(f[0]))) for f in run["fields"])
    if not (bdf1 or classical):
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

    if run["pcg"] is not None:
        check["pcg_iterations_last_step"], check["pcg_rel_residual_last_step"] = run["pcg"]
    if args.compare_classical and not classical:
        cl = timed_run(C, torch, members, "fp64", args.steps, args.warmup, 0, dev, False, bdf1,
                       True, False)
        cl_value = cells * args.steps / cl["wall"] / 1e6
        compare = dict(compare or {}, classical_value=cl_value,
                       classical_ms_per_step=1e3 * cl["wall"] / args.steps,
                       classical_pcg_iterations=cl["pcg"][0],
                       speedup_vs_classical=value / cl_value)
        if compare.get("fp64_value"):
            compare["fp64_speedup_vs_classical"] = compare["fp64_value"] / cl_value
        print(f"[bench] classical MSAV (FP64, PCG): {compare['classical_ms_per_step']:.4f} ms/step, "
              f"{cl_value:.1f} Mcell-steps/s, iterations {cl['pcg'][0]}; this path / classical = "
              f"{compare['speedup_vs_classical']:.2f}", file=sys.stderr, flush=True)

    if args.compare_persistent and not args.persistent:
        ps = timed_run(C, torch, members, args.precision, args.steps, args.warmup,
                       args.profile_steps, dev, args.graph, bdf1, False, False, True)
        same = all(np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
                   for a, b in zip(ps["fields"], run["fields"])) and all(
            np.array_equal(a, b) for a, b in zip(ps["savs"], run["savs"]))
        ps_value = cells * args.steps / ps["wall"] / 1e6
        compare = dict(compare or {}, persistent_value=ps_value,
                       persistent_ms_per_step=1e3 * ps["wall"] / args.steps,
                       persistent_bit_identical=bool(same),
                       persistent_vs_this=ps_value / value)
        print(f"[bench] persistent launch: {compare['persistent_ms_per_step']:.4f} ms/step, "
              f"{ps_value:.1f} Mcell-steps/s, bit-identical {same}; persistent / this = "
              f"{compare['persistent_vs_this']:.3f}", file=sys.stderr, flush=True)

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
              "boundaries": "periodic" if args.periodic else "neumann",
              "launch": "persistent" if args.persistent else "per-pass",
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
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "gemm": "bf16-split+f32+f64"}[args.precision],
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
