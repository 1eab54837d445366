"""Benchmark: periodic 2D Cahn-Hilliard ADI steps on one MI355X.

Default workload (the large single run at HBM scale): 8192 x 8192 grid on
(0, 2 pi)^2, D = 1, gamma = 0.001, dt = 1e-6, c0 = 0.05 sin(3x) sin(5y) +
U[-0.01, 0.01] (seed 5), FP64, mass and free energy recorded every step.
One step = the explicit right-hand side + batched cyclic pentadiagonal solves
along every column and every row (the whole hot path); the state stays
resident in HBM.

Prints one JSON line: throughput in grid-point updates/s, the roofline of the
dominant kernel (per-kernel HIP-event timing on the library's stream), the
oracle timed on the host, and the standalone batched-solve throughput.

    python bench.py [--gpus 1] [--steps 500] [--warmup 10]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "CH ADI grid-pt updates/s; penta-solve HBM GB/s % peak; FP32-refined vs FP64"
CSRC = os.path.join(ROOT, "paper_2101_06550_amd", "csrc")
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "ch_adi_8192x8192_fp64_traffic.md")
KERNEL_PROFILE = os.path.join(ROOT, "profiles", "ch_adi_8192x8192_fp64_kernel_stats.md")
KERNEL_OF_PHASE = {"column_pass": "ch_column_pass", "column_separators": "reduced_il_lds",
                   "row_pass": "row_solve_half", "separator_rows": "rows_sep",
                   "separators_and_interior_rows": "rows_split_fused"}
FIRST_WHOLE_COLUMN_SHAPE = 12  # separator shapes from here on run reduced_whole
HBM_PEAK_GBS = 8000.0
CHUNK = 32  # unknowns per thread-chunk in the library's chunked kernels


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def column_pass_bytes(nx, ny, m=CHUNK):
    """Algorithmic HBM bytes of one column-pass launch with m-point chunks:
    read the state once, write the chunk-interior solution, write 4
    separator parts per chunk."""
    n = nx * ny
    sc = ny // m
    return 8 * n + 8 * nx * (ny - 2 * sc) + 8 * 4 * sc * nx


def row_pass_bytes(nx, ny):
    return 16 * nx * ny


def reduced_bytes(nx, ny, m=CHUNK):
    sc = ny // m
    return 8 * 4 * sc * nx + 8 * 2 * sc * nx


# library sources that no kernel of the ADI step (nor the calibration copy)
# is built from: the standalone stencil and the per-system batched solves
NOT_IN_STEP = ("stencil.hip", "varband.hip")


def source_hash():
    """sha256 over the HIP/C++ sources that the step's kernels, their launch
    and tuning code and the calibration copy are built from (what the
    counters were taken on)."""
    import hashlib
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".hpp", ".cpp")) and name not in NOT_IN_STEP:
            with open(os.path.join(CSRC, name), "rb") as fh:
                h.update(name.encode() + b"\0" + fh.read())
    return h.hexdigest()


def summarize_pmc(fetch_dir, write_dir, out_path, command):
    """Turn two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
    dispatch) into per-kernel HBM bytes per dispatch, scaled by what the same
    counters read for the library's plain 1 GiB streaming copy run first
    (--calibrate-copy): scale = true KiB / counter KiB."""
    import collections
    import csv

    def load(d, counter):
        rows = []
        for root, _, files in os.walk(d):
            for f in files:
                if f.endswith("counter_collection.csv"):
                    with open(os.path.join(root, f)) as fh:
                        rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        return rows

    def after_marker(rows):
        # the calibration copies run after the handle is created (and tuned):
        # only the dispatches that follow them belong to the timed workload
        last = max(int(r["Dispatch_Id"]) for r in rows if "stream_copy_kernel" in r["Kernel_Name"])
        return [r for r in rows if int(r["Dispatch_Id"]) > last]

    true_kib = float(1 << 20)  # 1 GiB copy: 1 GiB read and 1 GiB written
    per = {}
    scale = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = load(d, counter)
        calib = [float(r["Counter_Value"]) for r in rows if "stream_copy_kernel" in r["Kernel_Name"]]
        calib = [v for v in calib if 0.5 * true_kib < v < 2 * true_kib]
        scale[counter] = true_kib / (sum(calib) / len(calib))
        acc = collections.defaultdict(list)
        for r in after_marker(rows):
            name = r["Kernel_Name"]
            short = name.split("(")[0].replace("void ", "").split("<")[0].split("::")[-1]
            acc[short].append(float(r["Counter_Value"]))
        per[counter] = {k: sum(v) / len(v) for k, v in acc.items()}
    # the library's kernels only (not the calibration copy, fills or blits)
    kernels = sorted(k for k in set(per["FETCH_SIZE"]) & set(per["WRITE_SIZE"])
                     if not k.startswith("__amd") and "elementwise" not in k
                     and "stream_copy" not in k)
    table = {}
    for k in kernels:
        fb = per["FETCH_SIZE"][k] * scale["FETCH_SIZE"] * 1024
        wb = per["WRITE_SIZE"][k] * scale["WRITE_SIZE"] * 1024
        table[k] = {"fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb}
    blob = {"source_sha256": source_hash(), "scale": scale, "kernels": table}
    lines = ["# HBM traffic per dispatch: CH ADI step, 8192 x 8192, FP64", "",
             "Commands (run from the repository root on one MI355X, each pass on its own):", "",
             "    " + command.replace("{C}", "FETCH_SIZE").replace("{D}", os.path.relpath(fetch_dir)),
             "    " + command.replace("{C}", "WRITE_SIZE").replace("{D}", os.path.relpath(write_dir)),
             "", "Summarised with `python bench.py --summarize-pmc <fetch dir> <write dir>`.",
             f"Copy calibration (1 GiB streaming copy, same run): FETCH_SIZE x "
             f"{scale['FETCH_SIZE']:.4f}, WRITE_SIZE x {scale['WRITE_SIZE']:.4f}.", "",
             "| Kernel | fetch MB/dispatch | write MB/dispatch | total MB |", "|---|---|---|---|"]
    for k, v in table.items():
        lines.append(f"| {k} | {v['fetch_bytes']/1e6:.1f} | {v['write_bytes']/1e6:.1f} | "
                     f"{v['traffic_bytes']/1e6:.1f} |")
    lines += ["", "Algorithmic bytes per dispatch at 8192 x 8192 (what bench.py divides by "
              "the launch time): ch_column_pass 1107.3 MB (read c, write the "
              "half-solved field and the separator right-hand sides, read the previous "
              "step's separator corrections), the separator kernel (reduced_whole or "
              "reduced_il_lds) 100.7 MB, row_solve_half "
              "1073.7 MB (read and write the field once).",
              "", "Valid for the library sources with this hash (bench.py reports `traffic` only "
              "while it matches):", "", "<!-- traffic-json: " + json.dumps(blob) + " -->", ""]
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines))
    return blob


def summarize_trace(trace_dir, out_path, command, note):
    """Per-kernel duration statistics of the dispatches that follow the last
    calibration copy in a rocprofv3 --kernel-trace run (the timed workload,
    without the autotuning launches of handle creation)."""
    import csv
    rows = []
    for root, _, files in os.walk(trace_dir):
        for f in files:
            if f.endswith("kernel_trace.csv"):
                with open(os.path.join(root, f)) as fh:
                    rows += list(csv.DictReader(fh))
    last = max(int(r["Dispatch_Id"]) for r in rows if "stream_copy_kernel" in r["Kernel_Name"])
    stats = {}
    for r in rows:
        if int(r["Dispatch_Id"]) <= last:
            continue
        name = r["Kernel_Name"].split("(")[0].replace("void ", "").split("<")[0].split("::")[-1]
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        stats.setdefault(name, []).append(d)
    total = sum(sum(v) for v in stats.values())
    lines = ["# Kernel trace: CH ADI step, 8192 x 8192, FP64 (large single-run workload)", "",
             "Command (run from the repository root on one MI355X):", "", "    " + command, "",
             "Summarised with `python bench.py --summarize-trace <trace dir>` over the "
             "dispatches that follow the calibration copy (the warm-up, timed and "
             "per-kernel-timing steps; not the autotuning launches of handle creation).", "",
             note, "",
             "| Kernel | Calls | Total ns | Average ns | % | Min ns | Max ns |",
             "|---|---|---|---|---|---|---|"]
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| {name} | {len(v)} | {sum(v)} | {sum(v) / len(v):.1f} | "
                     f"{100.0 * sum(v) / total:.2f} | {min(v)} | {max(v)} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return {k: sum(v) / len(v) for k, v in stats.items()}


def summarize_leg(trace_dir, out_path, title, command, note):
    """Per-kernel duration statistics of every dispatch of a rocprofv3
    --kernel-trace run of one side measurement (`bench.py --only ...`)."""
    import csv
    rows = []
    for root, _, files in os.walk(trace_dir):
        for f in files:
            if f.endswith("kernel_trace.csv"):
                with open(os.path.join(root, f)) as fh:
                    rows += list(csv.DictReader(fh))
    def short(raw):
        sig = raw.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "").strip()
        if sig.startswith("chx::"):  # this library: keep the template arguments
            return sig[len("chx::"):]
        base = sig.split("<")[0].split("::")[-1]
        return base or raw[:60]

    stats = {}
    for r in rows:
        name = short(r["Kernel_Name"])
        d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        stats.setdefault(name, []).append(d)
    total = sum(sum(v) for v in stats.values())
    lines = [f"# Kernel trace: {title}", "",
             "Command (run from the repository root on one MI355X):", "", "    " + command, "",
             "Summarised with `python bench.py --summarize-leg <trace dir> <this file> ...` over "
             "every dispatch of the run (handle creation, warm-up and timed calls).", "",
             note, "",
             "| Kernel | Calls | Total ns | Average ns | % | Min ns | Max ns |",
             "|---|---|---|---|---|---|---|"]
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1]))[:16]:
        lines.append(f"| {name} | {len(v)} | {sum(v)} | {sum(v) / len(v):.1f} | "
                     f"{100.0 * sum(v) / total:.2f} | {min(v)} | {max(v)} |")
    with open(out_path, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def stored_traffic(kernel):
    """Bytes per dispatch of `kernel` from the committed profile, or None if
    the profile is absent or was taken on different sources."""
    try:
        text = open(TRAFFIC_PROFILE).read()
        blob = json.loads(text.split("<!-- traffic-json: ", 1)[1].split(" -->", 1)[0])
    except (OSError, IndexError, ValueError):
        return None
    if blob.get("source_sha256") != source_hash():
        return None
    ent = blob["kernels"].get(kernel)
    return None if ent is None else ent["traffic_bytes"]


def cpu_baseline(c0, L, D, gamma, dt, budget_s=12.0, max_steps=3):
    """The oracle timed on the host (one thread) on a bounded sample of the
    workload; also returns its first step for the GPU error check."""
    import oracle
    orc = oracle.oracle()
    n = c0.size
    steps, t0 = 0, time.perf_counter()
    c = c0
    first = None
    while steps < max_steps:
        c = orc.ch_step(c, L, L, D, gamma, dt)
        if first is None:
            first = c
        steps += 1
        if time.perf_counter() - t0 > budget_s:
            break
    el = time.perf_counter() - t0
    return {"value": n * steps / el, "unit": "grid-point updates/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{steps} serial FP64 oracle ADI steps of the {c0.shape[1]}x{c0.shape[0]} "
                      f"workload ({el:.1f} s, single thread)"}, first


def _oracle_worker(job):
    """One process of the all-cores oracle timing: the serial oracle on its
    share of a workload until budget_s has passed.  Returns (units, seconds)."""
    kind, share, budget_s = job
    import oracle
    from paper_2101_06550_amd import inputs
    orc = oracle.oracle()
    L = 2 * math.pi
    units, t0 = 0, time.perf_counter()
    if kind == "ensemble":  # whole steps of this process's runs, in turn
        fields = [(n, inputs.noise_field(n, n, 1000 + r)) for r, n in share]
        while time.perf_counter() - t0 < budget_s:
            for k, (n, c) in enumerate(fields):
                fields[k] = (n, orc.ch_step(c, L, L, 1.0, 0.01, 1e-4))
                units += n * n
                if time.perf_counter() - t0 >= budget_s:
                    break
    else:  # cyclic penta solves, N = 1024, alpha = 0.5: this process's systems as rows
        a = 0.5
        coefs = (a, -4 * a, 1 + 6 * a, -4 * a, a)
        rhs = np.stack([inputs.uniform(2 + s, (1024,), -1, 1) for s in share])
        while time.perf_counter() - t0 < budget_s:
            orc.cpenta_lines(rhs, 0, coefs)
            units += len(share)
    return units, time.perf_counter() - t0


def cpu_all_cores(budget_s=8.0, procs=None):
    """The serial oracle run as independent processes on all host cores (at
    most 16), for the two workloads made of independent pieces: the uneven
    ensemble (each process steps its share of the 256 runs) and the batched
    cyclic penta solves (each process solves its share of 1024 systems).
    Aggregate rate = total units / longest process time."""
    import multiprocessing
    from concurrent.futures import ProcessPoolExecutor
    procs = procs or min(16, os.cpu_count() or 1)
    sizes = [128] * 96 + [256] * 96 + [512] * 64
    runs = list(enumerate(sizes))
    out = {"cores": procs, "kind": "oracle, one serial process per core"}
    ctx = multiprocessing.get_context("spawn")  # no fork of a process that holds the GPU
    with ProcessPoolExecutor(max_workers=procs, mp_context=ctx) as ex:
        for kind, items, unit in (("ensemble", runs, "grid-point updates/s"),
                                  ("solves", list(range(1024)), "solves/s")):
            jobs = [(kind, items[p::procs], budget_s) for p in range(procs)]
            res = list(ex.map(_oracle_worker, jobs))
            total = sum(u for u, _ in res)
            el = max(t for _, t in res)
            out[kind] = {"value": total / el, "unit": unit,
                         "sample": f"{procs} processes x {budget_s:.0f} s of the serial oracle "
                                   + ("stepping their share of the 256 runs (96 x 128^2, "
                                      "96 x 256^2, 64 x 512^2)" if kind == "ensemble" else
                                      "solving their share of 1024 cyclic penta systems "
                                      "(N = 1024, alpha = 0.5)")}
    return out


def solve_throughput(chx, torch, reps=10):
    """Standalone batched cyclic penta solves, N = 1024, alpha = 0.5, scaled
    batch of 131072 systems (1 GiB FP64), interleaved and contiguous."""
    from paper_2101_06550_amd import inputs
    n, batch, a = 1024, 131072, 0.5
    plan = chx.penta_factor(n, a, -4 * a, 1 + 6 * a, -4 * a, a)
    out = {}
    for name, layout, shape, bpu in (("interleaved", 0, (n, batch), None),
                                     ("contiguous", 1, (batch, n), 16)):
        x = torch.tensor(inputs.uniform(2, shape, -1, 1), device="cuda")
        ws = torch.empty(chx.penta_solve_ws_bytes(plan, batch, layout) + 256, dtype=torch.uint8,
                         device="cuda")
        chx.penta_solve_batch(plan, batch, x, layout=layout, ws=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            chx.penta_solve_batch(plan, batch, x, layout=layout, ws=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        if bpu is None:
            # first pass (read f, write 4 separator parts per chunk) + separators
            # + second pass (read the interior of f and the separators of the
            # chunk and its predecessor, write the interior of x)
            mi = CHUNK - 2
            bpu = (8 + 32 / CHUNK) + (32 + 16) / CHUNK + (2 * 8 * mi / CHUNK + 32 / CHUNK)
        gbs = bpu * n * batch / (ms * 1e-3) / 1e9
        out[name] = {"systems": batch, "n": n, "ms_per_solve_batch": round(ms, 4),
                     "solves_per_s": batch / (ms * 1e-3),
                     "algorithmic_bytes_per_unknown": round(bpu, 3),
                     "effective_GBps": round(gbs, 1),
                     "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                     # a two-sweep one-thread-per-system solve moves 32 B per unknown
                     "GBps_at_32B_per_unknown": round(32 * n * batch / (ms * 1e-3) / 1e9, 1)}
        del x, ws
    return out


def per_system_throughput(chx, torch, reps=10):
    """Batches with one matrix per system (Ch.4 benchmark shape: identical
    periodic Crank-Nicolson hyperdiffusion systems, gamma = D = L = 1,
    dt = 1e-8, n = 1024, 65536 systems, each stored with its own diagonals),
    in the factor-once mode and in the Rewrite mode (factor and solve at every
    call); the tridiagonal analogue with beta = 0.5.  Algorithmic bytes: the
    accesses a one-thread-per-system two-pass solve must make per unknown
    (periodic penta: rewrite 17, solve 13; tri: rewrite 11, solve 9; 8 B
    each)."""
    from paper_2101_06550_amd import inputs
    n, batch = 1024, 65536
    sig = 1e-8 / (2 * (1.0 / n) ** 4)
    dev = dict(dtype=torch.float64, device="cuda")
    f = torch.tensor(inputs.uniform(4, (n, batch), -1, 1), **dev)
    out = {"n": n, "systems": batch, "periodic": True}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    def entry(ms, acc):
        gbs = 8 * acc * n * batch / (ms * 1e-3) / 1e9
        return {"ms": round(ms, 4), "solves_per_s": batch / (ms * 1e-3),
                "algorithmic_bytes_per_unknown": 8 * acc, "effective_GBps": round(gbs, 1),
                "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}

    diag = [torch.full((n, batch), v, **dev)
            for v in (sig, -4 * sig, 1 + 6 * sig, -4 * sig, sig)]
    x = f.clone()
    ws = torch.empty(chx.penta_batch_ws_bytes(n, batch, True, chx.CHX_BATCH_REWRITE) + 256,
                     dtype=torch.uint8, device="cuda")
    out["penta_rewrite"] = entry(timed(lambda: chx.penta_batch_rewrite(*diag, x, ws=ws)), 17)
    del ws
    fws = chx.penta_batch_factor(*diag)
    out["penta_solve_factored"] = entry(
        timed(lambda: chx.penta_batch_solve(*diag, x, ws=fws)), 13)
    del diag, fws
    tri = [torch.full((n, batch), v, **dev) for v in (-0.5, 2.0, -0.5)]
    ws = torch.empty(chx.tri_batch_ws_bytes(n, batch, True, chx.CHX_BATCH_REWRITE) + 256,
                     dtype=torch.uint8, device="cuda")
    out["tri_rewrite"] = entry(timed(lambda: chx.tri_batch_rewrite(*tri, x, ws=ws)), 11)
    del ws
    fws = chx.tri_batch_factor(*tri)
    out["tri_solve_factored"] = entry(timed(lambda: chx.tri_batch_solve(*tri, x, ws=fws)), 9)
    out["finite"] = bool(torch.isfinite(x).all())
    del tri, fws, x, f
    return out


def stencil_throughput(chx, torch, n=8192, reps=20):
    """The standalone 2D stencil (Ch.3 API) on an n x n FP64 field, input and
    output separate: the 5-point Laplacian, the same applied to c^3 - c (the
    non-linear Cahn-Hilliard term), a full 5 x 5 stencil, the 8th-order second
    derivative in x of the Ch.3 example (non-periodic) and a full 9 x 9
    stencil, on FP64 arrays and again on FP32 arrays (names ending _f32).
    Algorithmic bytes: 16 (FP32: 8) per point (each input read once, each
    output written once); flops: 2 per weight per point (every weight of the
    rectangle is applied, zeros included)."""
    from paper_2101_06550_amd import inputs
    lap = [0, 1, 0, 1, -4, 1, 0, 1, 0]
    d8 = [-1 / 560, 8 / 315, -1 / 5, 8 / 5, -205 / 72, 8 / 5, -1 / 5, 8 / 315, -1 / 560]
    cases = {"laplacian_5pt": (lap, (1, 1, 1, 1), True, 0),
             "laplacian_of_c3_minus_c": (lap, (1, 1, 1, 1), True, 1),
             "full_5x5": (list(inputs.uniform(12, (25,), -1, 1)), (2, 2, 2, 2), True, 0),
             "x_8th_order_nonperiodic": (d8, (4, 4, 0, 0), False, 0),
             "full_9x9": (list(inputs.uniform(13, (81,), -1, 1)), (4, 4, 4, 4), True, 0)}
    out = {"n": n}
    finite = True
    # FP64 arrays (16 B per point), then the same stencils on FP32 arrays
    # (dtype CHX_F32: 8 B per point, sums in FP32)
    for dt_, tag, prec in ((torch.float64, "", "fp64"), (torch.float32, "_f32", "fp32")):
        x = torch.tensor(inputs.uniform(11, (n, n), -1, 1), dtype=dt_, device="cuda")
        y = torch.empty_like(x)
        bpp = 2.0 * x.element_size()
        for name, (w, ext, per, pm) in cases.items():
            def run():
                chx.stencil2d_apply(x, y, w, *ext, periodic=per, premap=pm)
            run()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            gbs = bpp * n * n / (ms * 1e-3) / 1e9
            out[name + tag] = {"ms": round(ms, 4), "points_per_s": n * n / (ms * 1e-3),
                               "effective_GBps": round(gbs, 1),
                               "frac_of_hbm_peak": round(gbs / HBM_PEAK_GBS, 4),
                               f"{prec}_TFLOPs": round(2.0 * len(w) * n * n / (ms * 1e-3) / 1e12,
                                                       2)}
        finite = finite and bool(torch.isfinite(y).all())
        del x, y
    out["finite"] = finite
    return out


def ensemble_throughput(chx, torch, steps=2000, warmup=20):
    """Uneven ensemble: 96 x 128^2 + 96 x 256^2 + 64 x 512^2 runs (seeds
    1000-1255, U[-0.1, 0.1]), D = 1, gamma = 0.01, dt = 1e-4, FP64; all runs
    advance together (one launch per phase, whole call replayed as a graph)."""
    from paper_2101_06550_amd import inputs
    L = 2 * math.pi
    sizes = [128] * 96 + [256] * 96 + [512] * 64
    ens = chx.ch_ensemble_create([(n, n, L, L, 1.0, 0.01, 1e-4) for n in sizes])
    fields = [torch.tensor(inputs.noise_field(n, n, 1000 + r), device="cuda")
              for r, n in enumerate(sizes)]
    points = sum(n * n for n in sizes)
    out = {"runs": len(sizes), "points_per_step": points}
    for name, graph, k in (("graph", True, steps), ("eager", False, min(steps, 200))):
        chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=graph)  # warm (and capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=graph)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"steps": k, "ms_per_step": round(1e3 * el / k, 5),
                     "updates_per_s": points * k / el,
                     "algorithmic_GBps": round(34.0 * points * k / el / 1e9, 1)}
    # the same runs with Cahn-Hilliard-Cook forcing (sigma = 1e-10, seed
    # 5000 + r per run), replayed from a graph
    chx.ch_ensemble_set_noise(ens, 1e-10, [5000 + r for r in range(len(sizes))])
    k = min(steps, 200)
    chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["cook_forced_graph"] = {"steps": k, "ms_per_step": round(1e3 * el / k, 5),
                                "updates_per_s": points * k / el}
    del ens
    # the same runs FP32-refined (2 passes: kappa = 706 at 512^2), replayed
    # from a graph: every phase of the refined step one launch for all runs
    ens = chx.ch_ensemble_create([(n, n, L, L, 1.0, 0.01, 1e-4) for n in sizes],
                                 dtype=chx.CHX_F32_REFINED, refine_passes=2)
    k = min(steps, 100)
    chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chx.ch_ensemble_step(ens, fields, nsteps=k, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rb = refined_bytes_per_point(2, k)
    out["f32_refined_2pass_graph"] = {"steps": k, "ms_per_step": round(1e3 * el / k, 5),
                                      "updates_per_s": points * k / el,
                                      "algorithmic_bytes_per_point": rb,
                                      "algorithmic_GBps": round(rb * points * k / el / 1e9, 1)}
    f64 = out["graph"]["updates_per_s"]
    ref = out["f32_refined_2pass_graph"]["updates_per_s"]
    out["f32_refined_vs_f64"] = {
        "refined_beats_f64": bool(ref > f64), "updates_ratio_refined_over_f64": round(ref / f64, 3),
        "bytes_per_point_f64": 34.0, "bytes_per_point_refined_2pass": round(rb, 2),
        "why": "both paths stream HBM at similar rates; FP64 sweeps cost no more time than FP32 "
               "ones here, and refinement must still read and write FP64 right-hand sides, "
               "states and the deferred FP32 solutions of every pass"}
    del fields, ens
    return out


def refined_bytes_per_point(p, steps=1):
    """Algorithmic HBM bytes per point and step of FP32-refined ADI steps with
    p refinement passes, averaged over a call of `steps` steps.  A step: the
    first column pass reads the state (the caller's c on the first step, 8 B;
    on later steps the previous step's deferred FP32 solutions V_0..V_p,
    4 (p + 1) B), writes r (8) and the FP32 chunk interiors and parts (4.25);
    FP32 separators 0.75; FP32 row solves 8; pass k adds the residual column
    pass (read r 8 and V_0..V_{k-1} 4 k, write 4.25), separators 0.75 and rows
    8.  After the last step the state is rebuilt from V_0..V_p (4 (p + 1)) and
    written to c (8).  Per step in a long call: 54, 87, 124 B for p = 1, 2, 3
    (the FP64 step: 34 B)."""
    steady = 21.0 + 4.0 * (p + 1) + sum(21.0 + 4.0 * k for k in range(1, p + 1))
    return steady + 16.0 / steps


def small_run(chx, torch, steps=1000):
    """128^2, U[-0.1, 0.1] (seed 1), D = 1, gamma = 0.01, dt = 1e-4, 1000
    steps, FP64: the single-workgroup path (field resident in LDS, one launch
    for all steps) against the multi-kernel path (three launches per step),
    eager and replayed from a captured graph (the ensemble entry point with
    one run)."""
    from paper_2101_06550_amd import inputs
    L = 2 * math.pi
    n = 128
    c0 = inputs.noise_field(n, n, 1)
    out = {"points": n * n, "steps": steps}
    h = chx.ch_create(n, n, L, L, 1.0, 0.01, 1e-4)
    res = {}
    for name, small in (("single_workgroup_lds", 1), ("multi_kernel", 0)):
        chx.ch_set_tuning(h, small, what=chx.CHX_TUNE_SMALL_PATH)
        c = torch.tensor(c0, device="cuda")
        chx.ch_adi_step(h, c, nsteps=10)
        torch.cuda.synchronize()
        c = torch.tensor(c0, device="cuda")
        t0 = time.perf_counter()
        chx.ch_adi_step(h, c, nsteps=steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"ms_per_step": round(1e3 * el / steps, 5), "updates_per_s": n * n * steps / el}
        res[name] = c.cpu().numpy()
    out["paths_max_abs_diff"] = float(np.max(np.abs(res["single_workgroup_lds"] -
                                                    res["multi_kernel"])))
    ens = chx.ch_ensemble_create([(n, n, L, L, 1.0, 0.01, 1e-4)])
    g = [torch.tensor(c0, device="cuda")]
    chx.ch_ensemble_step(ens, g, nsteps=steps, use_graph=True)  # capture
    torch.cuda.synchronize()
    g[0].copy_(torch.tensor(c0, device="cuda"))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chx.ch_ensemble_step(ens, g, nsteps=steps, use_graph=True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out["graph_single_workgroup"] = {"ms_per_step": round(1e3 * el / steps, 5),
                                     "updates_per_s": n * n * steps / el}
    return out


def p2_run(chx, torch):
    """The thesis's own delta-form scheme (Ch.3 eq. 3:ch_adi): time per step
    at 1024^2 (dt = 1e-5, gamma = 0.01) and 8192^2 (the large workload's
    parameters), FP64, and the one-step error against the oracle at 1024^2."""
    import oracle
    from paper_2101_06550_amd import inputs
    L = 2 * math.pi
    out = {}
    for n, g, dt, c0, k in ((1024, 0.01, 1e-5, inputs.noise_field(1024, 1024, 3), 200),
                           (8192, 0.001, 1e-6, inputs.mode_plus_noise(8192, 5), 20)):
        h = chx.ch_create(n, n, L, L, 1.0, g, dt, scheme=chx.CHX_SCHEME_P2)
        c, cp = torch.tensor(c0, device="cuda"), torch.tensor(c0, device="cuda")
        chx.ch_adi_step_p2(h, c, cp, nsteps=2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chx.ch_adi_step_p2(h, c, cp, nsteps=k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        ent = {"steps": k, "ms_per_step": round(1e3 * el / k, 5), "updates_per_s": n * n * k / el}
        if n == 1024:
            c, cp = torch.tensor(c0, device="cuda"), torch.tensor(c0, device="cuda")
            chx.ch_adi_step_p2(h, c, cp, nsteps=1)
            ref, _ = oracle.oracle().ch2_step(c0, c0, L, L, 1.0, g, dt)
            ent["one_step_rel_err_vs_oracle"] = rel_inf(c.cpu().numpy(), ref)
        out[f"{n}x{n}"] = ent
        del c, cp, h
    return out


def table31_run(chx, torch, sizes=(64, 128, 256, 512, 1024, 2048, 4096, 8192), T=10.0,
                eps=1e-6):
    """The convergence study of Table 3.1 with the thesis's scheme on the GPU:
    C(x, 0) = eps tanh(r - pi) with r the distance from the box's centre
    (pi, pi) and eps = 1e-6 as printed, D = 1, gamma = 0.01, to T = 10 with
    dt = 0.1 dx (rounded to a whole number of steps ending exactly at T), and
    E_N = mean over the coarse cells of |(2 x 2 average of C_N) - C_{N/2}|
    (Ch.2 eq. 2:converge2D); the printed column is reported beside it."""
    printed = {128: 0.1510, 256: 0.0246, 512: 0.0116, 1024: 0.0057, 2048: 0.0028,
               4096: 0.0014, 8192: 0.0007}
    L = 2 * math.pi
    fields, out = {}, {}
    for n in sizes:
        dx = L / n
        steps = int(round(T / (0.1 * dx)))
        dt = T / steps
        x = np.arange(n) * dx
        r = np.sqrt((x[None, :] - math.pi) ** 2 + (x[:, None] - math.pi) ** 2)
        c0 = eps * np.tanh(r - math.pi)
        h = chx.ch_create(n, n, L, L, 1.0, 0.01, dt, scheme=chx.CHX_SCHEME_P2)
        c, cp = torch.tensor(c0, device="cuda"), torch.tensor(c0, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:  # chunks of at most 4096 steps keep progress visible
            k = min(4096, steps - done)
            chx.ch_adi_step_p2(h, c, cp, nsteps=k)
            torch.cuda.synchronize()
            done += k
        el = time.perf_counter() - t0
        fields[n] = c.cpu().numpy()
        out[str(n)] = {"steps": steps, "dt": dt, "seconds": round(el, 3),
                       "max_abs_C": float(np.max(np.abs(fields[n])))}
        log(f"table 3.1 run N={n}: {steps} steps in {el:.2f} s")
        del c, cp, h
        if n // 2 in fields:
            f, cg = fields[n], fields.pop(n // 2)
            avg = 0.25 * (f[0::2, 0::2] + f[0::2, 1::2] + f[1::2, 0::2] + f[1::2, 1::2])
            out[str(n)]["E_N"] = float(np.mean(np.abs(avg - cg)))
            out[str(n)]["E_N_printed"] = printed.get(n)
    for n in sizes[1:-1]:
        out[str(n)]["log2_E_N_over_E_2N"] = math.log2(out[str(n)]["E_N"] /
                                                      out[str(2 * n)]["E_N"])
    return out


def batch1d_run(chx, torch):
    """Batched 1D periodic schemes: the 1D Cahn-Hilliard batch of the thesis's
    coarsening statistics (2^20 systems of N = 256 on (0, 2 pi), gamma = 0.01,
    dt = 0.1 dx, U[-0.1, 0.1], Ch.6-7) and Crank-Nicolson hyperdiffusion
    (65536 systems of N = 1024, dt = 1e-12, the Ch.4 scheme); FP64, 100 steps;
    algorithmic traffic 18 B per unknown per step (sweep: read the state,
    write the chunk interior and 4 parts per 32 unknowns; separators: 1.5 B),
    the correction deferred into the next sweep."""
    from paper_2101_06550_amd import inputs
    out = {}
    for name, kind, n, batch, L, dt, a in (
            ("cahn_hilliard_1d_1048576x256", 2, 256, 1 << 20, 2 * math.pi,
             0.1 * 2 * math.pi / 256, 0.01),
            ("hyperdiffusion_cn_65536x1024", 0, 1024, 1 << 16, 1.0, 1e-12, 1.0)):
        b = chx.batch1d_create(kind, n, L, dt, a)
        x = torch.tensor(inputs.uniform(60, (n, batch), -0.1, 0.1), device="cuda")
        chx.batch1d_step(b, x, nsteps=5)
        torch.cuda.synchronize()
        k = 100
        t0 = time.perf_counter()
        chx.batch1d_step(b, x, nsteps=k)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"steps": k, "ms_per_step": round(1e3 * el / k, 5),
                     "system_steps_per_s": batch * k / el,
                     "algorithmic_GBps": round(18.0 * n * batch * k / el / 1e9, 1),
                     "finite": bool(torch.isfinite(x).all())}
        if kind == 0:
            # the thesis's Rewrite mode on the same batch: diagonals written and
            # every system factored and solved afresh each step; 192 B per unknown
            # (right-hand side 16, five bands 40, fused factor-and-solve 136)
            ws = chx.batch1d_step_rewrite(b, x, nsteps=2)
            torch.cuda.synchronize()
            kr = 20
            t0 = time.perf_counter()
            chx.batch1d_step_rewrite(b, x, nsteps=kr, ws=ws)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[name + "_rewrite"] = {"steps": kr, "ms_per_step": round(1e3 * el / kr, 5),
                                      "system_steps_per_s": batch * kr / el,
                                      "algorithmic_GBps": round(192.0 * n * batch * kr / el / 1e9, 1),
                                      "finite": bool(torch.isfinite(x).all())}
            del ws
        del x, b
    return out


def cook_run(chx, torch, n=8192, steps=20):
    """The large workload with the Cahn-Hilliard-Cook forcing of Ch.7
    (sigma = 1e-14, the thesis's value): time per step with the per-step
    Box-Muller draws and the forced column pass, FP64."""
    from paper_2101_06550_amd import inputs
    L = 2 * math.pi
    h = chx.ch_create(n, n, L, L, 1.0, 0.001, 1e-6)
    chx.ch_set_noise(h, 1e-14, seed=2021)
    c = torch.tensor(inputs.mode_plus_noise(n, 5), device="cuda")
    chx.ch_adi_step(h, c, nsteps=2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chx.ch_adi_step(h, c, nsteps=steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms, cnt = chx.ch_adi_step_timed(h, c, nsteps=steps)
    return {"steps": steps, "ms_per_step": round(1e3 * el / steps, 5),
            "updates_per_s": n * n * steps / el,
            "column_phase_incl_draws_avg_ms": round(ms[0] / steps, 5)}


def copy_reference(chx, torch, reps=20):
    """The library's plain streaming copy of 1 GiB of FP64 (read 1 GiB, write
    1 GiB): the HBM rate a simple streaming kernel reaches on this part, for
    context next to the 8 TB/s peak."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    chx.chx_stream_copy(src, dst)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        chx.chx_stream_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    ok = bool(torch.equal(src, dst))
    del src, dst
    return {"bytes": 2 << 30, "ms": round(ms, 4), "GBps": round((2 << 30) / (ms * 1e-3) / 1e9, 1),
            "copy_exact": ok}


def settle_clocks(chx, torch, ms):
    """Stream 1 GiB copies until ms milliseconds have passed (synchronising
    every 8 copies); returns the time spent."""
    src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < ms:
        for _ in range(8):
            chx.chx_stream_copy(src, dst)
        torch.cuda.synchronize()
    spent = (time.perf_counter() - t0) * 1e3
    del src, dst
    return spent


def tuning_sweep(chx, torch, n=8192, steps=20):
    """Per-phase kernel times of the large workload for every separator tile
    shape (plain row pass) and every split-row-pass shape."""
    from paper_2101_06550_amd import inputs
    L = 2 * math.pi
    h = chx.ch_create(n, n, L, L, 1.0, 0.001, 1e-6)
    c0 = torch.tensor(inputs.mode_plus_noise(n, 5), device="cuda")
    out = {"tuned": {"separator_shape": chx.ch_get_tuning(h),
                     "row_split": chx.ch_get_tuning(h, chx.CHX_TUNE_ROW_SPLIT)}}
    choices = [("shape", k, -1) for k in range(chx.CHX_NUM_REDUCED_SHAPES)] + \
              [("split", 0, k) for k in range(chx.CHX_NUM_SPLIT_SHAPES)]
    for what in (chx.CHX_TUNE_COLUMN_CHUNK, chx.CHX_TUNE_ROW_CHUNK):  # split forms need 32
        chx.ch_set_tuning(h, CHUNK, what=what)
    for kind, shape, split in choices:
        chx.ch_set_tuning(h, shape)
        chx.ch_set_tuning(h, split, what=chx.CHX_TUNE_ROW_SPLIT)
        c = c0.clone()
        ms, cnt = chx.ch_adi_step_timed(h, c, nsteps=steps)
        c = c0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        chx.ch_adi_step(h, c, nsteps=steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[f"{kind}_{shape if kind == 'shape' else split}"] = {
            "phase_avg_ms": [round(m / k, 5) if k else 0.0 for m, k in zip(ms, cnt)],
            "ms_per_step": round(1e3 * el / steps, 5)}
    return out


def rel_inf(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def solve_precision(chx, torch, reps=20):
    """1024 cyclic penta (alpha = 0.5) and tri (beta = 0.5) systems of
    N = 1024, RHS ~ U[-1, 1] (seed 2): FP64 vs FP32 sweeps + FP64-residual
    refinement, time per batch and error vs the oracle."""
    import oracle
    from paper_2101_06550_amd import inputs
    orc = oracle.oracle()
    n = batch = 1024
    f = inputs.uniform(2, (n, batch), -1, 1)
    out = {}
    for kind, co in (("penta", (0.5, -2.0, 4.0, -2.0, 0.5)), ("tri", (-0.5, 2.0, -0.5))):
        plan = chx.penta_factor(n, *co) if kind == "penta" else chx.tri_factor(n, *co)
        solve = chx.penta_solve_batch if kind == "penta" else chx.tri_solve_batch
        for layout, lname in ((0, "interleaved"), (1, "contiguous")):
            fl = f if layout == 0 else np.ascontiguousarray(f.T)
            ref = (orc.cpenta_lines if kind == "penta" else orc.ctri_lines)(
                fl, 1 if layout == 0 else 0, co)
            for dtype, passes, tag in ((chx.CHX_F64, 0, "f64"), (chx.CHX_F32_REFINED, 1, "f32r1"),
                                       (chx.CHX_F32_REFINED, 2, "f32r2")):
                x0 = torch.tensor(fl, device="cuda")
                x = x0.clone()
                ws = torch.empty(chx.penta_solve_ws_bytes(plan, batch, layout, dtype) + 256
                                 if kind == "penta" else
                                 chx.tri_solve_ws_bytes(plan, batch, layout, dtype) + 256,
                                 dtype=torch.uint8, device="cuda")
                solve(plan, batch, x, layout=layout, dtype=dtype, refine_passes=passes, ws=ws)
                torch.cuda.synchronize()
                err = rel_inf(x.cpu().numpy(), ref)
                xs = [x0.clone() for _ in range(reps)]
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for xi in xs:
                    solve(plan, batch, xi, layout=layout, dtype=dtype, refine_passes=passes, ws=ws)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                out[f"{kind}_{lname}_{tag}"] = {"ms": round(ms, 5),
                                                "solves_per_s": batch / (ms * 1e-3),
                                                "rel_err_vs_oracle": err}
    return out


def precision_run(chx, torch, steps=10000, every=1000):
    """1024^2, U[-0.1, 0.1] (seed 3), D = 1, gamma = 0.01, dt = 1e-5: FP64 vs
    FP32-refined (1 and 2 passes) trajectories, L-inf difference from the FP64
    trajectory every 1000 steps, and the one-step error vs the oracle from the
    FP64 state at those steps."""
    import oracle
    from paper_2101_06550_amd import inputs
    orc = oracle.oracle()
    L = 2 * math.pi
    n, D, g, dt = 1024, 1.0, 0.01, 1e-5
    c0 = inputs.noise_field(n, n, 3)
    hs = {"f64": chx.ch_create(n, n, L, L, D, g, dt),
          "f32r1": chx.ch_create(n, n, L, L, D, g, dt, dtype=chx.CHX_F32_REFINED, refine_passes=1),
          "f32r2": chx.ch_create(n, n, L, L, D, g, dt, dtype=chx.CHX_F32_REFINED, refine_passes=2)}
    fields = {k: torch.tensor(c0, device="cuda") for k in hs}
    out = {k: {"ms_per_step": 0.0, "linf_vs_f64": [], "one_step_rel_err_vs_oracle": []}
           for k in hs}
    for m in range(0, steps, every):
        ref_state = fields["f64"].cpu().numpy()
        ref_next = orc.ch_step(ref_state, L, L, D, g, dt)
        for k, h in hs.items():
            probe = torch.tensor(ref_state, device="cuda")
            chx.ch_adi_step(h, probe, nsteps=1)
            torch.cuda.synchronize()
            out[k]["one_step_rel_err_vs_oracle"].append(rel_inf(probe.cpu().numpy(), ref_next))
        for k, h in hs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            chx.ch_adi_step(h, fields[k], nsteps=every)
            torch.cuda.synchronize()
            out[k]["ms_per_step"] += 1e3 * (time.perf_counter() - t0) / steps
        base = fields["f64"].cpu().numpy()
        for k in hs:
            out[k]["linf_vs_f64"].append(float(np.max(np.abs(fields[k].cpu().numpy() - base))))
    for k in hs:
        out[k]["ms_per_step"] = round(out[k]["ms_per_step"], 5)
        out[k]["updates_per_s"] = n * n / (out[k]["ms_per_step"] * 1e-3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-solves", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-refined", action="store_true")
    ap.add_argument("--no-precision", action="store_true")
    ap.add_argument("--only", choices=["solves", "per_system", "ensemble", "precision", "small",
                                       "tuning", "p2",
                                       "table31", "batch1d", "cook", "stencil", "cpu_all_cores"],
                    help="run only this side measurement and print its JSON")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into the traffic profile and exit")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="summarise a rocprofv3 --kernel-trace run into the kernel profile")
    ap.add_argument("--trace-note", default="",
                    help="text added to the kernel profile (--summarize-trace)")
    ap.add_argument("--summarize-leg", nargs=3, metavar=("TRACE_DIR", "OUT", "ONLY"),
                    help="summarise a rocprofv3 --kernel-trace run of `bench.py --only ONLY` "
                         "into the markdown file OUT and exit")
    ap.add_argument("--large-only", action="store_true",
                    help="only the large workload: no side measurements (profiling runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run the plain 1 GiB streaming copy three times (the "
                         "reference kernel for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.summarize_pmc:
        # the recorded commands name the trace directories given here
        cmd = ("timeout -s KILL 120 rocprofv3 --pmc {C} -d {D} -o run --output-format csv -- "
               "python3 bench.py --steps 3 --warmup 0 --no-cpu-baseline --large-only "
               "--calibrate-copy")
        print(json.dumps(summarize_pmc(*args.summarize_pmc, TRAFFIC_PROFILE, cmd)))
        return
    if args.summarize_leg:
        tdir, out, only = args.summarize_leg
        titles = {"solves": "batched cyclic penta solves, N = 1024, 131072 systems, interleaved "
                            "and contiguous, FP64",
                  "p2": "thesis delta-form scheme (P2), 1024 x 1024 and 8192 x 8192, FP64",
                  "cook": "Cahn-Hilliard-Cook forced step, 8192 x 8192, FP64",
                  "ensemble": "uneven ensemble of 256 runs (96 x 128^2, 96 x 256^2, 64 x 512^2): "
                              "FP64, forced, FP32-refined",
                  "per_system": "batched solves with one matrix per system, n = 1024, "
                                "65536 systems",
                  "batch1d": "batched 1D schemes (Cahn-Hilliard 2^20 x 256, hyperdiffusion "
                             "65536 x 1024)",
                  "stencil": "standalone 2D stencils on 8192 x 8192, FP64 and FP32",
                  "precision": "1024 x 1024 precision run (FP64, FP32-refined 1 and 2 passes, "
                               "10 x 1000 steps) and the standalone solves' precision"}
        cmd = ("rocprofv3 --kernel-trace --stats -d " + os.path.relpath(tdir) + " -o run "
               "--output-format csv -- python3 bench.py --only " + only)
        summarize_leg(tdir, out, titles.get(only, only), cmd, args.trace_note)
        return
    if args.summarize_trace:
        cmd = ("rocprofv3 --kernel-trace --stats -T -d " + os.path.relpath(args.summarize_trace) +
               " -o run --output-format csv -- python3 bench.py --no-cpu-baseline --large-only "
               "--calibrate-copy --steps 500 --warmup 10")
        print(json.dumps(summarize_trace(args.summarize_trace, KERNEL_PROFILE, cmd,
                                         args.trace_note)))
        return
    if args.only == "cpu_all_cores":  # host only: the oracle on every core
        print(json.dumps({"cpu_all_cores": cpu_all_cores()}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); ensembles would "
              "shard by runs and a large grid by row slabs; only one GPU is measured.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2101_06550_amd import chx, inputs
    if not os.path.exists(chx.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    chx.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.only:
        fn = {"solves": solve_throughput, "per_system": per_system_throughput,
              "ensemble": ensemble_throughput,
              "small": small_run, "tuning": tuning_sweep, "p2": p2_run,
              "table31": table31_run, "batch1d": batch1d_run, "cook": cook_run,
              "stencil": stencil_throughput,
              "precision": lambda c, t: {
                  "solves": solve_precision(c, t), "run_1024": precision_run(c, t)}}[args.only]
        print(json.dumps({args.only: fn(chx, torch)}), flush=True)
        return
    L = 2 * math.pi
    n, D, gamma, dt = args.n, 1.0, 0.001, 1e-6
    log(f"building initial state {n}x{n}")
    c0 = inputs.mode_plus_noise(n, 5)
    h = chx.ch_create(n, n, L, L, D, gamma, dt)  # factors and autotunes
    if args.calibrate_copy:  # after creation: also marks where the workload starts
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            chx.chx_stream_copy(src, dst)  # reads 1 GiB, writes 1 GiB
        torch.cuda.synchronize()
        del src, dst
    c = torch.tensor(c0, device="cuda")
    K, W = args.steps, args.warmup
    diag = torch.zeros(2 * (K + 1), dtype=torch.float64, device="cuda")
    # after the host work above (the initial state, the factorisation) the
    # idle GPU has dropped to a low-power state, and it takes some 50 ms of
    # sustained load to return: measured, 20 steps right after 50 ms of host
    # idle run at 0.51 ms/step against 0.45 once loaded.  A plain streaming
    # copy (no step kernel, nothing of the workload) keeps the GPU loaded for
    # settle_ms before the warmup steps, so that the timed steps see the
    # sustained clocks a long run sees; the cost of starting from idle is
    # measured separately below
    settle_ms = settle_clocks(chx, torch, 150.0)
    if W > 0:
        log(f"warmup {W} steps")
        cw = c.clone()
        chx.ch_adi_step(h, cw, nsteps=W, diag_out=torch.zeros(2 * (W + 1), dtype=torch.float64,
                                                              device="cuda"))
        torch.cuda.synchronize()
        del cw
    # the timed region: K plain steps in one call (no instrumentation), the
    # host clock around it with the device synchronised on both sides
    log(f"timing {K} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    chx.ch_adi_step(h, c, nsteps=K, diag_out=diag)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # then the same K steps again from the same initial state, with HIP events
    # recorded on the library's stream around every kernel of every step
    # (events created before the call): the per-kernel durations of the
    # roofline; this pass is reported beside the headline, not as it
    log(f"per-kernel event timing of the same {K} steps")
    ct = torch.tensor(c0, device="cuda")
    dt_ = torch.zeros_like(diag)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    phase_ms, phase_n = chx.ch_adi_step_timed(h, ct, nsteps=K, diag_out=dt_, sample_every=1)
    torch.cuda.synchronize()
    el_timed = time.perf_counter() - t1
    timed_same = bool(torch.equal(ct, c)) and bool(torch.equal(dt_, diag))
    del ct, dt_
    # the same K steps started after 0.2 s of host idle, without settling
    # (not in profiling runs, whose traces cover the timed workload)
    el_idle = None
    if not args.large_only:
        log(f"the same {K} steps after host idle")
        ci = torch.tensor(c0, device="cuda")
        di = torch.zeros_like(diag)
        torch.cuda.synchronize()
        time.sleep(0.2)
        t2 = time.perf_counter()
        chx.ch_adi_step(h, ci, nsteps=K, diag_out=di)
        torch.cuda.synchronize()
        el_idle = time.perf_counter() - t2
        del ci, di
    d = diag.cpu().numpy()
    mass, energy = d[0::2], d[1::2]
    l1 = float(np.sum(np.abs(c0))) * (L / n) ** 2
    mass_drift = float(np.max(np.abs(mass - mass[0])) / l1)
    energy_monotone = bool(np.all(np.diff(energy) <= 1e-12 * np.abs(energy[:-1])))

    split = chx.ch_get_tuning(h, chx.CHX_TUNE_ROW_SPLIT)
    if split >= 0:  # separators fused with the interior rows, then the separator rows
        names = ["column_pass", "separator_rows", "separators_and_interior_rows",
                 "finalize_and_diag"]
        sep_rows = row_pass_bytes(n, n) * 2 // CHUNK
        bytes_per = [column_pass_bytes(n, n), sep_rows,
                     row_pass_bytes(n, n) - sep_rows + reduced_bytes(n, n), None]
    else:
        names = ["column_pass", "column_separators", "row_pass", "finalize_and_diag"]
        mcol = chx.ch_get_tuning(h, chx.CHX_TUNE_COLUMN_CHUNK)
        bytes_per = [column_pass_bytes(n, n, mcol), reduced_bytes(n, n, mcol),
                     row_pass_bytes(n, n), None]
    phases = {}
    for k, nm in enumerate(names):
        if phase_n[k] == 0:
            continue
        avg = phase_ms[k] / phase_n[k]
        ent = {"launches": phase_n[k], "avg_ms": round(avg, 5), "total_ms": round(phase_ms[k], 3)}
        if bytes_per[k]:
            ent["algorithmic_bytes"] = bytes_per[k]
            ent["achieved_GBps"] = round(bytes_per[k] / (avg * 1e-3) / 1e9, 1)
        phases[nm] = ent
    dom = max((k for k in range(3) if phase_n[k]), key=lambda k: phase_ms[k])
    dom_avg = phase_ms[dom] / phase_n[dom]
    achieved = bytes_per[dom] / (dom_avg * 1e-3) / 1e9
    kernel_of = dict(KERNEL_OF_PHASE)
    if chx.ch_get_tuning(h) >= FIRST_WHOLE_COLUMN_SHAPE:
        kernel_of["column_separators"] = "reduced_whole"
    traffic = stored_traffic(kernel_of[names[dom]])
    roofline = {"bound": "hbm", "kernel": kernel_of[names[dom]],
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic)}

    extra = {}
    if args.large_only:
        args.no_solves = args.no_ensemble = args.no_precision = args.no_refined = True
    else:
        extra["hbm_copy_reference_1GiB"] = copy_reference(chx, torch)
        log("small 128^2 run")
        extra["small_128_1000_steps"] = small_run(chx, torch)
        log("thesis delta-form scheme")
        extra["thesis_scheme_p2"] = p2_run(chx, torch)
        log("batched 1D schemes")
        extra["batched_1d"] = batch1d_run(chx, torch)
        log("Cahn-Hilliard-Cook forcing")
        extra["cook_forced_8192"] = cook_run(chx, torch)
        log("standalone 2D stencils")
        extra["stencil_8192"] = stencil_throughput(chx, torch)
    if not args.no_solves:
        log("standalone batched solves")
        extra["penta_solve_N1024_batch131072"] = solve_throughput(chx, torch)
        log("batched solves with one matrix per system")
        extra["per_system_N1024_batch65536"] = per_system_throughput(chx, torch)

    if not args.no_ensemble:
        log("uneven ensemble")
        extra["ensemble_256_runs_fp64"] = ensemble_throughput(chx, torch)

    if not args.no_precision:
        log("FP64 vs FP32-refined: batched solves")
        extra["solves_N1024_batch1024_f64_vs_f32_refined"] = solve_precision(chx, torch)
        log("FP64 vs FP32-refined: 1024^2 precision run")
        extra["precision_run_1024"] = precision_run(chx, torch)

    hr = None
    if not args.no_refined:
        # the large workload with the FP32-sweep refined path (3 passes)
        log("large workload, FP32-refined (3 passes)")
        hr = chx.ch_create(n, n, L, L, D, gamma, dt, dtype=chx.CHX_F32_REFINED, refine_passes=3)
        cr = torch.tensor(c0, device="cuda")
        chx.ch_adi_step(hr, cr, nsteps=2)
        torch.cuda.synchronize()
        kr = max(1, min(K, 50))
        t0 = time.perf_counter()
        chx.ch_adi_step(hr, cr, nsteps=kr)
        torch.cuda.synchronize()
        elr = time.perf_counter() - t0
        rb = refined_bytes_per_point(3, kr)
        gbps = rb * n * n * kr / elr / 1e9
        extra["large_f32_refined_3pass"] = {"steps": kr, "ms_per_step": round(1e3 * elr / kr, 5),
                                            "updates_per_s": n * n * kr / elr,
                                            "algorithmic_bytes_per_point": round(rb, 2),
                                            "algorithmic_GBps": round(gbps, 1),
                                            "frac_of_hbm_peak": round(gbps / HBM_PEAK_GBS, 4)}
        del cr

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle CPU baseline")
        cpu, first = cpu_baseline(c0, L, D, gamma, dt)
        errs = {}
        for tag, h_ in (("f64", h), ("f32_refined_3pass", hr)):
            if h_ is None:
                continue
            probe = torch.tensor(c0, device="cuda")
            chx.ch_adi_step(h_, probe, nsteps=1)
            torch.cuda.synchronize()
            errs[tag] = rel_inf(probe.cpu().numpy(), first)
            del probe
        extra["large_one_step_rel_err_vs_oracle"] = errs
        log("oracle on all host cores (ensemble runs, batched solves)")
        allc = cpu_all_cores()
        ens = extra.get("ensemble_256_runs_fp64", {}).get("graph")
        if ens:
            allc["ensemble"]["gpu_fp64_over_oracle_all_cores"] = round(
                ens["updates_per_s"] / allc["ensemble"]["value"], 1)
        extra["oracle_all_cores"] = allc

    res = {
        "metric": METRIC,
        "value": n * n * K / el,
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1e3 * el / K, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"large single run: {n}x{n} periodic Cahn-Hilliard ADI on "
                               f"(0,2pi)^2, D=1, gamma=0.001, dt=1e-6, c0=0.05 sin3x sin5y + "
                               f"U[-0.01,0.01] (seed 5), FP64, mass+energy every step",
                   "nx": n, "ny": n, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "instrumented_pass": {"ms_per_step": round(1e3 * el_timed / K, 5),
                              "bitwise_equal_to_timed_run": timed_same},
        "clock_settle": {"copy_ms_before_warmup": round(settle_ms, 1),
                         "ms_per_step_after_0.2s_host_idle":
                             round(1e3 * el_idle / K, 5) if el_idle else None},
        "tuning": {"separator_kernel_shape": chx.ch_get_tuning(h),
                   "row_split_shape": split,
                   "single_workgroup_path": chx.ch_get_tuning(h, chx.CHX_TUNE_SMALL_PATH),
                   "column_tile_order": chx.ch_get_tuning(h, chx.CHX_TUNE_COLUMN_ORDER),
                   "column_chunk": chx.ch_get_tuning(h, chx.CHX_TUNE_COLUMN_CHUNK),
                   "row_chunk": chx.ch_get_tuning(h, chx.CHX_TUNE_ROW_CHUNK)},
        "checks": {"mass_drift_rel_L1": mass_drift, "energy_monotone": energy_monotone},
        "extra": extra,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
