"""Benchmark of the one-pass quaternion low-rank approximation on one MI355X.

Workload (default): A in Q^{20000 x 15000}, four FP32 planes (4.8 GB), rank-50
quaternion factors with sigma_i = i^-2 plus 1e-4 relative Gaussian noise,
streamed once in column blocks of 2048, Gaussian test matrices, k = 100,
l = 201, both rangefinders.  Inputs are synthetic and resident in HBM before
timing starts.

One step = one whole one-pass approximation: reset, all column-block updates
of the sketches, then the QB stages with pseudo-QR and with pseudo-SVD, side
by side on two streams (each path also reports the QB stage alone, paired and
one rangefinder after the other, under `qb_stage`).  Paths:
  fp64   FP64 sketch on the GPU (the FP64 plain method; error reference, not timed)
  fp32   FP32 sketch on the matrix cores (the same-GPU FP32 plain path)
  bf16   BF16 sketch with the data split in `--terms` bf16 terms (timed: `value`)

The default run also measures the other workloads, reported in the same
JSON line under `workloads`:
  image    31365 x 27125 pure quaternion in BF16 (5.1 GB), quaternion
           Rademacher test matrices, k = 200, l = 401, BF16 operands (exact:
           one term), column blocks of 2048, both rangefinders
  batch64  64 independent FP32 problems (m 512-8192, n 256-4096 log-uniform,
           k = 2r, l = 2k + 1), BF16 two-term operands, autotuned tiles
  flow     2,097,152 x 300 pure quaternion FP32 snapshot matrix (7.55 GB),
           streamed as 30 linear updates of 10 columns, e4m3 operands with
           per-tile scales plus the residual terms, Gaussian, k = 60, l = 121
each with its wall time, algorithmic sketch TFLOP/s, the roofline fraction of
its dominant kernel and the relative-error difference against the same
GPU's FP64 path.

Prints one JSON line.  `value` = algorithmic sketch TFLOP/s of the bf16 path
on the 20000 x 15000 workload (2 * 16 * m * n * (k + l) flops over the time of
its updates).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_2404_14783_amd as qs  # noqa: E402
import synth  # noqa: E402

PEAK_BF16 = 2.5e15     # dense bf16 MFMA, MI355X
PEAK_F32 = 157.3e12    # fp32 MFMA
PEAK_FP8 = 5.0e15      # dense fp8 MFMA
PEAK_HBM = 8e12
CALIB_BYTES = 256 << 20                    # the plain copy used to scale the HBM counters
KERNEL_SRC = os.path.join(ROOT, "paper_2404_14783_amd", "csrc", "sketch_mfma.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "w_mfma_c2_bf16x2_traffic.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sketch_flops(m, n, k, l, pure=False):
    return 2.0 * (12 if pure else 16) * m * n * (k + l)


def run_pass(sk, a, block, kinds=("pseudo_qr", "pseudo_svd")):
    """One whole one-pass approximation; returns (update_ms, total_ms, results).
    Two rangefinders run their QB stages side by side (qsketch_finalize_pair)."""
    st = torch.cuda.current_stream()
    sk.reset()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(st)
    n = a.shape[2]
    for c0 in range(0, n, block):
        sk.update(c0, a[:, :, c0:c0 + block])
    e1.record(st)
    if len(kinds) == 2:
        res = dict(zip(kinds, sk.finalize_pair(kinds)))
    else:
        res = {kind: sk.finalize(kind) for kind in kinds}
    e2.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), e0.elapsed_time(e2), res


def qb_stage_times(sk, reps=3, kinds=("pseudo_qr", "pseudo_svd")):
    """Median time of the QB stage alone on the current sketches: the two
    rangefinders side by side (qsketch_finalize_pair) and one after the other
    (two qsketch_finalize calls)."""
    st = torch.cuda.current_stream()
    out = {}
    for name, fn in (("pair", lambda: sk.finalize_pair(kinds)),
                     ("sequential", lambda: [sk.finalize(kd) for kd in kinds])):
        fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            fn()
            e1.record(st)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        out[name + "_ms"] = float(np.median(ts))
    return out


def cpu_threads():
    """Threads the oracle's BLAS actually uses (threadpoolctl when present)."""
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads") for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count()


def cpu_baseline(a_dev, m, n, k, l, block, seconds=20.0):
    """The oracle timed on the host cores on a bounded sample of the same
    workload: its FP64 sketch update over the first column blocks, until
    about `seconds`, then its QB stage (both rangefinders and the core solve)
    on that sketch, timed separately."""
    from oracle import onepass
    from oracle.sketch import Sketch, SketchConfig
    sk = Sketch(SketchConfig(m, n, k, l, seed=0))
    t0 = time.perf_counter()
    sk.psi()                                            # Psi generation counted
    cols = 0
    c0 = 0
    sample_block = min(block, 512)
    while c0 < n and time.perf_counter() - t0 < seconds:
        blk = a_dev[:, :, c0:c0 + sample_block].double().cpu().numpy()
        sk.update(c0, blk)
        cols += blk.shape[2]
        c0 += sample_block
    dt = time.perf_counter() - t0
    flops = sketch_flops(m, cols, k, l)
    fin = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        t1 = time.perf_counter()
        onepass.qb_stage(sk, kind)
        fin[kind] = time.perf_counter() - t1
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": cpu_threads(),
            "kind": "oracle", "sketch_s": dt, "sketch_columns": cols,
            "finalize_s": fin, "host_cpus": os.cpu_count(),
            "sample": f"FP64 NumPy sketch update of the first {cols} of {n} columns "
                      f"(m={m}, k={k}, l={l}, Gaussian, Psi generation included), {dt:.1f} s; "
                      f"then the QB stage on that sketch (Y {m}x{k}, W {l}x{n}): pseudo-QR "
                      f"{fin['pseudo_qr']:.2f} s, pseudo-SVD {fin['pseudo_svd']:.2f} s"}


def source_digest():
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _pmc_rows(directory):
    files = glob.glob(os.path.join(directory, "**", "*counter_collection*.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection csv under {directory}")
    with open(files[0]) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter):
    """{dispatch id: (kernel name, value)} for one counter (values summed over
    the rows of a dispatch)."""
    out = {}
    for r in rows:
        if r.get("Counter_Name") != counter:
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        name, val = out.get(d, (r.get("Kernel_Name", ""), 0.0))
        out[d] = (name, val + float(r["Counter_Value"]))
    return out


def summarize_traffic(fetch_dir, write_dir, cmd_fetch, cmd_write):
    """Per-launch HBM traffic of the W kernel from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
    same counter reads for the plain copy of CALIB_BYTES."""
    fetch = _per_dispatch(_pmc_rows(fetch_dir), "FETCH_SIZE")
    write = _per_dispatch(_pmc_rows(write_dir), "WRITE_SIZE")

    def pick(tab, key):
        return [v for (n, v) in tab.values() if key in n]
    cf = max(pick(fetch, "copyBuffer")) * 1024.0
    cw = max(pick(write, "copyBuffer")) * 1024.0
    ff, fw = CALIB_BYTES / cf, CALIB_BYTES / cw
    wf = pick(fetch, "w_mfma_kernel")
    ww = pick(write, "w_mfma_kernel")
    f_avg = float(np.mean(wf)) * 1024.0 * ff
    w_avg = float(np.mean(ww)) * 1024.0 * fw
    lines = [
        "# HBM traffic of w_mfma_kernel: 20000x15000 FP32 quaternion, BF16 2-term sketch, k=100, l=201",
        "",
        "Two counter passes over the same program (from the repository root, on one MI355X):",
        "",
        f"    {cmd_fetch}",
        f"    {cmd_write}",
        "",
        f"Calibration: a plain copy of {CALIB_BYTES} bytes reads FETCH_SIZE = {cf / 1024:.0f} KiB and "
        f"WRITE_SIZE = {cw / 1024:.0f} KiB (scale factors {ff:.4f}, {fw:.4f}).",
        "",
        "| quantity | value |",
        "|---|---:|",
        f"| W-kernel dispatches | {len(wf)} |",
        f"| FETCH_SIZE per launch (KiB, raw) | {np.mean(wf):.0f} |",
        f"| WRITE_SIZE per launch (KiB, raw) | {np.mean(ww):.0f} |",
        f"| fetched bytes per launch (scaled) | {f_avg:.4e} |",
        f"| written bytes per launch (scaled) | {w_avg:.4e} |",
        "",
        f"traffic_bytes_per_launch: {f_avg + w_avg:.6e}",
        f"kernel_source_sha256_16: {source_digest()}",
        "",
    ]
    with open(TRAFFIC_FILE, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


STATS_TITLES = {
    "c2": ("20000x15000 FP32 quaternion, BF16 (2-term) sketch, both rangefinders",
           "The bench line's own run of this workload (FP32, BF16 two-term and FP8 paths, one warm-up and "
           "three timed one-pass approximations each: 8 column-block updates of 2048 columns, then the QB "
           "stages with pseudo-QR and with pseudo-SVD side by side; the FP64 reference, the CPU baseline and the extras "
           "left out); input generation kernels are listed too."),
    "image": ("31365x27125 pure quaternion BF16 image, Rademacher, k=200, l=401, BF16 operands, both rangefinders",
              "Whole one-pass approximations (14 column-block updates of 2048 columns, then the QB stages with "
              "pseudo-QR and with pseudo-SVD side by side); input generation kernels are listed too."),
    "flow": ("2097152x300 pure quaternion FP32 flow snapshots, 30 updates of 10 columns gathered into "
             "blocks of up to 256 (250 and 50), 3 e4m3 terms on the fp8 matrix cores, k=60, l=121, both rangefinders",
             "Whole one-pass approximations (30 linear updates of 10 columns, gathered into two products, "
             "then the QB stages with pseudo-QR and with pseudo-SVD side by side); input generation kernels are listed too."),
    "batch64": ("64 FP32 quaternion problems, BF16 two-term operands, autotuned tiles",
                "Batched runs (autotuning, then runs with pseudo-QR and with pseudo-SVD); input generation "
                "kernels are listed too."),
}


def summarize_stats(directory, cmd, out_path, workload="c2"):
    """Short kernel-time table from a rocprofv3 --kernel-trace --stats run."""
    files = glob.glob(os.path.join(directory, "**", "*kernel_stats.csv"), recursive=True)
    rows = list(csv.DictReader(open(files[0])))
    title, what = STATS_TITLES[workload]
    lines = [
        f"# Kernel time summary: {title}",
        "",
        "Command (from the repository root, on one MI355X):",
        "",
        f"    {cmd}",
        "",
        what,
        "",
        "| total ms | calls | avg us | kernel |",
        "|---:|---:|---:|---|",
    ]
    for r in rows:
        name = r["Name"].replace("|", "/")
        if len(name) > 110:
            name = name[:110]
        lines.append(f"| {float(r['TotalDurationNs']) / 1e6:.3f} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | `{name}` |")
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines[:30]))


BUSY_COUNTERS = ("SQ_WAVES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_MFMA "
                 "SQ_INSTS_VALU SQ_WAIT_ANY SQ_INSTS_LDS")


def summarize_busy(directory, cmd, out_path, workload="c2"):
    """Matrix-core busy fraction per library kernel from one rocprofv3 --pmc
    pass over BUSY_COUNTERS: SQ_VALU_MFMA_BUSY_CYCLES over (1024 SIMDs x the
    dispatch's duration x 2.4 GHz), averaged over the dispatches."""
    rows = _pmc_rows(directory)
    per = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if not name.startswith(("qsk::", "void qsk::")):
            continue
        d = r.get("Dispatch_Id") or r.get("Correlation_Id")
        rec = per.setdefault(name, {}).setdefault(d, {"dur": (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9})
        rec[r["Counter_Name"]] = rec.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    title, _ = STATS_TITLES[workload]
    lines = [
        f"# Matrix-core busy time: {title}",
        "",
        "One counter pass (from the repository root, on one MI355X):",
        "",
        f"    {cmd}",
        "",
        "busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x duration x 2.4 GHz): the fraction of the",
        "kernel's time the matrix cores of the whole chip were busy (duration from the dispatch",
        "timestamps of the counter pass).  Per dispatch averages, library kernels of 40 us or more.",
        "",
        "| kernel | dispatches | avg us | MFMA instr | MFMA busy | VALU instr | LDS instr |",
        "|---|---:|---:|---:|---:|---:|---:|",
    ]
    out = []
    for name, ds in per.items():
        recs = list(ds.values())
        dur = float(np.mean([x["dur"] for x in recs]))
        if dur < 40e-6:
            continue
        busy = float(np.mean([x.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (1024 * x["dur"] * 2.4e9) for x in recs]))
        mean = lambda c: float(np.mean([x.get(c, 0.0) for x in recs]))
        out.append((dur * len(recs), f"| `{name.replace('|', '/')[:100]}` | {len(recs)} | {dur * 1e6:.1f} | "
                    f"{mean('SQ_INSTS_MFMA'):.3g} | {busy:.2f} | {mean('SQ_INSTS_VALU'):.3g} | "
                    f"{mean('SQ_INSTS_LDS'):.3g} |"))
    lines += [s for _, s in sorted(out, reverse=True)]
    with open(out_path, "w") as f:
        f.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def committed_traffic():
    """Per-launch HBM bytes of the W kernel from the committed counter
    summary, or None when the kernel source changed since it was taken."""
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in text.splitlines()
                if line.startswith(("traffic_bytes_per_launch:", "kernel_source_sha256_16:")))
    if vals.get("kernel_source_sha256_16", "").strip() != source_digest():
        return None
    return float(vals["traffic_bytes_per_launch"])


METRIC = "one-pass qLRA wall time + sketch TFLOP/s at equal rel. error, BF16/FP8 vs FP32"


def bench_batch(args, profile_only=False):
    """64 independent problems (m in [512, 8192], n in [256, 4096] log-uniform,
    rank 8..64 with geometric decay, k = 2r, l = 2k + 1, FP32 data, 1e-4
    noise) through the batched path: one run = both sketches of every
    problem and the QB stage with one rangefinder, all problems together.
    Returns the workload's record."""
    specs = synth.batch_specs(64)
    mats = [qs.to_colmajor(synth.batch_matrix(sp, i, device="cuda")) for i, sp in enumerate(specs)]
    shapes = [(sp["m"], sp["n"], sp["k"], sp["l"], i) for i, sp in enumerate(specs)]
    torch.cuda.synchronize()
    flops = sum(sketch_flops(m, n, k, l) for (m, n, k, l, _) in shapes)
    if profile_only:
        b = qs.Batch(shapes, input_dtype="f32", sketch_dtype="bf16", split_terms=args.batch_terms)
        b.autotune(mats)
        outs = b.outputs()
        for kind in ("pseudo_qr", "pseudo_svd"):
            for _ in range(max(1, args.steps)):
                b.run(mats, kind, outputs=outs)
        torch.cuda.synchronize()
        b.close()
        return {"profile_only": True, "workload": "batch64"}
    out = {}
    errs = {}
    tiles = {}
    for name, sketch, terms in (("fp32", "f32", 1), ("bf16", "bf16", args.batch_terms)):
        b = qs.Batch(shapes, input_dtype="f32", sketch_dtype=sketch, split_terms=terms)
        tiles[name] = b.autotune(mats)
        outs = b.outputs()
        st = torch.cuda.current_stream()
        for kind in ("pseudo_qr", "pseudo_svd"):
            for _ in range(args.warmup):
                b.run(mats, kind, outputs=outs)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(st)
            for _ in range(args.steps):
                b.run(mats, kind, outputs=outs)
            e1.record(st)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            errs[(name, kind)] = b.rel_error(mats, *outs)
            out[f"{name}_{kind}_ms"] = ms
            log(f"[bench] batch {name} {kind}: {ms:.2f} ms per run")
        b.close()
    # the GPU FP64 path for every problem, with the bf16-rounded test
    # matrices of the BF16 path: the equal-error reference
    worst = 0.0
    for i in range(len(shapes)):
        m, n, k, l, seed = shapes[i]
        sk = qs.Sketcher(m, n, k, l, seed=seed, input_dtype="f32", sketch_dtype="f64", max_block_cols=n,
                         embedding_round="bf16")
        sk.update(0, mats[i])
        for kind in ("pseudo_qr", "pseudo_svd"):
            q, x, _ = sk.finalize(kind)
            ref = sk.rel_error(mats[i], q, x)
            worst = max(worst, abs(errs[("bf16", kind)][i] - ref) / ref)
            del q, x
        sk.close()
    step_ms = out["bf16_pseudo_qr_ms"] + out["bf16_pseudo_svd_ms"]
    fp32_ms = out["fp32_pseudo_qr_ms"] + out["fp32_pseudo_svd_ms"]
    ach = 2 * flops / (step_ms * 1e-3)
    return {
        "workload": f"batch of 64 FP32 quaternion problems, m 512-8192, n 256-4096, k = 2r (r 8-64), "
                    f"l = 2k + 1, Gaussian, BF16 operands ({args.batch_terms} terms); step = one batched run "
                    f"with pseudo-QR plus one with pseudo-SVD (sketches recomputed in each)",
        "problems": len(shapes), "sketch_flops_per_run": flops, "bf16_terms": args.batch_terms,
        "total_entries": int(sum(m * n for (m, n, _, _, _) in shapes)),
        "ms_per_step": step_ms, "sketch_tflops_whole_run": ach / 1e12,
        "paths": out, "speedup_vs_fp32_wall": fp32_ms / step_ms,
        "autotuned_tiles": {k: {"w_row_tiles": v[0], "y_col_tiles": v[1], "w_blocks": v[2]}
                            for k, v in tiles.items()},
        "equal_error": {"max_rel_diff_bf16_vs_fp64": worst, "problems_checked": len(shapes)},
        "roofline": {"bound": "mfma", "kernel": "whole batched run (sketches and QB stage)",
                     "achieved": ach / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                     "frac": ach / PEAK_BF16},
    }


def timed_passes(sk, a, block, args, kinds=("pseudo_qr", "pseudo_svd")):
    """W untimed and K timed whole passes with per-kernel timing; returns
    (median update ms, median pass ms, results of the last pass, timing)."""
    for _ in range(args.warmup):
        run_pass(sk, a, block, kinds)
    sk.set_timing(True)
    ups, tots = [], []
    torch.cuda.synchronize()
    for _ in range(args.steps):
        up, tot, res = run_pass(sk, a, block, kinds)
        ups.append(up)
        tots.append(tot)
    timing = sk.timing()
    sk.set_timing(False)
    return float(np.median(ups)), float(np.median(tots)), res, timing


def kernel_rooflines(timing, m, n, k, l, pure, steps, peak, y_bytes_per_update=None, updates=None):
    """Achieved rate of the two product kernels over the timed passes: the
    algorithmic flops of all their launches (2 P m n k for Y, 2 P m n l for W,
    P = 12 for pure input, else 16) over the summed HIP-event durations of
    the launches; for a streamed workload also the Y kernel's algorithmic
    HBM bytes (A's block plus the read-modify-write of Y) per second."""
    P = 12 if pure else 16
    out = {}
    for name, kk in (("w", l), ("y", k)):
        ms, cnt = timing[name]
        fl = 2.0 * P * m * n * kk * steps
        ach = fl / (ms * 1e-3) if ms > 0 else 0.0
        out[name] = {"achieved_tflops": ach / 1e12, "frac": ach / peak, "launches": cnt,
                     "avg_launch_ms": ms / max(cnt, 1)}
    if y_bytes_per_update is not None:
        ms, cnt = timing["y"]
        by = y_bytes_per_update * updates * steps
        out["y"]["achieved_gbs"] = by / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        out["y"]["hbm_frac"] = by / (ms * 1e-3) / PEAK_HBM if ms > 0 else 0.0
    return out


EMB_ROUND = {"fp32": "f32", "f32": "f32", "bf16": "bf16", "fp8": "fp8", "fp8x": "fp8"}


def fp64_reference(a, m, n, k, l, block, emb, input_dtype, pure, rnd):
    """Relative errors of the GPU FP64 path (both rangefinders) with the
    test matrices rounded to `rnd` as the low-precision path uses them: the
    equal-error reference.  The FP64 result does not depend on the column
    blocking (linear updates), so it streams in blocks of `block`."""
    sk = qs.Sketcher(m, n, k, l, seed=0, embedding=emb, input_dtype=input_dtype, sketch_dtype="f64",
                     pure=pure, max_block_cols=block, embedding_round=rnd)
    up, tot, r = run_pass(sk, a, block)
    errs = {kind: sk.rel_error(a, q, x) for kind, (q, x, rep) in r.items()}
    sk.close()
    return errs, {"update_ms": up, "total_ms": tot, "embedding_round": rnd}


def bench_stream_leg(args, label, a, m, n, k, l, block, emb, input_dtype, pure, paths, peak,
                     ref_block=None):
    """One streamed workload: each low-precision path timed, and the GPU FP64
    path (untimed) with the same rounded test matrices as the reference of
    its equal-error comparison; returns the workload's record."""
    res = {}
    errors = {}
    flops = sketch_flops(m, n, k, l, pure)
    refs = {}
    for path in paths:
        name, sketch, terms = path[:3]
        coalesce = path[3] if len(path) > 3 else 0
        rnd = "f64" if emb == "rademacher" else EMB_ROUND[sketch]    # +-1 is exact in every format
        if rnd not in refs:
            log(f"[bench] {label}: FP64 reference pass, test matrices rounded to {rnd} (untimed)")
            refs[rnd] = fp64_reference(a, m, n, k, l, ref_block or block, emb, input_dtype, pure, rnd)
        res["fp64_" + rnd] = refs[rnd][1]
        sk = qs.Sketcher(m, n, k, l, seed=0, embedding=emb, input_dtype=input_dtype, sketch_dtype=sketch,
                         split_terms=terms, pure=pure, max_block_cols=block, coalesce_cols=coalesce)
        up, tot, r, timing = timed_passes(sk, a, block, args)
        rec = {"update_ms": up, "total_ms": tot, "sketch_tflops": flops / (up * 1e-3) / 1e12,
               "terms": terms, "coalesce_cols": coalesce,
               "kernels_ms": {kk: v[0] / args.steps for kk, v in timing.items()}}
        for kind, (q, x, rep) in r.items():
            errors[(name, kind)] = sk.rel_error(a, q, x)
            rec[kind + "_kappa"] = rep["kappa"]
        rec["qb_stage"] = qb_stage_times(sk)
        eff = (coalesce // block) * block if coalesce else block      # columns per sketch product
        nupd = (n + eff - 1) // eff
        ybytes = None
        if eff < 64:
            # streamed in thin blocks: Y's read-modify-write dominates the traffic
            ybytes = (3 if pure else 4) * m * (n / nupd) * (4 if input_dtype == "f32" else 2) + 2 * 4 * m * k * 4
        rec["kernels"] = kernel_rooflines(timing, m, n, k, l, pure, args.steps,
                                          PEAK_FP8 if sketch == "fp8x" else peak, ybytes, nupd)
        rec["peak_tflops"] = (PEAK_FP8 if sketch == "fp8x" else peak) / 1e12
        if sketch == "fp8x" and timing.get("stage", (0.0, 0))[0] > 0:
            # the e4m3 term split: reads the block once, writes T bytes per
            # value in each of its two layouts (algorithmic bytes, no padding)
            planes = 3 if pure else 4
            qbytes = m * n * planes * ((4 if input_dtype == "f32" else 2) + 2 * terms) * args.steps
            qs_ms = timing["stage"][0]
            rec["kernels"]["quant"] = {"bytes_per_pass": qbytes / args.steps,
                                       "achieved_gbs": qbytes / (qs_ms * 1e-3) / 1e9,
                                       "hbm_frac": qbytes / (qs_ms * 1e-3) / PEAK_HBM,
                                       "launches": timing["stage"][1]}
        res[name] = rec
        log(f"[bench] {label} {name}: updates {up:.2f} ms, step {tot:.2f} ms, "
            f"{rec['sketch_tflops']:.1f} TFLOP/s, kernels {rec['kernels']}")
        sk.close()
        del r
    eq = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        eq[kind] = {}
        for path in paths:
            name = path[0]
            rnd = "f64" if emb == "rademacher" else EMB_ROUND[path[1]]
            ref = refs[rnd][0][kind]
            e = errors[(name, kind)]
            eq[kind]["e_fp64_" + rnd] = ref
            eq[kind]["e_" + name] = e
            eq[kind]["rel_diff_" + name] = abs(e - ref) / ref if ref else None
    return {"paths": res, "equal_error": eq, "sketch_flops": flops}


def bench_image(args, profile_only=False):
    """The 31365 x 27125 pure-quaternion BF16 image, Rademacher, k = 200,
    l = 401, BF16 operands (exact in one term)."""
    m, n, k, l, block = 31365, 27125, 200, 401, 2048
    log(f"[bench] image: generating {m}x{n} (3 BF16 planes) on the GPU")
    a = qs.to_colmajor(synth.image_planes(m, n, device="cuda", dtype=torch.bfloat16))
    torch.cuda.synchronize()
    if profile_only:
        sk = qs.Sketcher(m, n, k, l, seed=0, embedding="rademacher", input_dtype="bf16",
                         sketch_dtype="bf16", pure=True, max_block_cols=block)
        for _ in range(max(1, args.steps)):
            up, tot, _ = run_pass(sk, a, block)
            log(f"[bench] image bf16 pass: updates {up:.2f} ms, total {tot:.2f} ms")
        sk.close()
        return {"profile_only": True, "workload": "image", "update_ms": up, "total_ms": tot}
    leg = bench_stream_leg(args, "image", a, m, n, k, l, block, "rademacher", "bf16", True,
                           [("bf16", "bf16", 1)], PEAK_BF16)
    del a
    torch.cuda.empty_cache()
    bf = leg["paths"]["bf16"]
    w = bf["kernels"]["w"]
    leg.update({
        "workload": f"{m}x{n} pure quaternion image in BF16, column blocks of {block}, Rademacher "
                    f"k={k} l={l}, BF16 operands (one term), both rangefinders",
        "ms_per_step": bf["total_ms"], "sketch_tflops": bf["sketch_tflops"],
        "roofline": {"bound": "mfma", "kernel": "w_mfma_kernel (bf16, 1 term, pure)",
                     "achieved": w["achieved_tflops"], "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                     "frac": w["frac"], "avg_launch_ms": w["avg_launch_ms"],
                     "y_kernel_frac": bf["kernels"]["y"]["frac"]},
    })
    return leg


def graph_saving(args, a, m, n, k, l, block, sketch, terms, coalesce):
    """The stream of column-block updates issued one call per block and as
    one replayed HIP graph (qsketch_update_many): median update-phase times
    over the timed passes, and whether the two give bit-identical sketches."""
    sk = qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32", sketch_dtype=sketch,
                     split_terms=terms, pure=True, max_block_cols=block, coalesce_cols=coalesce)
    cols = list(range(0, n, block))
    blocks = [a[:, :, c0:c0 + block] for c0 in cols]
    st = torch.cuda.current_stream()

    def once(graph):
        sk.reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        if graph:
            sk.update_many(cols, blocks)
        else:
            for c0, b in zip(cols, blocks):
                sk.update(c0, b)
        sk.sketches()                                  # runs the pending gathered columns
        e1.record(st)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    out = {}
    for graph in (False, True):
        for _ in range(max(1, args.warmup)):
            once(graph)
        out["graph_ms" if graph else "eager_ms"] = float(np.median([once(graph) for _ in range(args.steps)]))
        ys = [t.clone() for t in sk.sketches()]
        if graph:
            out["bit_identical"] = bool(all(torch.equal(u, v) for u, v in zip(ys, prev)))
        prev = ys
    sk.close()
    out.update({"updates": len(cols), "coalesce_cols": coalesce,
                "saving_ms": out["eager_ms"] - out["graph_ms"]})
    return out


def bench_flow(args, profile_only=False):
    """The 128^3 x 300 pure-quaternion FP32 flow snapshots, 30 linear updates
    of 10 columns, e4m3 operands plus the residual terms, Gaussian, k = 60,
    l = 121."""
    grid, n, k, l, block = 128, 300, 60, 121, 10
    m = grid ** 3
    log(f"[bench] flow: generating {m}x{n} (3 FP32 planes) on the GPU")
    a = qs.to_colmajor(synth.flow_snapshots(grid, n, device="cuda"))
    torch.cuda.synchronize()
    if profile_only:
        sk = qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32",
                         sketch_dtype="fp8x", split_terms=3, pure=True, max_block_cols=block,
                         coalesce_cols=args.coalesce_fp8x)
        for _ in range(max(1, args.steps)):
            up, tot, _ = run_pass(sk, a, block)
            log(f"[bench] flow fp8x3 pass: updates {up:.2f} ms, total {tot:.2f} ms")
        sk.close()
        return {"profile_only": True, "workload": "flow", "update_ms": up, "total_ms": tot}
    # per update, and with the updates gathered into blocks of `coalesce`
    # columns before the products (the linear updates commute)
    co = args.coalesce
    leg = bench_stream_leg(args, "flow", a, m, n, k, l, block, "gaussian", "f32", True,
                           [("fp8", "fp8", 2), ("fp8_coalesced", "fp8", 2, co),
                            ("bf16", "bf16", 2), ("bf16_coalesced", "bf16", 2, co),
                            ("fp8x1_coalesced", "fp8x", 1, args.coalesce_fp8x),
                            ("fp8x2_coalesced", "fp8x", 2, args.coalesce_fp8x),
                            ("fp8x3_coalesced", "fp8x", 3, args.coalesce_fp8x),
                            ("fp8x4_coalesced", "fp8x", 4, args.coalesce_fp8x)],
                           PEAK_BF16, ref_block=n)
    leg["update_graph"] = {}
    for name, dt, terms, co_cols in (("fp8", "fp8", 2, 0), ("fp8_coalesced", "fp8", 2, co),
                                     ("fp8x3_coalesced", "fp8x", 3, args.coalesce_fp8x)):
        g = graph_saving(args, a, m, n, k, l, block, dt, terms, co_cols)
        leg["update_graph"][name] = g
        log(f"[bench] flow {name} updates as one graph: {g}")
    del a
    torch.cuda.empty_cache()
    # the headline: e4m3 terms on the fp8 matrix cores, three terms (the
    # fewest that meet the equal-error criterion here)
    f8 = leg["paths"]["fp8x3_coalesced"]
    leg.update({
        "workload": f"{m}x{n} pure quaternion FP32 flow snapshots, {n // block} linear updates of {block} "
                    f"columns gathered into blocks of up to {args.coalesce_fp8x} before the products, 3 e4m3 "
                    f"terms with per-tile scales on the fp8 matrix cores, Gaussian k={k} l={l}, "
                    f"both rangefinders",
        "ms_per_step": f8["total_ms"], "sketch_tflops": f8["sketch_tflops"],
        "roofline": {"bound": "mfma", "kernel": "w_fp8x_kernel (3 e4m3 terms, pure, gathered blocks)",
                     "achieved": f8["kernels"]["w"]["achieved_tflops"], "peak": PEAK_FP8 / 1e12,
                     "unit": "TFLOP/s", "frac": f8["kernels"]["w"]["frac"],
                     "avg_launch_ms": f8["kernels"]["w"]["avg_launch_ms"],
                     "per_update_y_hbm_frac": leg["paths"]["fp8"]["kernels"]["y"].get("hbm_frac")},
    })
    return leg


def bench_extras(args, a, m, n, k, l, block, make):
    """The general linear update and the two-pass variant on the same
    workload (BF16 operands, the bench's term count): medians over the timed
    steps."""
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    # A <- 0.999 A + 1.001 H per block: one in-place scaling of Y and W plus
    # the products with eta folded into their epilogues
    sk = make("bf16", args.terms)
    lin = []
    for it in range(args.warmup + args.steps):
        sk.reset()
        ev[0].record(st)
        for c0 in range(0, n, block):
            sk.update(c0, a[:, :, c0:c0 + block], theta=0.999, eta=1.001)
        ev[1].record(st)
        torch.cuda.synchronize()
        if it >= args.warmup:
            lin.append(ev[0].elapsed_time(ev[1]))
    sk.close()
    # two-pass: Y-only sketch, rangefinder only, projection pass over A
    sk = qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32", sketch_dtype="bf16",
                     split_terms=args.terms, max_block_cols=block, y_only=True)
    x = qs.qzeros(4, k, n, torch.float64, a.device)
    ys, rfs, prs = [], [], []
    for it in range(args.warmup + args.steps):
        sk.reset()
        ev[0].record(st)
        for c0 in range(0, n, block):
            sk.update(c0, a[:, :, c0:c0 + block])
        ev[1].record(st)
        q, _, rep = sk.finalize("pseudo_svd")
        ev[2].record(st)
        for c0 in range(0, n, block):
            sk.project(c0, a[:, :, c0:c0 + block], q, x)
        ev[3].record(st)
        torch.cuda.synchronize()
        if it >= args.warmup:
            ys.append(ev[0].elapsed_time(ev[1]))
            rfs.append(ev[1].elapsed_time(ev[2]))
            prs.append(ev[2].elapsed_time(ev[3]))
    err = sk.rel_error(a, q, x)
    sk.close()
    pr = float(np.median(prs))
    out = {
        "linear_update": {"theta": 0.999, "eta": 1.001, "update_ms": float(np.median(lin))},
        "two_pass": {"y_update_ms": float(np.median(ys)), "rangefinder_ms": float(np.median(rfs)),
                     "project_ms": pr, "total_ms": float(np.median(ys) + np.median(rfs) + pr),
                     "project_fp64_tflops": 2.0 * 16 * m * n * k / (pr * 1e-3) / 1e12,
                     "rel_error_pseudo_svd": err},
    }
    log(f"[bench] extras: {out}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=20000)
    ap.add_argument("--n", type=int, default=15000)
    ap.add_argument("--k", type=int, default=100)
    ap.add_argument("--l", type=int, default=201)
    ap.add_argument("--block", type=int, default=2048)
    ap.add_argument("--terms", type=int, default=2)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the general-update and two-pass measurements")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--batch-terms", type=int, default=3,
                    help="batch workload: bf16 terms of the data split (3 keeps every problem's error "
                         "within 1e-3 of the FP64 path's)")
    ap.add_argument("--coalesce", type=int, default=150,
                    help="flow workload: columns gathered per sketch product (coalesce_cols)")
    ap.add_argument("--coalesce-fp8x", type=int, default=256,
                    help="flow workload, e4m3-term paths: columns gathered per product (whole "
                         "update blocks, so 250 of the 10-column blocks)")
    ap.add_argument("--profile-only", action="store_true",
                    help="one bf16 pass only (for rocprofv3 runs)")
    ap.add_argument("--summarize-traffic", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "CMD_FETCH", "CMD_WRITE"),
                    help="write the W-kernel traffic summary from two rocprofv3 --pmc runs")
    ap.add_argument("--workload", default="all", choices=["all", "c2", "batch64", "image", "flow"],
                    help="all (default): the 20000 x 15000 matrix (headline) plus the image, batch "
                         "and flow workloads in the same line; or one of them alone")
    ap.add_argument("--summarize-stats", nargs=3, metavar=("DIR", "CMD", "OUT"),
                    help="write a kernel-time summary from a rocprofv3 --stats run")
    ap.add_argument("--summarize-busy", nargs=3, metavar=("DIR", "CMD", "OUT"),
                    help="write a matrix-core busy summary from a rocprofv3 --pmc run")
    args = ap.parse_args()
    if args.summarize_busy:
        summarize_busy(*args.summarize_busy, workload="c2" if args.workload == "all" else args.workload)
        return
    if args.summarize_stats:
        summarize_stats(*args.summarize_stats, workload="c2" if args.workload == "all" else args.workload)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    others = {"image": bench_image, "batch64": bench_batch, "flow": bench_flow}
    if args.workload in others:
        rec = others[args.workload](args, profile_only=args.profile_only)
        if args.profile_only:
            print(json.dumps(rec))
            return
        line = {"metric": METRIC, "value": rec.get("sketch_tflops", rec.get("sketch_tflops_whole_run")),
                "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": rec["ms_per_step"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "fp8" if args.workload == "flow" else "bf16",
                "data": "synthetic", "config": {"workload": rec["workload"]},
                "roofline": rec.get("roofline"), "cpu_baseline": None, "detail": rec}
        print(json.dumps(line))
        return
    m, n, k, l, block = args.m, args.n, args.k, args.l, args.block

    log(f"[bench] generating input {m}x{n} (4 FP32 planes) on the GPU")
    a = qs.to_colmajor(synth.config2(device="cuda", m=m, n=n))
    torch.cuda.synchronize()
    flops = sketch_flops(m, n, k, l)

    def make(sketch, terms=1):
        return qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32",
                           sketch_dtype=sketch, split_terms=terms, max_block_cols=block)

    if args.profile_only:
        # a plain copy of known size (one read and one write of CALIB_BYTES)
        # scales the HBM counters of the profiled kernels
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        sk = make("bf16", args.terms)
        for _ in range(max(1, args.steps)):
            up, tot, _ = run_pass(sk, a, block)
            log(f"[bench] bf16 pass: updates {up:.2f} ms, total {tot:.2f} ms")
        print(json.dumps({"profile_only": True, "update_ms": up, "total_ms": tot}))
        return

    errors = {}
    out_paths = {}
    if not args.no_fp64:
        # the FP64 path with the unrounded test matrices, and with the
        # rounded ones of each low-precision path (the equal-error references)
        for rnd in ("f64", "f32", "bf16", "fp8"):
            t0 = time.perf_counter()
            errs, rec = fp64_reference(a, m, n, k, l, block, "gaussian", "f32", False, rnd)
            for kind, e in errs.items():
                errors[("fp64_" + rnd, kind)] = e
            out_paths["fp64_" + rnd] = rec
            log(f"[bench] fp64 ({rnd} test matrices): updates {rec['update_ms']:.1f} ms, total "
                f"{rec['total_ms']:.1f} ms, errors {list(errs.values())} ({time.perf_counter() - t0:.1f} s)")

    # fp8: e4m3 data with per-tile scales plus a two-term residual correction
    paths = [("fp32", "f32", 1), ("bf16", "bf16", args.terms), ("fp8", "fp8", 2)]
    timing = {}
    for name, sketch, terms in paths:
        sk = make(sketch, terms)
        for _ in range(args.warmup):
            run_pass(sk, a, block)
        sk.set_timing(True)
        ups, tots = [], []
        torch.cuda.synchronize()
        for _ in range(args.steps):
            up, tot, res = run_pass(sk, a, block)
            ups.append(up)
            tots.append(tot)
        timing[name] = sk.timing()
        sk.set_timing(False)
        for kind, (q, x, rep) in res.items():
            errors[(name, kind)] = sk.rel_error(a, q, x)
            out_paths.setdefault(name, {})[kind + "_kappa"] = rep["kappa"]
        out_paths[name]["qb_stage"] = qb_stage_times(sk)
        out_paths.setdefault(name, {}).update({
            "update_ms": float(np.median(ups)), "total_ms": float(np.median(tots)),
            "sketch_tflops": flops / (np.median(ups) * 1e-3) / 1e12, "terms": terms})
        log(f"[bench] {name}: updates {np.median(ups):.2f} ms, step {np.median(tots):.2f} ms, "
            f"{out_paths[name]['sketch_tflops']:.1f} TFLOP/s, kernels {timing[name]}")
        sk.close()
        del res

    extras = None if args.no_extras else bench_extras(args, a, m, n, k, l, block, make)
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(a, m, n, k, l, block, args.cpu_seconds)
    del a
    torch.cuda.empty_cache()
    workloads = None
    if args.workload == "all":
        workloads = {}
        for name, fn in others.items():
            t0 = time.perf_counter()
            workloads[name] = fn(args)
            log(f"[bench] {name} done in {time.perf_counter() - t0:.1f} s")
            torch.cuda.empty_cache()

    bf = out_paths["bf16"]
    # roofline of the dominant kernel (the W product): algorithmic flops per
    # launch = 2 * 16 * m * ncols * l, averaged over the timed launches
    w_ms, w_n = timing["bf16"]["w"]
    y_ms, y_n = timing["bf16"]["y"]
    w_flops_total = 2.0 * 16 * m * n * l * args.steps
    y_flops_total = 2.0 * 16 * m * n * k * args.steps
    w_avg_ms = w_ms / max(w_n, 1)
    traffic = committed_traffic() if args.terms == 2 and (m, n, k, l, block) == (20000, 15000, 100, 201, 2048) else None
    w_ach = w_flops_total / (w_ms * 1e-3) if w_ms > 0 else 0.0
    y_ach = y_flops_total / (y_ms * 1e-3) if y_ms > 0 else 0.0
    roofline = {"bound": "mfma", "kernel": "w_mfma_kernel (bf16, %d terms)" % args.terms,
                "achieved": w_ach / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                "frac": w_ach / PEAK_BF16, "traffic": traffic,
                "avg_launch_ms": w_avg_ms, "launches": w_n,
                "executed_frac": w_ach * args.terms / PEAK_BF16,
                "y_kernel_achieved": y_ach / 1e12}

    eq = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        eq[kind] = {"e_fp64": errors.get(("fp64_f64", kind))}
        for name, _, _ in paths:
            # against the FP64 path with the same rounded test matrices
            # (and, for context, against the unrounded ones)
            ref = errors.get(("fp64_" + EMB_ROUND[name], kind))
            ref0 = errors.get(("fp64_f64", kind))
            e = errors.get((name, kind))
            eq[kind]["e_fp64_" + EMB_ROUND[name]] = ref
            eq[kind]["e_" + name] = e
            eq[kind]["rel_diff_" + name] = (abs(e - ref) / ref) if ref else None
            eq[kind]["rel_diff_unrounded_" + name] = (abs(e - ref0) / ref0) if ref0 else None
    speedup = out_paths["fp32"]["total_ms"] / bf["total_ms"]
    line = {
        "metric": METRIC,
        "value": bf["sketch_tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bf["total_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"{m}x{n} FP32 quaternion, rank 50 + 1e-4 noise, column blocks "
                               f"of {block}, Gaussian k={k} l={l}, both rangefinders",
                   "m": m, "n": n, "k": k, "l": l, "block": block, "bf16_terms": args.terms},
        "paths": out_paths, "equal_error": eq,
        "speedup_vs_fp32_wall": speedup,
        "speedup_vs_fp32_wall_fp8": out_paths["fp32"]["total_ms"] / out_paths["fp8"]["total_ms"],
        "roofline": roofline, "cpu_baseline": cpu, "extras": extras, "workloads": workloads,
        "host": {"cpu": platform.processor() or platform.machine(), "cores": os.cpu_count()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
