"""Benchmark of the one-pass quaternion low-rank approximation on one MI355X.

Workload (default): A in Q^{20000 x 15000}, four FP32 planes (4.8 GB), rank-50
quaternion factors with sigma_i = i^-2 plus 1e-4 relative Gaussian noise,
streamed once in column blocks of 2048, Gaussian test matrices, k = 100,
l = 201, both rangefinders.  Inputs are synthetic and resident in HBM before
timing starts.

One step = one whole one-pass approximation: reset, all column-block updates
of the sketches, then the QB stage with pseudo-QR and with pseudo-SVD.  Paths:
  fp64   FP64 sketch on the GPU (the FP64 plain method; error reference, not timed)
  fp32   FP32 sketch on the matrix cores (the same-GPU FP32 plain path)
  bf16   BF16 sketch with the data split in `--terms` bf16 terms (timed: `value`)

Prints one JSON line.  `value` = algorithmic sketch TFLOP/s of the bf16 path
(2 * 16 * m * n * (k + l) flops over the time of its updates).
"""
from __future__ import annotations

import argparse
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
PEAK_HBM = 8e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def sketch_flops(m, n, k, l, pure=False):
    return 2.0 * (12 if pure else 16) * m * n * (k + l)


def run_pass(sk, a, block, kinds=("pseudo_qr", "pseudo_svd")):
    """One whole one-pass approximation; returns (update_ms, total_ms, results)."""
    st = torch.cuda.current_stream()
    sk.reset()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(st)
    n = a.shape[2]
    for c0 in range(0, n, block):
        sk.update(c0, a[:, :, c0:c0 + block])
    e1.record(st)
    res = {}
    for kind in kinds:
        res[kind] = sk.finalize(kind)
    e2.record(st)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1), e0.elapsed_time(e2), res


def cpu_baseline(a_dev, m, n, k, l, block, seconds=20.0):
    """The oracle's FP64 sketch update timed on the host cores on a bounded
    sample: the first column blocks of the same input, until ~`seconds`."""
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
    return {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": os.cpu_count(),
            "kind": "oracle",
            "sample": f"FP64 NumPy sketch update of the first {cols} of {n} columns "
                      f"(m={m}, k={k}, l={l}, Gaussian, Psi generation included), {dt:.1f} s"}


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
    ap.add_argument("--terms", type=int, default=3)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 reference run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--profile-only", action="store_true",
                    help="one bf16 pass only (for rocprofv3 runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    m, n, k, l, block = args.m, args.n, args.k, args.l, args.block

    log(f"[bench] generating input {m}x{n} (4 FP32 planes) on the GPU")
    a = qs.to_colmajor(synth.config2(device="cuda", m=m, n=n))
    torch.cuda.synchronize()
    flops = sketch_flops(m, n, k, l)

    def make(sketch, terms=1):
        return qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32",
                           sketch_dtype=sketch, split_terms=terms, max_block_cols=block)

    if args.profile_only:
        sk = make("bf16", args.terms)
        for _ in range(max(1, args.steps)):
            up, tot, _ = run_pass(sk, a, block)
            log(f"[bench] bf16 pass: updates {up:.2f} ms, total {tot:.2f} ms")
        print(json.dumps({"profile_only": True, "update_ms": up, "total_ms": tot}))
        return

    errors = {}
    out_paths = {}
    if not args.no_fp64:
        log("[bench] FP64 reference pass (untimed)")
        sk64 = qs.Sketcher(m, n, k, l, seed=0, embedding="gaussian", input_dtype="f32",
                           sketch_dtype="f64", max_block_cols=block)
        t0 = time.perf_counter()
        up, tot, res = run_pass(sk64, a, block)
        for kind, (q, x, rep) in res.items():
            errors[("fp64", kind)] = sk64.rel_error(a, q, x)
        out_paths["fp64"] = {"update_ms": up, "total_ms": tot}
        log(f"[bench] fp64: updates {up:.1f} ms, total {tot:.1f} ms, errors "
            f"{[errors[('fp64', kd)] for kd in res]} ({time.perf_counter() - t0:.1f} s)")
        sk64.close()
        del res

    paths = [("fp32", "f32", 1), ("bf16", "bf16", args.terms)]
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
        out_paths.setdefault(name, {}).update({
            "update_ms": float(np.median(ups)), "total_ms": float(np.median(tots)),
            "sketch_tflops": flops / (np.median(ups) * 1e-3) / 1e12, "terms": terms})
        log(f"[bench] {name}: updates {np.median(ups):.2f} ms, step {np.median(tots):.2f} ms, "
            f"{out_paths[name]['sketch_tflops']:.1f} TFLOP/s, kernels {timing[name]}")
        sk.close()
        del res

    bf = out_paths["bf16"]
    # roofline of the dominant kernel (the W product): algorithmic flops per
    # launch = 2 * 16 * m * ncols * l, averaged over the timed launches
    w_ms, w_n = timing["bf16"]["w"]
    y_ms, y_n = timing["bf16"]["y"]
    nblocks = (n + block - 1) // block
    w_flops_total = 2.0 * 16 * m * n * l * args.steps
    y_flops_total = 2.0 * 16 * m * n * k * args.steps
    w_avg_ms = w_ms / max(w_n, 1)
    w_ach = w_flops_total / (w_ms * 1e-3) if w_ms > 0 else 0.0
    y_ach = y_flops_total / (y_ms * 1e-3) if y_ms > 0 else 0.0
    roofline = {"bound": "mfma", "kernel": "w_mfma_kernel (bf16, %d terms)" % args.terms,
                "achieved": w_ach / 1e12, "peak": PEAK_BF16 / 1e12, "unit": "TFLOP/s",
                "frac": w_ach / PEAK_BF16, "traffic": None,
                "avg_launch_ms": w_avg_ms, "launches": w_n,
                "executed_frac": w_ach * args.terms / PEAK_BF16,
                "y_kernel_achieved": y_ach / 1e12}

    eq = {}
    for kind in ("pseudo_qr", "pseudo_svd"):
        ref = errors.get(("fp64", kind))
        e16 = errors.get(("bf16", kind))
        e32 = errors.get(("fp32", kind))
        eq[kind] = {"e_fp64": ref, "e_fp32": e32, "e_bf16": e16,
                    "rel_diff_bf16": (abs(e16 - ref) / ref) if ref else None,
                    "rel_diff_fp32": (abs(e32 - ref) / ref) if ref else None}
    cpu = None
    if not args.no_cpu:
        log("[bench] CPU oracle baseline")
        cpu = cpu_baseline(a, m, n, k, l, block, args.cpu_seconds)
    speedup = out_paths["fp32"]["total_ms"] / bf["total_ms"]
    line = {
        "metric": "one-pass qLRA wall time + sketch TFLOP/s at equal rel. error, BF16/FP8 vs FP32",
        "value": bf["sketch_tflops"], "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": bf["total_ms"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"{m}x{n} FP32 quaternion, rank 50 + 1e-4 noise, column blocks "
                               f"of {block}, Gaussian k={k} l={l}, both rangefinders",
                   "m": m, "n": n, "k": k, "l": l, "block": block, "bf16_terms": args.terms},
        "paths": out_paths, "equal_error": eq,
        "speedup_vs_fp32_wall": speedup,
        "roofline": roofline, "cpu_baseline": cpu,
        "host": {"cpu": platform.processor() or platform.machine(), "cores": os.cpu_count()},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
