"""Benchmark of the MLS hot path on one MI355X.

One step = one pass of the whole path over the 1024^2-node workload:
N = 5,000 points drawn from an 8-component Gaussian mixture, D = 13 smooth
attributes, linear basis, Gaussian weight h = 0.03 (mls_fit: weights,
float64 contraction, float64 per-node solve), with the inputs resident in
HBM.  Prints one JSON line with throughput (node x point pairs per second),
fields per second, p50/p99 step latency, the fit kernel's roofline figures,
and the FP64 CPU oracle timed on a sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_F64_MFMA_TFLOPS = 78.6     # MI355X dense float64 matrix peak
PEAK_HBM_GBS = 8000.0


def moment_terms(basis):
    return {"constant": 1, "linear": 6, "quadratic": 15}[basis]


def basis_terms(basis):
    return {"constant": 1, "linear": 3, "quadratic": 6}[basis]


def cpu_baseline(w, row_stride=16):
    """The oracle on every row_stride-th grid row of the same workload."""
    from oracle import oracle
    W, H = w.grid["width"], w.grid["height"]
    rows = np.arange(0, H, row_stride)
    pix = (rows[:, None] * W + np.arange(W)[None, :]).ravel()
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.fit_grid(w.points, w.values, w.grid, basis=w.basis, h=w.h, pixels=pix,
                    threads=threads)
    dt = time.perf_counter() - t0
    pairs = pix.size * w.n
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"every {row_stride}th row of the {W}x{H} grid ({pix.size} nodes x "
                      f"{w.n} points), FP64, {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by node rows, which this build does not run across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1408_0677_amd import api, workloads as wl

    w = wl.c2()
    dev = torch.device("cuda:0")
    P = torch.from_numpy(w.points).to(dev)
    V = torch.from_numpy(w.values).to(dev)
    W, H = w.grid["width"], w.grid["height"]
    fields = torch.empty((w.d, H, W), dtype=torch.float32, device=dev)
    degree = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ctx = api.default_context(0)
    stream = torch.cuda.current_stream()

    def step():
        api.fit(P, V, w.grid, basis=w.basis, h=w.h, out=fields, degree_out=degree,
                ctx=ctx, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        step()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array([s.elapsed_time(e) for s, e in ev])

    nodes = W * H
    pairs = nodes * w.n
    F = moment_terms(w.basis) + basis_terms(w.basis) * w.d
    flops = 2.0 * F * pairs
    ms_per_step = wall * 1e3 / args.steps
    kern_ms = float(np.mean(step_ms))   # one fit kernel launch per step
    achieved = flops / (kern_ms * 1e-3) / 1e12

    out = {
        "metric": "MLS pixel·point pairs/s and fields/s at 1024² grid; p50/p99 fit latency",
        "value": pairs * args.steps / wall,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": nodes, "points": w.n, "attributes": w.d,
                   "basis": w.basis, "weight": "gaussian", "h": w.h,
                   "contraction": "f64 mfma", "solve": "f64"},
        "fields_per_s": w.d * args.steps / wall,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99))},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_F64_MFMA_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_F64_MFMA_TFLOPS,
                     "traffic": None, "kernel": "fit_f64_kernel",
                     "algorithmic_flops_per_launch": flops,
                     "kernel_ms": kern_ms},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
