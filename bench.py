"""Benchmark of the MLS hot path on one MI355X.

One step = one pass of the whole path over the 1024^2-node workload:
N = 5,000 points drawn from an 8-component Gaussian mixture, D = 13 smooth
attributes, linear basis, Gaussian weight h = 0.03.  mls_fit (weights,
float64 contraction, float64 per-node solve) followed by mls_contour (10
isovalues per field, marching squares), inputs resident in HBM.  Prints one
JSON line with throughput (node x point pairs per second), fields per
second, p50/p99 step latency, the fit kernel's roofline figures, and the FP64
CPU oracle timed on a sample of the same workload.

--copy-calibration additionally runs a plain 256 MiB device copy after the
timed region, so that a counter run (FETCH_SIZE / WRITE_SIZE) of this script
sees a kernel of known traffic next to the fit kernel.
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
PEAK_BF16_MFMA_TFLOPS = 2500.0  # MI355X dense bfloat16 / float16 matrix peak
PEAK_HBM_GBS = 8000.0


def moment_terms(basis):
    # the rigid map is computed from the linear-basis contraction
    return {"constant": 1, "linear": 6, "quadratic": 15, "rigid": 6}[basis]


def basis_terms(basis):
    return {"constant": 1, "linear": 3, "quadratic": 6, "rigid": 3}[basis]


def cpu_baseline(w, row_stride=1, precision_note="FP64"):
    """The oracle on every row_stride-th grid row of the same workload,
    with the host's threads (at most 16)."""
    from oracle import oracle
    W, H = w.grid["width"], w.grid["height"]
    rows = np.arange(0, H, row_stride)
    pix = (rows[:, None] * W + np.arange(W)[None, :]).ravel()
    threads = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.fit_grid(w.points, w.values, w.grid, basis=w.basis, weight=w.weight, h=w.h,
                    alpha=w.alpha,
                    pixels=pix, threads=threads)
    dt = time.perf_counter() - t0
    if w.weight == "wendland":
        pairs = support_pairs(w.points, w.grid, w.h, rows=rows)
        what = "node-point pairs inside the support"
    else:
        pairs = pix.size * w.n
        what = "node-point pairs"
    sample = (f"all {H} rows" if row_stride == 1 else f"every {row_stride}th row") + \
        f" of the {W}x{H} grid ({pix.size} nodes x {w.n} points), {precision_note}, {dt:.2f} s"
    return {"value": pairs / dt, "unit": f"pairs/s ({what})", "cores": threads,
            "kind": "oracle", "sample": sample}


def support_pairs(points, grid, h, rows=None):
    """Number of (node, point) pairs with |node - point| < h (the pairs a
    compactly supported weight leaves), counted per point and node row."""
    x0, y0, dx, dy = grid["x0"], grid["y0"], grid["dx"], grid["dy"]
    W, H = grid["width"], grid["height"]
    px = points[:, 0].astype(np.float64)
    py = points[:, 1].astype(np.float64)
    row_ok = np.zeros(H, dtype=bool)
    row_ok[np.arange(H) if rows is None else rows] = True
    r_lo = np.ceil((py - h - y0) / dy).astype(np.int64)
    span = int(np.ceil(2 * h / abs(dy))) + 2
    total = 0
    for k in range(span + 1):
        r = r_lo + k
        ok = (r >= 0) & (r < H)
        r_c = np.clip(r, 0, H - 1)
        ok &= row_ok[r_c]
        ddy = y0 + r_c * dy - py
        rem = h * h - ddy * ddy
        ok &= rem > 0
        half = np.sqrt(np.where(ok, rem, 0.0))
        c_lo = np.maximum(np.floor((px - half - x0) / dx).astype(np.int64) + 1, 0)
        c_hi = np.minimum(np.ceil((px + half - x0) / dx).astype(np.int64) - 1, W - 1)
        total += int(np.where(ok, np.maximum(c_hi - c_lo + 1, 0), 0).sum())
    return total


def source_digest(paths):
    import hashlib
    hsh = hashlib.sha256()
    for rel in paths:
        with open(os.path.join(ROOT, rel), "rb") as f:
            hsh.update(f.read())
    return hsh.hexdigest()


def profiled_traffic(summary, sources):
    """HBM bytes per launch from a committed counter summary, if it was taken
    from the kernel sources as they are now; else None."""
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if ":" in line and line.split(":", 1)[0].strip() in (
                    "traffic_bytes_per_launch", "source_sha256"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip().strip("`")
    if rec.get("source_sha256") != source_digest(sources):
        return None
    try:
        return int(rec["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# committed FETCH_SIZE / WRITE_SIZE summaries, by workload name
TRAFFIC_SUMMARIES = {
    "c2_n5000_d13_linear_gauss_h0.03_1024": "fit_f64_c2_1024_traffic.md",
    "c3_n50000_d64_quadratic_gauss_h0.015_2048": "fit_lp_c3_traffic.md",
    "c5_n1000000_d16_quadratic_wendland_h0.01_4096": "fit_lp_c5_traffic.md",
}

# the sources that decide each contraction kernel's memory traffic
F64_SOURCES = ["paper_1408_0677_amd/csrc/mls_fit_f64.hip", "paper_1408_0677_amd/csrc/mls_solve.h"]
LP_SOURCES = ["paper_1408_0677_amd/csrc/mls_fit_lp.hip", "paper_1408_0677_amd/csrc/mls_solve.h"]


def serve_bench(args):
    """The served form on the request mix: closed-loop saturation for the
    16-bit served precision (with the library plan, then with the autotuner
    choosing slab widths per shape class) and the plain path, then Poisson
    arrivals at 0.5, 0.8 and 1.0 times the saturation rate.  16-bit
    requests of one kernel class share persistent batch kernels."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl

    reqs = wl.c4_requests(count=args.requests)
    dev = torch.device("cuda:0")
    budget = 2 << 30
    # a slot stages a whole batch (room for about 16 of the largest 16-bit
    # requests) or one float64 request (its Gaussian factor tables)
    slot_scratch = max(16 * max(api.fit_scratch_bytes(r.n, r.d, r.grid, "fp16") for r in reqs),
                       max(api.fit_scratch_bytes(r.n, r.d, r.grid, "f64") for r in reqs)) + \
        (1 << 20)
    # points + slots + the tuner's context scratch and output buffer
    srv = api.Server(0, budget + (args.slots + 2) * slot_scratch, args.slots, slot_scratch)
    pids = [srv.put_points(torch.from_numpy(r.points).to(dev),
                           torch.from_numpy(r.values).to(dev)) for r in reqs]
    pairs = [r.grid["width"] * r.grid["height"] * r.n for r in reqs]

    def run(prec, arrivals=None):
        """Submit every request (at its arrival time if given), collect
        results; returns (wall seconds, latencies)."""
        outs = {}
        pending = {}
        lat = []
        t0 = time.perf_counter()
        k = 0
        while k < len(reqs) or pending:
            now = time.perf_counter() - t0
            while k < len(reqs) and (arrivals is None or arrivals[k] <= now):
                r = reqs[k]
                out = torch.empty((r.d, r.grid["height"], r.grid["width"]), device=dev)
                t = srv.submit(pids[k], r.grid, out, None, basis=r.basis, h=r.h,
                               precision=prec)
                outs[t] = out
                pending[t] = k
                k += 1
            for t in list(pending):
                res = srv.poll(t)
                if res is not None:
                    assert res["status"] == 0, res
                    lat.append(res["t_end"] - res["t_submit"])
                    del pending[t], outs[t]
            time.sleep(0.0002)
        return time.perf_counter() - t0, np.array(lat)

    out = {"metric": "MLS served fit requests: throughput and p50/p99 latency",
           "unit": "requests/s", "n_gpus": 1, "data": "synthetic",
           "config": {"workload": "c4_256_requests_mixed", "requests": len(reqs),
                      "slots": args.slots, "budget_bytes": budget,
                      "pairs_total": int(sum(pairs))}}
    n_classes = 0
    for label, prec, tune in (("fp16", "fp16", False), ("fp16_tuned", "fp16", True),
                              ("f64", "f64", False)):
        srv.tuning(tune)
        run(prec)                                  # warm-up pass (queues new shape classes)
        if tune:
            # the tuner thread times the classes beside the scheduler
            t_end = time.time() + 120
            while srv.tuning_pending() and time.time() < t_end:
                time.sleep(0.01)
            n_classes = srv.tuned_classes()
        wall, lat = run(prec)
        rate = len(reqs) / wall
        rec = {"saturation_requests_per_s": rate, "pairs_per_s": sum(pairs) / wall,
               "closed_loop_p50_ms": 1e3 * float(np.percentile(lat, 50)),
               "closed_loop_p99_ms": 1e3 * float(np.percentile(lat, 99))}
        for frac in (0.5, 0.8, 1.0):
            arr = wl.poisson_arrivals(1, len(reqs), frac * rate)
            wall2, lat2 = run(prec, arr)
            rec[f"poisson_{frac}"] = {"offered_requests_per_s": frac * rate,
                                      "achieved_requests_per_s": len(reqs) / wall2,
                                      "p50_ms": 1e3 * float(np.percentile(lat2, 50)),
                                      "p99_ms": 1e3 * float(np.percentile(lat2, 99))}
        out[label] = rec
    out["tuned_shape_classes"] = n_classes
    out["value"] = out["fp16_tuned"]["saturation_requests_per_s"]
    srv.close()
    return out


LAYOUT_ITERS = 1000
# fp64 operations of one ordered source-node pair of the repulsion (Eq. 1),
# each fusible multiply-add counted once, as the lane peak counts one FMA
# per lane and clock: two differences, the squared distance (a product and
# a multiply-add), sqrt, the cube, +eta, the division, and the two force
# components accumulated by multiply-adds
LAYOUT_OPS_PER_PAIR = 10
# one fp64 add or multiply per lane per clock: 256 CUs x 64 lanes x 2.4 GHz
FP64_LANE_OPS_PEAK = 256 * 64 * 2.4e9


def layout_bench(args):
    """Layout runs of LAYOUT_ITERS iterations (t_k = t0 lambda^k) on the
    Delaunay meshes of the timing-table sizes, plus a 65536-node run that
    fills the chip; positions resident in HBM, timed with events on the
    stream the iterations are launched on."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    paper_s = {306: 0.783082, 1000: 1.314509, 2245: 1.777599}
    stream = torch.cuda.current_stream()
    rows = []
    for n, iters in ((306, LAYOUT_ITERS), (1000, LAYOUT_ITERS), (2245, LAYOUT_ITERS),
                     (65536, 50)):
        pts, mesh, prm = wl.layout_workload(n)
        P0 = torch.from_numpy(pts.astype(np.float32)).cuda()
        M = {k: torch.from_numpy(np.ascontiguousarray(mesh[k])).cuda()
             for k in ("adj_start", "adj", "fan_start", "fan")}
        P = P0.clone()

        def run(k):
            P.copy_(P0)
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            api.layout(P, M, iterations=k, **prm)
            b.record(stream)
            b.synchronize()
            return a.elapsed_time(b)

        for _ in range(max(args.warmup, 1)):
            run(iters)
        steps = max(args.steps // 4, 3)
        full = [run(iters) for _ in range(steps)]
        empty = [run(0) for _ in range(steps)]
        per_it_us = (np.median(full) - np.median(empty)) * 1e3 / iters
        ops = LAYOUT_OPS_PER_PAIR * n * (n - 1)
        row = {"nodes": n, "triangles": int(mesh["triangles"].shape[0]), "iterations": iters,
               "run_ms_p50": float(np.median(full)), "run_ms_p99": float(np.percentile(full, 99)),
               "us_per_iteration": float(per_it_us),
               "iterations_per_s": 1e6 / per_it_us,
               "repulsion_ops_per_s": ops / (per_it_us * 1e-6)}
        if n in paper_s:
            row["paper_layout_s"] = paper_s[n]
        rows.append(row)
        note = f"layout n={n}: {per_it_us:.2f} us/iteration"
        print(note, file=sys.stderr, flush=True)
    main_row = rows[2]
    big = rows[3]
    achieved = big["repulsion_ops_per_s"] / 1e12
    peak = FP64_LANE_OPS_PEAK / 1e12
    out = {
        "metric": "layout iterations/s (2245-node Delaunay mesh, Eq. 1-3 with the "
                  "limiting-line clamp, float64)",
        "value": main_row["iterations_per_s"], "unit": "iterations/s", "n_gpus": 1,
        "steps": max(args.steps // 4, 3), "warmup": max(args.warmup, 1),
        "ms_per_step": main_row["run_ms_p50"], "higher_is_better": True, "scaling": "weak",
        # the paper states no iteration count for its layout times
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "layout_2245_nodes_1000_iterations", "canvas": 600,
                   "nodes": 2245, "iterations": LAYOUT_ITERS},
        "per_n": rows,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "Tops/s (fp64 lane operations)", "frac": achieved / peak,
                     "traffic": None, "kernel": "layout_step_kernel<16> at 65536 nodes",
                     "algorithmic_ops_per_launch": LAYOUT_OPS_PER_PAIR * 65536 * 65535,
                     "kernel_us": big["us_per_iteration"]},
    }
    if not args.no_cpu_baseline:
        from oracle import oracle
        pts, mesh, prm = wl.layout_workload(2245)
        threads = min(os.cpu_count() or 1, 16)
        k = 10000
        t0 = time.perf_counter()
        oracle.layout(pts.astype(np.float32).astype(np.float64), mesh, iterations=k,
                      threads=threads, **prm)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": k / dt, "unit": "iterations/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"{k} iterations of the 2245-node layout, {dt:.2f} s"}
    return out


def maps_bench(args):
    """The space mappings of Sec. 3.4 on the 1024^2 / 13-field fit: discrete
    bands with colours, and adaptive contour lines from the fit's
    gradients; HBM bound (algorithmic bytes: bands 4 B read + 5 B written
    per node and field; lines 12 B read + 4 B written)."""
    import torch
    from paper_1408_0677_amd import api, workloads as wl
    w = wl.c2()
    dev = torch.device("cuda:0")
    P = torch.from_numpy(w.points).to(dev)
    V = torch.from_numpy(w.values).to(dev)
    F, G, _ = api.fit_grad(P, V, w.grid, basis=w.basis, h=w.h)
    iso = torch.from_numpy(w.iso()).to(dev)
    cmap = torch.arange(w.d * (w.n_iso + 1), dtype=torch.int32, device=dev)
    lo, hi = w.values.min(0), w.values.max(0)
    levels = torch.from_numpy(np.stack([lo, (hi - lo) / 11.0], 1).astype(np.float32)).to(dev)
    ctx = api.default_context(0)
    stream = torch.cuda.current_stream()
    nodes = w.grid["width"] * w.grid["height"] * w.d
    res = {}
    for name, fn, nbytes in (
            ("bands", lambda: api.map_bands(F, w.grid, iso, colormap=cmap, ctx=ctx), 9 * nodes),
            ("lines", lambda: api.map_adaptive(F, G, w.grid, levels, ctx=ctx), 16 * nodes)):
        for _ in range(max(args.warmup, 1)):
            fn()
        ctx.trace(True)
        ms = []
        for _ in range(max(args.steps, 10)):
            fn()
            ms.append(list(ctx.trace_last()["stages"].values())[0])
        ctx.trace(False)
        k = float(np.mean(ms))
        res[name] = {"kernel_ms": k, "algorithmic_bytes": nbytes,
                     "achieved_GBs": nbytes / (k * 1e-3) / 1e9}
    lines = res["lines"]
    return {
        "metric": "space mappings (Sec. 3.4): fields/s at 1024^2, bands + colours and adaptive "
                  "lines",
        "value": w.d / ((res["bands"]["kernel_ms"] + lines["kernel_ms"]) * 1e-3),
        "unit": "fields/s", "n_gpus": 1, "steps": max(args.steps, 10),
        "warmup": max(args.warmup, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 in, f64 lines", "data": "synthetic",
        "config": {"workload": "c2_maps_13_fields_1024", "fields": w.d, "isovalues": w.n_iso,
                   "adaptive_levels": 3},
        "per_mapping": res,
        "roofline": {"bound": "hbm", "achieved": lines["achieved_GBs"], "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": lines["achieved_GBs"] / PEAK_HBM_GBS,
                     "traffic": None, "kernel": "map_adaptive_kernel"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--latency-fits", type=int, default=0,
                    help="single fits behind the p50/p99 fit latency (default: 100, "
                         "fewer where 100 would take over 20 s)")
    ap.add_argument("--workload", default="c2",
                    choices=["c2", "c3", "c4", "c5", "t1", "layout", "maps"],
                    help="c2: the 1024^2 float64 fit + contour step (default); c3: the "
                         "2048^2 / D = 64 quadratic bfloat16 fit; c5: the 4096^2 / "
                         "N = 10^6 Wendland bfloat16 fit + contour; c4: the served "
                         "request mix with Poisson arrivals; t1: the paper's timing-table "
                         "shape (600^2, N = 306 / 1000 / 2245, D = 2, linear, the "
                         "inverse-distance weight of Eq. 4), float64; layout: the "
                         "planarity-preserving layout of Sec. 3.2 at the timing-table "
                         "sizes, float64; maps: the discrete-colour and adaptive-line "
                         "mappings of Sec. 3.4 of the 1024^2 / 13-field fit")
    ap.add_argument("--requests", type=int, default=256)
    ap.add_argument("--slots", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path "
              "shards by node rows, which this library does not yet run across GPUs.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1408_0677_amd import api, workloads as wl

    if args.workload == "c4":
        print(json.dumps(serve_bench(args)), flush=True)
        return

    if args.workload == "layout":
        print(json.dumps(layout_bench(args)), flush=True)
        return

    if args.workload == "maps":
        print(json.dumps(maps_bench(args)), flush=True)
        return

    if args.workload == "t1":
        import dataclasses
        recs = [fit_step_bench(args, wl.t1(n), "f64") for n in (306, 1000, 2245)]
        # the paper's other two modes at the same shape: Mean MLS (Eq. 5, the
        # constant basis) and Rigid MLS (Eq. 9-10)
        quiet = argparse.Namespace(**dict(vars(args), no_cpu_baseline=True))
        mean = [fit_step_bench(quiet, dataclasses.replace(wl.t1(n), basis="constant"), "f64")
                for n in (306, 1000, 2245)]
        rigid = [fit_step_bench(quiet, dataclasses.replace(wl.t1(n), basis="rigid"), "f64")
                 for n in (306, 1000, 2245)]
        out = dict(recs[-1])
        out["metric"] = ("MLS pixel·point pairs/s at the timing-table shape (600^2, D = 2, "
                         "linear, inverse-distance weight)")
        # the paper's Affine MLS timings at this shape (Table 1, GTX 285, its
        # own shader): context for the same workload on other hardware
        paper_s = {306: 0.026670, 1000: 0.100724, 2245: 0.242192}
        paper_mean_s = {306: 0.017420, 1000: 0.064938, 2245: 0.147089}
        paper_rigid_s = {306: 0.028846, 1000: 0.116083, 2245: 0.246789}
        out["per_n"] = []
        for r, rm, rr in zip(recs, mean, rigid):
            n = r["config"]["points"]
            out["per_n"].append({
                "points": n, "ms_per_step": r["ms_per_step"],
                "fit_p50_ms": r["latency_ms"]["fit_p50"], "pairs_per_s": r["value"],
                "paper_affine_s": paper_s[n],
                "speedup_vs_paper_fit": paper_s[n] * 1e3 / r["latency_ms"]["fit_p50"],
                "mean_fit_p50_ms": rm["latency_ms"]["fit_p50"], "paper_mean_s": paper_mean_s[n],
                "rigid_fit_p50_ms": rr["latency_ms"]["fit_p50"],
                "paper_rigid_s": paper_rigid_s[n],
                "cpu_baseline": r.get("cpu_baseline")})
        # value (pairs/s of the whole step at N = 2245) over the paper's pairs/s
        out["vs_baseline"] = out["value"] / (600 * 600 * 2245 / paper_s[2245])
        print(json.dumps(out), flush=True)
        return
    if args.workload == "c2":
        w, prec = wl.c2(), "f64"
    elif args.workload == "c3":
        w, prec = wl.c3(), "bf16"
    else:
        w, prec = wl.c5(), "bf16"
    out = fit_step_bench(args, w, prec)
    print(json.dumps(out), flush=True)


def fit_step_bench(args, w, prec):
    """One step = mls_fit over the whole grid, then mls_contour over every
    field if the workload has isovalues; inputs resident in HBM."""
    import torch
    from paper_1408_0677_amd import api

    dev = torch.device("cuda:0")
    P = torch.from_numpy(w.points).to(dev)
    V = torch.from_numpy(w.values).to(dev)
    iso = torch.from_numpy(w.iso()).to(dev) if w.n_iso else None
    W, H = w.grid["width"], w.grid["height"]
    fields = torch.empty((w.d, H, W), dtype=torch.float32, device=dev)
    degree = torch.empty((H, W), dtype=torch.uint8, device=dev)
    ctx = api.default_context(0)
    stream = torch.cuda.current_stream()
    kw = dict(basis=w.basis, weight=w.weight, h=w.h, alpha=w.alpha, precision=prec, out=fields,
              degree_out=degree, ctx=ctx, stream=stream)

    # size the segment buffer once (outside the timed region)
    api.fit(P, V, w.grid, **kw)
    capacity = 0
    seg_count = 0
    if iso is not None:
        segs0, _, _ = api.contour(fields, w.grid, iso, want_cases=False, ctx=ctx,
                                  stream=stream)
        capacity = int(segs0.shape[0] * 1.25) + 1024
        seg_count = int(segs0.shape[0])

    fit_ev = []

    def step(timed):
        if timed:
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
        api.fit(P, V, w.grid, **kw)
        if timed:
            b.record(stream)
            fit_ev.append((a, b))
        if iso is not None:
            # the product is the segments and their (field, iso, cell) ids; the
            # per-(cell, iso) case bytes are an optional output left off here
            api.contour(fields, w.grid, iso, want_cases=False, capacity=capacity,
                        want_ids=True, ctx=ctx, stream=stream)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()

    step_ms = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        step(True)            # mls_contour returns after the stream has delivered its count
        if iso is None:
            torch.cuda.current_stream().synchronize()
        step_ms.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_ms = np.array(step_ms)
    fit_ms = np.array([a.elapsed_time(b) for a, b in fit_ev])

    # fit latency over single fits, each bracketed by events on the launch
    # stream (at least 100, fewer only where 100 would take over 20 s)
    n_lat = args.latency_fits if args.latency_fits > 0 else (
        100 if float(np.mean(fit_ms)) * 100 <= 20e3 else max(
            args.steps, int(20e3 / float(np.mean(fit_ms)))))
    # the library's own stage events time the contraction kernel alone
    # (staging and the cell list are separate stages), on the launch stream
    lat_ms, contract_ms, stage_ms = [], [], {}
    form = None
    ctx.trace(True)
    for _ in range(n_lat):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        api.fit(P, V, w.grid, **kw)
        b.record(stream)
        b.synchronize()
        lat_ms.append(a.elapsed_time(b))
        rec = ctx.trace_last()
        form = rec["form"]
        contract_ms.append(rec["stages"]["contract"])
        for k, v in rec["stages"].items():
            stage_ms.setdefault(k, []).append(v)
    ctx.trace(False)
    lat_ms = np.array(lat_ms)

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    nodes = W * H
    F = moment_terms(w.basis) + basis_terms(w.basis) * w.d
    if w.weight == "wendland":
        pairs = support_pairs(w.points, w.grid, w.h)
        pair_kind = "node-point pairs inside the support"
    else:
        pairs = nodes * w.n
        pair_kind = "node-point pairs"
    flops = 2.0 * F * pairs
    # the two-pass (shape-function) form contracts n_mom + D columns, not
    # n_mom + m D: its roofline counts its own work
    if form == 2:
        F_form = moment_terms(w.basis) + w.d
    else:
        F_form = F
    flops_form = 2.0 * F_form * pairs
    ms_per_step = wall * 1e3 / args.steps
    # the contraction kernel's own time, from the library's stage events
    kern_ms = float(np.mean(contract_ms))
    achieved = flops_form / (kern_ms * 1e-3) / 1e12
    if prec == "f64":
        peak, kernel, sources = PEAK_F64_MFMA_TFLOPS, "fit_f64_kernel", F64_SOURCES
    else:
        peak, sources = PEAK_BF16_MFMA_TFLOPS, LP_SOURCES
        kernel = "fit_shape_kernel" if form == 2 else "fit_lp_kernel"
    # counter summaries exist per workload; any other workload reports none
    summary = TRAFFIC_SUMMARIES.get(w.name)
    traffic = profiled_traffic(summary, sources) if summary else None

    metric = ("MLS pixel·point pairs/s and fields/s at 1024² grid; p50/p99 fit latency"
              if args.workload == "c2" else
              f"MLS pixel·point pairs/s and fields/s ({args.workload}); p50/p99 fit latency")
    out = {
        "metric": metric,
        "value": pairs * args.steps / wall,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": {"workload": w.name, "nodes": nodes, "points": w.n, "attributes": w.d,
                   "basis": w.basis, "weight": w.weight, "h": w.h, "pairs": pairs,
                   "pair_kind": pair_kind,
                   "contraction": "f64 mfma" if prec == "f64" else
                                  f"{prec} mfma, float32 accumulation",
                   "solve": "f64", "isovalues_per_field": w.n_iso,
                   "segments": seg_count},
        "fields_per_s": w.d * args.steps / wall,
        "latency_ms": {"p50": float(np.percentile(step_ms, 50)),
                       "p99": float(np.percentile(step_ms, 99)),
                       "fit_p50": float(np.percentile(lat_ms, 50)),
                       "fit_p99": float(np.percentile(lat_ms, 99)),
                       "fit_samples": int(n_lat),
                       "stages_mean": {k: float(np.mean(v)) for k, v in stage_ms.items()}},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak,
                     "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": traffic, "kernel": kernel,
                     "algorithmic_flops_per_launch": flops_form,
                     "form": {0: "f64 one pass", 1: "16-bit one pass",
                              2: "16-bit two passes (shape functions)"}.get(form),
                     "one_pass_equivalent_tflops": flops / (kern_ms * 1e-3) / 1e12,
                     "kernel_ms": kern_ms},
    }
    if not args.no_cpu_baseline:
        if args.workload in ("c2", "t1"):
            out["cpu_baseline"] = cpu_baseline(w, row_stride=1)
        elif args.workload == "c3":
            out["cpu_baseline"] = cpu_baseline(w, row_stride=128)
        else:
            out["cpu_baseline"] = cpu_baseline(w, row_stride=1024)
    return out


if __name__ == "__main__":
    main()
