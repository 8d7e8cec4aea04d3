"""Benchmark of the exact two-layer GRNG -> RNG build on one MI355X.

Workload: 100,000 points in 16-D, a Gaussian mixture of 32 isotropic clusters
(centres uniform in [0,10]^16, sigma 0.5) on the 2^-19 grid, with 1,000 random
pivots whose radius is the distance to their 100th nearest other point.  One
step = build the GRNG of the pivot layer, then the exact RNG of all points
(every kept/eliminated decision exact).  Inputs (points, pivot ids, radii) are
resident in device memory before timing starts.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: this build runs on one GPU.
``--workload subspace3`` times the 1M x 32-D three-layer build instead (for
profiling that configuration; the benchmark line is the default workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks, and the VALU issue peak derived from unit counts:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-operations/s (one
# float32 min or max per lane per cycle; packed FP32 is not used).
MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6
MI355X_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12


KERNEL_SOURCES = {"k_pairs_tiled": ["k_rng.hip", "common.h"], "k_pair_masks": ["k_rng.hip", "common.h"],
                  "k_lune_guided": ["k_rng.hip", "common.h"], "k_vgrng_tiles": ["k_pivots.hip", "common.h"]}


def source_hash(kernel: str) -> str:
    """sha256 of the sources a kernel is built from (to tell whether measured counters still apply)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2208_10022_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel source and this workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh).get(kernel)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_sha256") != source_hash(kernel) or rec.get("workload") != workload:
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


PAIR_RECORD_BYTES = 8 * (12 + 2 * 64)   # tile bounds, pivot ids and the two candidate-mask vectors


def attainable_peaks(torch) -> dict:
    """Attainable roofs on this device, beside the published ones: a 4 GiB
    device-to-device copy (bytes read + written per second, best of 5) and a
    float64 8192^3 library GEMM (best of 5)."""
    out = {}
    nbytes = 4 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    best = float("inf")
    for _ in range(6):
        ev[0].record()
        dst.copy_(src)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    out["copy_gb_s"] = 2 * nbytes / (best / 1e3) / 1e9
    out["hbm_peak_gb_s"] = MI355X_HBM_GBS
    del src, dst
    n = 8192
    a = torch.rand(n, n, dtype=torch.float64, device="cuda:0")
    b = torch.rand(n, n, dtype=torch.float64, device="cuda:0")
    best = float("inf")
    for _ in range(6):
        ev[0].record()
        torch.matmul(a, b)
        ev[1].record()
        torch.cuda.synchronize()
        best = min(best, ev[0].elapsed_time(ev[1]))
    out["dgemm_tflop_s"] = 2 * n ** 3 / (best / 1e3) / 1e12
    out["fp64_mfma_peak_tflop_s"] = MI355X_FP64_TFLOPS
    return out


def kernel_rooflines(st: dict) -> dict:
    """Per main kernel of the last build: time and achieved fraction of its roof.

    k_vgrng_tiles  (min,max) product, VALU: 2 ops per (point, pivot j, pivot k)
                   for each of two radius choices = 2 * vgrng_ops.
    k_pairs_tiled  MFMA f64 distance tiles (pairs_flops) and the Stage IV
                   (min,max) product on the VALU (stage4_ops); the roof is the
                   one with the longer time at peak.
    k_lune_guided  witness rows streamed: lune_bytes (row + cell bound per
                   witness test) against HBM bandwidth.
    k_pair_masks   one 1,120-byte record written per tile pair.
    """
    out = {}
    ms = st["ms_vgrng"]
    ach = 2.0 * st["vgrng_ops"] / (ms / 1e3) / 1e12
    out["k_vgrng_tiles"] = {"bound": "alu", "achieved": ach, "peak": MI355X_VALU_TOPS, "unit": "Tops/s",
                            "frac": ach / MI355X_VALU_TOPS, "ms": ms}
    ms = st["ms_pairs"]
    t_mfma = st["pairs_flops"] / (MI355X_FP64_TFLOPS * 1e12)
    t_valu = st["stage4_ops"] / (MI355X_VALU_TOPS * 1e12)
    if t_mfma >= t_valu:
        ach = st["pairs_flops"] / (ms / 1e3) / 1e12
        out["k_pairs_tiled"] = {"bound": "mfma", "achieved": ach, "peak": MI355X_FP64_TFLOPS, "unit": "TFLOP/s",
                                "frac": ach / MI355X_FP64_TFLOPS, "ms": ms,
                                "valu_frac": t_valu / (ms / 1e3)}
    else:
        ach = st["stage4_ops"] / (ms / 1e3) / 1e12
        out["k_pairs_tiled"] = {"bound": "alu", "achieved": ach, "peak": MI355X_VALU_TOPS, "unit": "Tops/s",
                                "frac": ach / MI355X_VALU_TOPS, "ms": ms, "mfma_frac": t_mfma / (ms / 1e3)}
    ms = st["ms_lune"]
    ach = st["lune_bytes"] / (ms / 1e3) / 1e9
    out["k_lune_guided"] = {"bound": "hbm", "achieved": ach, "peak": MI355X_HBM_GBS, "unit": "GB/s",
                            "frac": ach / MI355X_HBM_GBS, "ms": ms,
                            "note": "witness rows are served from L2/MALL, so the algorithmic bytes can exceed "
                                    "the HBM roof"}
    ms = st["ms_pair_masks"]
    if ms > 0:
        ach = PAIR_RECORD_BYTES * st["tile_pairs"] / (ms / 1e3) / 1e9
        out["k_pair_masks"] = {"bound": "hbm", "achieved": ach, "peak": MI355X_HBM_GBS, "unit": "GB/s",
                               "frac": ach / MI355X_HBM_GBS, "ms": ms,
                               "note": "record bytes written; the reads are dependent gathers (latency-bound)"}
    return out


def roofline(st: dict, workload: str) -> dict:
    """Roofline entry for the main kernel that took the longest in the last build."""
    ks = kernel_rooflines(st)
    k = max(ks, key=lambda name: ks[name]["ms"])
    r = dict(ks[k])
    r["kernel"] = k
    r["traffic"] = measured_traffic(k, workload)
    return r


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--precision", type=int, default=1, help="0 = float64 everywhere, 1 = float32 screens + "
                    "float64 re-decision (the plain float32 form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", type=int, default=1, help="1: the index autotunes its witness-pivot counts on "
                    "the first (warmup) build")
    ap.add_argument("--vgrng-pivots", type=int, default=0, help="Proposition 1 witness pivots per block (autotune 0)")
    ap.add_argument("--stage4-pivots", type=int, default=0, help="Stage IV pivot witnesses (autotune 0)")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle rows for the CPU baseline (0 = auto)")
    ap.add_argument("--queries", type=int, default=4096, help="queries timed against the built index (0 = none)")
    ap.add_argument("--workload", default="clustered", choices=["clustered", "subspace3"],
                    help="clustered: the 100k x 16-D two-layer build (the benchmark); subspace3: the 1M x 32-D "
                         "three-layer build (100 coarse, 3,000 fine pivots)")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (scales rocprofv3 FETCH/WRITE counters)")
    ap.add_argument("--attainable", action="store_true",
                    help="only measure attainable peaks: device copy bandwidth and a float64 library GEMM")
    return ap.parse_args()


def cpu_baseline(W, rows_hint: int):
    """The oracle (C, OpenMP) on a bounded sample: RNG rows of sampled points, scaled to all N rows."""
    import numpy as np

    from oracle import native
    native.build(force=False)
    threads = native.default_threads()
    g = np.random.default_rng(7)
    rows = rows_hint or 64
    xs = g.choice(W.n, rows, replace=False)
    t0 = time.perf_counter()
    native.rng_rows(W.X, W.q, xs, threads=threads)
    dt = time.perf_counter() - t0
    if not rows_hint and dt < 5.0:   # grow to roughly 10-30 s of CPU work
        rows = int(min(W.n, max(rows, rows * 12.0 / max(dt, 1e-3))))
        xs = g.choice(W.n, rows, replace=False)
        t0 = time.perf_counter()
        native.rng_rows(W.X, W.q, xs, threads=threads)
        dt = time.perf_counter() - t0
    est = dt * W.n / rows
    return {"value": est, "unit": "s", "cores": threads, "kind": "oracle",
            "sample": "RNG rows of %d random points (each row scans all %d points), %.2f s measured, "
                      "scaled by N/rows to the full build" % (rows, W.n, dt)}


def query_throughput(idx, W, nq: int) -> dict:
    """RNG neighbours of nq fresh points of the same mixture against the built
    index (device-resident queries; the index is unchanged)."""
    import numpy as np
    import torch

    import synth
    Q = torch.from_numpy(synth.queries_like(W, nq, sub=2)).cuda()
    idx.query_neighbors(Q)   # sizes the output once
    torch.cuda.synchronize()
    times = []
    for _ in range(3):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        off, _ = idx.query_neighbors(Q)
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    st = idx.stats()
    ms = float(np.median(times))
    return {"nq": nq, "ms": ms, "queries_per_s": nq / (ms / 1e3), "neighbours": int(off[-1].item()),
            "distance_computations_per_query": st["distance_computations"] / nq,
            "witness_tests_per_query": st["witness_tests"] / nq}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the build has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    if args.copy_calibration_mb:
        src = torch.ones(args.copy_calibration_mb * (1 << 20) // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration_mb, "copies": 3}))
        return

    if args.attainable:
        print(json.dumps(attainable_peaks(torch)))
        return

    import synth
    import paper_2208_10022_amd as P

    dev = torch.device("cuda:0")
    W = synth.subspace3() if args.workload == "subspace3" else synth.clustered(n=args.n)
    X = torch.from_numpy(W.X).to(dev)
    layers = [(torch.from_numpy(L.pivot_ids).to(dev), torch.from_numpy(L.radii).to(dev)) for L in W.layers]
    torch.cuda.synchronize()

    def step(idx):
        for level, (pid, rad) in enumerate(layers):
            idx.build_grng_layer(level, pid, rad)
        idx.build_rng()

    idx = P.Index(X, grid_exp=W.q, precision=args.precision, autotune=args.autotune,
                  vgrng_pivots=args.vgrng_pivots, stage4_pivots=args.stage4_pivots)
    if args.autotune and args.warmup < 1:
        print("--autotune needs at least one warmup step (the tuning runs there)", file=sys.stderr)
        sys.exit(2)
    for _ in range(args.warmup):
        step(idx)
    torch.cuda.synchronize()
    times, stats = [], []
    stream = torch.cuda.current_stream()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        step(idx)
        e1.record(stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
        stats.append(idx.stats())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = float(np.median(times))
    st = stats[-1]
    edges = idx.num_edges()
    queries = query_throughput(idx, W, args.queries) if args.queries > 0 else None
    idx.close()

    sizes = [int(len(L.pivot_ids)) for L in W.layers]
    if args.workload == "subspace3":
        workload = "subspace3-n%d-d%d-m%d-p%d" % (W.n, W.d, sizes[-1], args.precision)
        described = ("three-layer GRNG->GRNG->RNG, N=%d, D=%d near an 8-D subspace, %d coarse and %d fine "
                     "pivots" % (W.n, W.d, sizes[0], sizes[-1]))
    else:
        workload = "clustered-n%d-d16-m1000-p%d" % (W.n, args.precision)
        described = ("two-layer GRNG->RNG, N=%d, D=16, 32 Gaussian clusters (sigma 0.5), 1,000 random pivots with "
                     "100-NN radii" % W.n)
    line = {
        "metric": "exact-RNG build time (s) & witness tests/s vs plain GPU form; MFMA%/HBM GB/s",
        "value": ms / 1000.0,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 0 else "f32",
        "data": "synthetic",
        "config": {"workload": described,
                   "n": W.n, "d": W.d, "pivots": sizes[-1] if len(sizes) == 1 else sizes, "grid_exp": W.q,
                   "precision": "float64 distances" if args.precision == 0 else
                   "float32 screens, float64 re-decision of doubtful comparisons"},
        "edges": edges,
        "witness_tests": st["witness_tests"],
        "witness_tests_per_s": st["witness_tests"] / (ms / 1000.0),
        "lune_tests_per_s": st["lune_tests"] / (st["ms_lune"] / 1000.0) if st["ms_lune"] > 0 else None,
        # the work pruning avoids: every pair, and every (pair, witness) test
        "dense_pairs": W.n * (W.n - 1) // 2,
        "dense_tests": W.n * (W.n - 1) * (W.n - 2) // 2,
        "distance_computations": st["distance_computations"],
        "candidate_pairs": st["candidate_pairs"],
        "stage4_survivors": st["stage4_survivors"],
        "exhaustive_pairs": st["exhaustive_pairs"],
        "lune_tests": st["lune_tests"],
        "rechecks": st["rechecks"],
        "tile_pairs": st["tile_pairs"],
        "vgrng_pivots": st["vgrng_pivots"],
        "stage4_pivots": st["stage4_pivots"],
        "ms_autotune_once": st["ms_autotune"],
        "orphans": st["orphans"],
        "ms_layer": st["ms_layers"],
        "ms_rng": st["ms_rng"],
        "ms_vgrng": st["ms_vgrng"],
        "ms_pair_masks": st["ms_pair_masks"],
        "ms_pairs": st["ms_pairs"],
        "ms_lune": st["ms_lune"],
        "queries": queries,
        "roofline": roofline(st, workload),
        "kernels": kernel_rooflines(st),
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, args.cpu_rows)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
