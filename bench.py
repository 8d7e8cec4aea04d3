"""Benchmark of the exact GRNG-guided RNG build on one MI355X.

Default workload (the largest single-GPU configuration): 1,000,000 points in
32-D near a random 8-dimensional subspace (noise sigma 0.01, 2^-21 grid), a
three-layer hierarchy of 100 coarse and 3,000 fine pivots (the coarse layer a
subset of the fine one).  One step = build the GRNG of both pivot layers,
then the exact RNG of all points, in the bf16 form (bf16 MFMA distance tiles
with a per-tile error bound in the pair kernel; every kept/eliminated
decision exact).  After the timed steps the plain float32 form builds the
same graph once; its time and its edge set (compared in full) go into the
line's "forms" object.  Inputs (points, pivot ids, radii) are resident in
device memory before timing starts.

Other workloads (--workload), each printing its own line:
  clustered    100k x 16-D, 32 clusters, 1,000 pivots (plain float32 form),
               plus RNG-neighbour query throughput;
  clustered96  1M x 96-D, 256 clusters, 10,000 pivots: the learned and the
               lune visit orders against the distance order;
  insert       64 batches into the 100k index: the incremental insertion
               against a rebuild at every batch;
  hierarchy    number of layers and pivot counts over 300k x 32-D points;
  pivots       200 orphans of the 100k index promoted to pivots with
               insert_pivots, against a rebuild with the merged pivots.

Prints one JSON line.  ``--gpus N`` with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks (dense), and the VALU rates derived from unit counts:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz = 39.3e12 lane-operations/s (one
# 32-bit min, max or compare per lane per cycle) and twice that in float32
# flops for fused multiply-adds (78.6 TFLOP/s; packed FP32 is not used).
MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6
MI355X_BF16_TFLOPS = 2500.0
MI355X_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
MI355X_FP32_VALU_TFLOPS = 2 * MI355X_VALU_TOPS

PRECISION_NAMES = {0: "float64 tiles and scan", 1: "float64 MFMA tiles, float32 screens with float64 re-decision",
                   2: "bf16 MFMA tiles (two-part split, float32 accumulation) with a per-tile error bound, "
                      "float32 screens with float64 re-decision"}
PRECISION_DTYPE = {0: "f64", 1: "f64", 2: "bf16"}
PAIR_KERNEL = {0: "k_pairs_tiled", 1: "k_pairs_tiled", 2: "k_pairs_bf16"}

KERNEL_SOURCES = {"k_pairs_tiled": ["k_rng.hip", "dev_util.h", "common.h"],
                  "k_pairs_bf16": ["k_pairs_bf16.hip", "dev_util.h", "common.h"],
                  "k_pair_masks": ["k_rng.hip", "dev_util.h", "common.h"],
                  "k_lune_guided": ["k_rng.hip", "dev_util.h", "common.h"],
                  "k_partner_witness": ["k_rng.hip", "dev_util.h", "common.h"],
                  "k_vgrng_tiles": ["k_pivots.hip", "common.h"]}


def source_hash(kernel: str) -> str:
    """sha256 of the sources a kernel is built from (to tell whether measured counters still apply)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2208_10022_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per build from the committed rocprofv3 counter summary, if it
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


def _entry(bound, achieved, peak, unit, ms, **extra):
    r = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak, "ms": ms}
    r.update(extra)
    return r


def kernel_rooflines(st: dict, d: int, precision: int) -> dict:
    """Per main kernel of the last build: the roof that binds it at peak, and
    the achieved fraction, from algorithmic work only.

    pair kernel   two roofs.  Matrix cores: the squared distances the method
                  uses (candidate pairs, the pivot blocks, the Stage V witness
                  matrices: pair_method_distances), 2 d flops each, against the
                  MFMA peak of the tiles' type (bf16 or float64).  VALU: the
                  Stage IV (min,max) product, one max and one min per
                  (candidate pair, pivot witness).  The binding roof is the one
                  with the longer time at peak; the other is reported beside
                  it, with the dense-tile flops the kernel actually issues.
    k_lune_guided one witness test = two squared distances of d coordinates
                  (a subtraction and a fused multiply-add each), 4 d float32
                  flops, against the float32 VALU rate (the witness rows are
                  served from cache; HBM bytes are in 'traffic').
    k_partner_witness  (with the top-64 selection before it, in ms_partner) one
                  witness test = one squared distance of d coordinates, 3 d
                  float32 flops (the other end's distance is known), against
                  the float32 VALU rate.
    k_vgrng_tiles (min,max) product: 2 ops per (point, pivot j, witness k)
                  for each of two radius choices = 2 * vgrng_ops.
    k_pair_masks  one 1,120-byte record written per tile pair.
    """
    out = {}
    pk = PAIR_KERNEL[precision]
    ms = st["ms_pairs"]
    flops = st["pair_method_distances"] * 2.0 * d
    mfma_peak = MI355X_BF16_TFLOPS if precision == 2 else MI355X_FP64_TFLOPS
    kp = (d + 31) // 32 * 32 if precision == 2 else (d + 3) // 4 * 4
    dense = st["pair_tile_entries"] * 2.0 * kp * (3 if precision == 2 else 1)
    valu_ops = 2.0 * st["candidate_pairs"] * st["stage4_pivots"]
    t_mfma = flops / (mfma_peak * 1e12)
    t_valu = valu_ops / (MI355X_VALU_TOPS * 1e12)
    mfma_view = {"achieved": flops / (ms / 1e3) / 1e12, "peak": mfma_peak, "unit": "TFLOP/s",
                 "frac": t_mfma / (ms / 1e3), "dense_tile_tflop_s": dense / (ms / 1e3) / 1e12}
    valu_view = {"achieved": valu_ops / (ms / 1e3) / 1e12, "peak": MI355X_VALU_TOPS, "unit": "Tops/s",
                 "frac": t_valu / (ms / 1e3)}
    if t_mfma >= t_valu:
        out[pk] = _entry("mfma", mfma_view["achieved"], mfma_peak, "TFLOP/s", ms, valu=valu_view,
                         dense_tile_tflop_s=mfma_view["dense_tile_tflop_s"])
    else:
        out[pk] = _entry("alu", valu_view["achieved"], MI355X_VALU_TOPS, "Tops/s", ms, mfma=mfma_view)
    ms = st["ms_lune"]
    if ms > 0:
        fl = st["lune_tests"] * 4.0 * d
        out["k_lune_guided"] = _entry("alu", fl / (ms / 1e3) / 1e12, MI355X_FP32_VALU_TFLOPS, "TFLOP/s", ms)
    ms = st.get("ms_partner", 0.0)
    if ms > 0:
        fl = st["partner_tests"] * 3.0 * d
        out["k_partner_witness"] = _entry("alu", fl / (ms / 1e3) / 1e12, MI355X_FP32_VALU_TFLOPS, "TFLOP/s", ms,
                                          kills=st["partner_kills"])
    ms = st["ms_vgrng"]
    if ms > 0:
        ach = 2.0 * st["vgrng_ops"] / (ms / 1e3) / 1e12
        out["k_vgrng_tiles"] = _entry("alu", ach, MI355X_VALU_TOPS, "Tops/s", ms)
    ms = st["ms_pair_masks"]
    if ms > 0:
        ach = PAIR_RECORD_BYTES * st["tile_pairs"] / (ms / 1e3) / 1e9
        out["k_pair_masks"] = _entry("hbm", ach, MI355X_HBM_GBS, "GB/s", ms,
                                     note="record bytes written; the reads are dependent gathers")
    return out


def roofline(st: dict, d: int, precision: int, workload: str) -> dict:
    """Roofline entry of the main kernel that took the longest in the last build."""
    ks = kernel_rooflines(st, d, precision)
    k = max(ks, key=lambda name: ks[name]["ms"])
    r = dict(ks[k])
    r["kernel"] = k
    r["traffic"] = measured_traffic(k, workload)
    return r


def kernels_with_traffic(ks: dict, workload: str) -> dict:
    """Each kernel's entry with its measured HBM bytes per build and the
    rate they imply (null while the committed counters do not match the
    kernel's sources or this workload)."""
    for k, r in ks.items():
        t = measured_traffic(k, workload)
        r["traffic"] = t
        r["hbm_gb_s"] = t / (r["ms"] / 1e3) / 1e9 if t is not None and r["ms"] > 0 else None
    return ks


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(W, rows_hint: int, target_s: float = 15.0):
    """The C oracle (OpenMP, every host core) on a bounded sample: RNG rows of
    random points deciding only their neighbours y > x (the share of each row
    the full-edge oracle decides), scaled by N / rows to the full build."""
    import numpy as np

    from oracle import native
    native.build(force=False)
    threads = native.default_threads()
    K = native.grid_ints32(W.X, W.q)
    g = np.random.default_rng(7)
    rows = rows_hint or 4 * threads
    xs = g.choice(W.n, rows, replace=False)
    t0 = time.perf_counter()
    native.rng_rows_compact(W.X, W.q, xs, threads=threads, upper=True, K=K)
    dt = time.perf_counter() - t0
    if not rows_hint and dt < target_s / 3:   # grow to about target_s of CPU work
        rows = int(min(W.n, max(rows, rows * target_s / max(dt, 1e-3))))
        xs = g.choice(W.n, rows, replace=False)
        t0 = time.perf_counter()
        native.rng_rows_compact(W.X, W.q, xs, threads=threads, upper=True, K=K)
        dt = time.perf_counter() - t0
    return {"value": dt * W.n / rows, "unit": "s", "cores": threads, "kind": "oracle", "cpu": cpu_model(),
            "sample": "RNG rows of %d random points, each deciding its neighbours y > x over all %d points "
                      "(as the full oracle does), %.2f s measured on %d threads, scaled by N/rows to the "
                      "full build" % (rows, W.n, dt, threads)}


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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="subspace3",
                    choices=["subspace3", "clustered", "clustered96", "insert", "hierarchy", "pivots"])
    ap.add_argument("--precision", type=int, default=-1, help="0 = float64 everywhere, 1 = float32 screens "
                    "(the plain float32 form), 2 = bf16 tiles, 3 = float32 screens with the pair kernel's tile "
                    "shape (float64 or bf16 tiles) chosen by the autotuner; -1 = the workload's form (3 for "
                    "subspace3, else 1)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the comparison builds of the other forms")
    ap.add_argument("--form-warmup", type=int, default=1, help="untimed builds before each form's timed one")
    ap.add_argument("--autotune", type=int, default=1, help="1: the index autotunes its witness-pivot counts on "
                    "the first (warmup) build")
    ap.add_argument("--vgrng-pivots", type=int, default=0, help="Proposition 1 witness pivots per block (autotune 0)")
    ap.add_argument("--stage4-pivots", type=int, default=0, help="Stage IV pivot witnesses (autotune 0)")
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle rows for the CPU baseline (0 = auto)")
    ap.add_argument("--queries", type=int, default=4096, help="clustered: queries timed against the built index")
    ap.add_argument("--copy-calibration-mb", type=int, default=0,
                    help="only run a plain device copy of this many MiB (scales rocprofv3 FETCH/WRITE counters)")
    ap.add_argument("--attainable", action="store_true",
                    help="only measure attainable peaks: device copy bandwidth and a float64 library GEMM")
    return ap.parse_args()


def workload_of(name):
    import synth
    if name == "subspace3":
        W = synth.subspace3()
        sizes = [len(L.pivot_ids) for L in W.layers]
        desc = ("three-layer GRNG->GRNG->RNG, N=%d, D=%d near an 8-D subspace (noise 0.01), %d coarse and %d fine "
                "pivots" % (W.n, W.d, sizes[0], sizes[1]))
    elif name == "clustered96":
        W = synth.clustered(n=1_000_000, d=96, clusters=256, sigma=1.0, m=10_000, knn=100, q=18)
        desc = "two-layer GRNG->RNG, N=%d, D=96, 256 Gaussian clusters (sigma 1.0), 10,000 pivots with 100-NN radii" % W.n
    else:
        W = synth.clustered()
        desc = ("two-layer GRNG->RNG, N=%d, D=16, 32 Gaussian clusters (sigma 0.5), 1,000 random pivots with 100-NN "
                "radii" % W.n)
    return W, desc


class Builder:
    """One index over device-resident points and pivot layers; step() builds
    every layer and the RNG (timed with device events on the current stream)."""

    def __init__(self, P, W, **kw):
        import torch
        self.torch = torch
        self.X = torch.from_numpy(W.X).cuda()
        self.layers = [(torch.from_numpy(L.pivot_ids).cuda(), torch.from_numpy(L.radii).cuda()) for L in W.layers]
        self.idx = P.Index(self.X, grid_exp=W.q, **kw)

    def step(self):
        for level, (pid, rad) in enumerate(self.layers):
            self.idx.build_grng_layer(level, pid, rad)
        self.idx.build_rng()

    def timed(self):
        torch = self.torch
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        self.step()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1)


def progress(what, **kw):
    """A progress line on stderr (a C5 build runs for about 100 s)."""
    print(json.dumps(dict({"progress": what}, **kw)), file=sys.stderr, flush=True)


def other_form(P, W, precision, st, witness_order=0, scorer=None, warmup=1):
    """One build (after `warmup` untimed ones) of another form with the
    witness-pivot counts the timed index settled on: (ms, edges as a host
    array, stats)."""
    b = Builder(P, W, precision=precision, autotune=0, witness_order=witness_order,
                vgrng_pivots=int(st["vgrng_pivots"]), stage4_pivots=int(st["stage4_pivots"]))
    if scorer is not None:
        b.idx.set_scorer(scorer)
    for _ in range(warmup):
        b.step()
    ms = b.timed()
    progress("form", precision=precision, witness_order=witness_order, ms=ms)
    E = b.idx.edges().cpu().numpy()
    s2 = b.idx.stats()
    b.idx.close()
    return ms, E, s2


def form_entry(ms, st, same, base_ms):
    return {"ms": ms, "speedup_vs_plain": base_ms / ms, "identical_edges": bool(same),
            "exhaustive_pairs": st["exhaustive_pairs"], "lune_tests": st["lune_tests"],
            "lune_tests_kept": st["lune_tests_kept"], "partner_kills": st["partner_kills"],
            "ms_partner": st["ms_partner"], "rechecks": st["rechecks"],
            "screen_uncertain": st["screen_uncertain"], "ms_pairs": st["ms_pairs"], "ms_lune": st["ms_lune"]}


def train_scorer(P):
    """Scorer trained on witness-cell logs of the 100k x 16-D build and of a
    small 2-D build (the learned form's training set)."""
    import numpy as np
    import torch

    import synth
    feats, labels = [], []
    for W in (synth.clustered(), synth.clustered(n=20000, d=2, clusters=16, m=200, knn=50, q=19, sub=3)):
        b = Builder(P, W, precision=1)
        b.step()
        f, lab = b.idx.log_witness_cells(20000)
        feats.append(f)
        labels.append(lab)
        b.idx.close()
    feats, labels = torch.cat(feats), torch.cat(labels)
    theta = torch.from_numpy((np.random.default_rng(1).standard_normal(P.mlp_params()) * 0.1)
                             .astype(np.float32)).cuda()
    t0 = time.perf_counter()
    loss = P.mlp_train(theta, feats, labels, steps=400, lr=3e-3)
    progress("scorer trained", loss=loss)
    return theta, {"samples": int(feats.shape[0]), "loss": loss, "train_s": time.perf_counter() - t0}


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
    if args.workload == "insert":
        return bench_insert(args)
    if args.workload == "hierarchy":
        return bench_hierarchy(args)
    if args.workload == "pivots":
        return bench_pivots(args)

    import paper_2208_10022_amd as P

    # 1M x 32-D: the autotuner picks the pair kernel's tile shape (float64 or
    # split bf16 MFMA tiles) with the witness-pivot counts
    auto = args.precision == 3 or (args.precision < 0 and args.workload == "subspace3")
    prec = 3 if auto else (args.precision if args.precision >= 0 else 1)
    W, desc = workload_of(args.workload)
    scorer, train = None, None
    if args.workload == "clustered96":
        scorer, train = train_scorer(P)
    b = Builder(P, W, precision=prec, autotune=args.autotune, vgrng_pivots=args.vgrng_pivots,
                stage4_pivots=args.stage4_pivots)
    if args.autotune and args.warmup < 1:
        print("--autotune needs at least one warmup step (the tuning runs there)", file=sys.stderr)
        sys.exit(2)
    for _ in range(args.warmup):
        b.step()
        progress("warmup step")
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        times.append(b.timed())
        progress("timed step", ms=times[-1])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms = float(np.median(times))
    st = b.idx.stats()
    prec = int(st["precision_used"])   # the form that ran (the tuner's choice under automatic precision)
    E = b.idx.edges().cpu().numpy()
    queries = query_throughput(b.idx, W, args.queries) if args.workload == "clustered" and args.queries else None
    b.idx.close()

    forms = None
    if not args.no_forms:
        forms = {"plain_float32": None}
        if prec == 1:
            base_ms, base_st = ms, st
        else:
            base_ms, E1, base_st = other_form(P, W, 1, st, warmup=args.form_warmup)
            forms["plain_float32"] = form_entry(base_ms, base_st, np.array_equal(E1, E), base_ms)
        if prec == 2:
            forms["bf16"] = form_entry(ms, st, forms["plain_float32"]["identical_edges"], base_ms)
        elif args.workload == "clustered":
            ms2, E2, st2 = other_form(P, W, 2, st, warmup=args.form_warmup)
            forms["bf16"] = form_entry(ms2, st2, np.array_equal(E2, E), base_ms)
        if args.workload == "clustered96":
            forms["plain_float32"] = form_entry(ms, st, True, ms)
            ms_l, E_l, st_l = other_form(P, W, 1, st, witness_order=P.ORDER_LEARNED, scorer=scorer,
                                         warmup=args.form_warmup)
            forms["learned"] = form_entry(ms_l, st_l, np.array_equal(E_l, E), ms)
            forms["learned"]["scorer"] = train
            ms_u, E_u, st_u = other_form(P, W, 1, st, witness_order=P.ORDER_LUNE, warmup=args.form_warmup)
            forms["lune_order"] = form_entry(ms_u, st_u, np.array_equal(E_u, E), ms)
        if forms["plain_float32"] is None:
            forms["plain_float32"] = form_entry(base_ms, base_st, True, base_ms)

    sizes = [int(len(L.pivot_ids)) for L in W.layers]
    workload = "%s-n%d-d%d-m%s-p%d" % (args.workload, W.n, W.d, "-".join(map(str, sizes)), prec)
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
        "dtype": PRECISION_DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": desc, "n": W.n, "d": W.d, "pivots": sizes if len(sizes) > 1 else sizes[0],
                   "grid_exp": W.q, "precision": PRECISION_NAMES[prec] + (
                       " (tile shape chosen by the autotuner)" if auto and args.autotune else
                       " (tile shape chosen from the padded dimension)" if auto else "")},
        "edges": int(st["n_edges"]),
        "forms": forms,
        "witness_tests": st["witness_tests"],
        "witness_tests_per_s": st["witness_tests"] / (ms / 1000.0),
        "lune_tests_per_s": st["lune_tests"] / (st["ms_lune"] / 1000.0) if st["ms_lune"] > 0 else None,
        "stage4_tests_per_s": st["candidate_pairs"] * st["stage4_pivots"] / (st["ms_pairs"] / 1000.0),
        # the work pruning avoids: every pair, and every (pair, witness) test
        "dense_pairs": W.n * (W.n - 1) // 2,
        "dense_tests": W.n * (W.n - 1) * (W.n - 2) // 2,
        "distance_computations": st["distance_computations"],
        "candidate_pairs": st["candidate_pairs"],
        "stage4_survivors": st["stage4_survivors"],
        "exhaustive_pairs": st["exhaustive_pairs"],
        "lune_tests": st["lune_tests"],
        "lune_tests_kept": st["lune_tests_kept"],
        "partner_tests": st["partner_tests"],
        "partner_kills": st["partner_kills"],
        "ms_partner": st["ms_partner"],
        "rechecks": st["rechecks"],
        "screen_uncertain": st["screen_uncertain"],
        "tile_pairs": st["tile_pairs"],
        "vgrng_pivots": st["vgrng_pivots"],
        "stage4_pivots": st["stage4_pivots"],
        "ms_autotune_once": st["ms_autotune"],
        "orphans": st["orphans"],
        "ms_layers_last": st["ms_layers"],
        "ms_rng": st["ms_rng"],
        "ms_vgrng": st["ms_vgrng"],
        "ms_pair_masks": st["ms_pair_masks"],
        "ms_pairs": st["ms_pairs"],
        "ms_lune": st["ms_lune"],
        "queries": queries,
        "roofline": roofline(st, W.d, prec, workload),
        "kernels": kernels_with_traffic(kernel_rooflines(st, W.d, prec), workload),
        "wall_s": wall,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(W, args.cpu_rows)
    print(json.dumps(line), flush=True)


def bench_insert(args):
    """64 batches (log-uniform sizes in [1,000, 50,000]) into the 100k x 16-D
    index: incremental insertion against a rebuild from scratch after every
    batch, edges compared in full."""
    import numpy as np
    import torch

    import paper_2208_10022_amd as P
    import synth
    W, desc = workload_of("clustered")
    batches = synth.insert_batches(W)
    b = Builder(P, W, precision=1)
    b.step()
    tune = b.idx.stats()
    ins_ms, reb_ms, same = [], [], True
    allX = [W.X]
    for B in batches:
        Bd = torch.from_numpy(B).cuda()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.idx.insert_batch(Bd)
        e1.record()
        e1.synchronize()
        ins_ms.append(e0.elapsed_time(e1))
        allX.append(B)
        if args.no_forms:   # insertions only (e.g. under a profiler)
            progress("batch", n=len(allX) - 1, insert_ms=ins_ms[-1])
            continue
        Wb = synth.Workload(name="all", X=np.vstack(allX), q=W.q, layers=W.layers)
        r = Builder(P, Wb, precision=1, autotune=0, vgrng_pivots=int(tune["vgrng_pivots"]),
                    stage4_pivots=int(tune["stage4_pivots"]))
        r.step()
        reb_ms.append(r.timed())
        same = same and np.array_equal(r.idx.edges().cpu().numpy(), b.idx.edges().cpu().numpy())
        r.idx.close()
        progress("batch", n=len(allX) - 1, insert_ms=ins_ms[-1], rebuild_ms=reb_ms[-1])
    n_final = b.idx.stats()["n_points"]
    b.idx.close()
    total = sum(ins_ms)
    line = {
        "metric": "exact-RNG build time (s) & witness tests/s vs plain GPU form; MFMA%/HBM GB/s",
        "value": total / 1000.0, "unit": "s", "n_gpus": 1, "steps": len(batches), "warmup": 1,
        "ms_per_step": total / len(batches), "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "64 insertion batches (sizes log-uniform in [1000, 50000]) into the " + desc,
                   "n_final": int(n_final), "precision": PRECISION_NAMES[1]},
        "forms": None if args.no_forms else {
            "batched_insert_total_ms": total, "rebuild_total_ms": sum(reb_ms),
            "speedup_vs_rebuild": sum(reb_ms) / total, "identical_edges_after_every_batch": bool(same),
            "insert_ms": ins_ms, "rebuild_ms": reb_ms},
    }
    print(json.dumps(line), flush=True)


def bench_pivots(args):
    """Dynamic pivot layer on the 100k x 16-D index: 200 orphans (seeded
    choice) promoted to pivots with 100-NN radii by insert_pivots (the layer's
    GRNG updated in place, the per-point tables rebuilt against it), against
    building the merged layer and the RNG from scratch; layer and RNG edge
    sets compared in full."""
    import numpy as np
    import torch

    import paper_2208_10022_amd as P
    import synth
    W, desc = workload_of("clustered")
    L = W.layers[0]
    b = Builder(P, W, precision=1, autotune=0)
    b.step()
    b.step()
    orph = b.idx.orphans().cpu().numpy()
    g = np.random.default_rng(2208)
    promote = np.sort(g.choice(orph, min(200, len(orph)), replace=False)).astype(np.int32)
    prad = synth.knn_radii(W.X, W.q, promote, 100)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pid, rad = torch.from_numpy(promote).cuda(), torch.from_numpy(prad).cuda()
    torch.cuda.synchronize()
    e0.record()
    b.idx.insert_pivots(0, pid, rad)
    e1.record()
    e1.synchronize()
    ins_ms = e0.elapsed_time(e1)
    orph_after = int(b.idx.orphans().numel())
    E_layer, E = b.idx.edges(0).cpu().numpy(), b.idx.edges().cpu().numpy()
    b.idx.close()
    ids = np.concatenate([L.pivot_ids, promote])
    rads = np.concatenate([L.radii, prad])
    order = np.argsort(ids)
    Wm = synth.Workload(name="merged", X=W.X, q=W.q,
                        layers=[synth.PivotLayer(ids[order].astype(np.int32), rads[order].astype(np.float32))])
    r = Builder(P, Wm, precision=1, autotune=0)
    r.step()
    reb_ms = r.timed()
    same = np.array_equal(r.idx.edges(0).cpu().numpy(), E_layer) and np.array_equal(r.idx.edges().cpu().numpy(), E)
    r.idx.close()
    line = {
        "metric": "exact-RNG build time (s) & witness tests/s vs plain GPU form; MFMA%/HBM GB/s",
        "value": ins_ms / 1000.0, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 2, "ms_per_step": ins_ms,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "%d orphans of the %s promoted to pivots" % (len(promote), desc),
                   "precision": PRECISION_NAMES[1]},
        "forms": {"insert_pivots_ms": ins_ms, "rebuild_ms": reb_ms, "speedup_vs_rebuild": reb_ms / ins_ms,
                  "identical_layer_and_rng_edges": bool(same), "orphans_before": int(len(orph)),
                  "orphans_after": orph_after, "pivots_before": int(len(L.pivot_ids)),
                  "pivots_after": int(len(ids))},
    }
    print(json.dumps(line), flush=True)


HIERARCHIES = [(1000,), (3000,), (10000,), (100, 3000), (300, 10000), (30, 300, 3000), (100, 1000, 10000)]


def bench_hierarchy(args):
    """Number of layers L and pivot counts M: 300k x 32-D points of the
    subspace law, built with each pivot hierarchy of HIERARCHIES (coarsest
    layer first); build time and the paper's cost unit (distance
    computations) per hierarchy, edges compared across all of them."""
    import numpy as np
    import torch

    import paper_2208_10022_amd as P
    import synth
    out, E0 = [], None
    for ms in HIERARCHIES:
        W = synth.subspace_layers(300_000, ms=ms)
        b = Builder(P, W, precision=1)
        b.step()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        layer_ms, layer_dist = [], 0.0
        for level, (pid, rad) in enumerate(b.layers):
            b.idx.build_grng_layer(level, pid, rad)
            s = b.idx.stats()
            layer_ms.append(s["ms_layers"])
            layer_dist += s["distance_computations"]
        b.idx.build_rng()
        e1.record()
        e1.synchronize()
        st = b.idx.stats()
        E = b.idx.edges().cpu().numpy()
        if E0 is None:
            E0 = E
        out.append({"pivots": list(ms), "layers": len(ms) + 1, "ms_total": e0.elapsed_time(e1),
                    "ms_layers": layer_ms, "ms_rng": st["ms_rng"],
                    "distance_computations": layer_dist + st["distance_computations"],
                    "witness_tests": st["witness_tests"], "candidate_pairs": st["candidate_pairs"],
                    "exhaustive_pairs": st["exhaustive_pairs"], "identical_edges": bool(np.array_equal(E, E0))})
        b.idx.close()
        print(json.dumps({"progress": out[-1]}), file=sys.stderr, flush=True)
    best = min(out, key=lambda r: r["ms_total"])
    line = {
        "metric": "exact-RNG build time (s) & witness tests/s vs plain GPU form; MFMA%/HBM GB/s",
        "value": best["ms_total"] / 1000.0, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["ms_total"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "pivot hierarchies over 300,000 points in 32-D near an 8-D subspace",
                   "precision": PRECISION_NAMES[1]},
        "best": best, "sweep": out,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
