#!/usr/bin/env python3
"""Throughput of the real-space spherical convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step is one pass of the whole hot path over synthetic inputs already
resident in HBM (white-noise maps, the flat-spectrum inputs of the paper's
Sec. 3):

  fwd      Nside 2048, one map, Gaussian beam FWHM 5 arcmin, 16384-node table,
           theta_cut swept over 10, 15 and 20 arcmin (three plain launches);
  fwdbwd   Nside 2048, theta_cut 15 arcmin, 256 learnable knots: forward, then
           the fused adjoint (d/dmap and d/dknots);
  batch    16 maps of Nside 256..2048 and FWHM 5..30 arcmin (cut 3 FWHM) in one
           persistent launch, replayed from a captured graph.

The unit of work is one in-disc pair term (theta_pq < theta_cut), counted
exactly by the plan; `value` is total pairs / total step time, in
GPair-evals/s.  Rank 0 prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GPair-evals/s and maps/s at Nside 2048 (fwd, fwd+bwd, batched) vs plain kernel"
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0
# Algorithmic FP32 work of one pair term of the per-pair gather: longitude
# difference, sine series, chord, angle series, table index, interpolation
# and the accumulating FMA.
FLOP_PER_PAIR = 24.0
PROFILES = os.path.join(ROOT, "profiles")


def _kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "arkcos_internal.hpp"):
        with open(os.path.join(ROOT, "paper_1211_3556_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str):
    """Per-launch HBM bytes of `kernel` from the committed rocprofv3 counter
    summary, or None if absent or taken on different kernel sources."""
    path = os.path.join(PROFILES, "hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != _kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain-compare", action="store_true",
                    help="skip the 16 plain launches the batch is compared with")
    ap.add_argument("--cpu-sample", type=int, default=6_000_000,
                    help="output pixels of the Nside-2048 oracle sample")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        return 2

    import torch
    import paper_1211_3556_amd as A
    import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    # ---------------------------------------------------------------- setup --
    def table(spec):
        return A.tabulate_legendre(A.gaussian_bl(spec.fwhm, spec.ell_max), spec.theta_cut,
                                   spec.ntab)

    log("building plans")
    fwd_specs = list(W.C3)
    fwd_plans = [A.Plan(s.nside, s.theta_cut, table(s)) for s in fwd_specs]
    x2048 = torch.from_numpy(W.white_noise(2048, fwd_specs[0].seed).astype(np.float32)).to(dev)
    fwd_out = [torch.empty_like(x2048) for _ in fwd_plans]
    fwd_pairs = [p.pair_count() for p in fwd_plans]

    gspec = W.MapSpec(nside=2048, fwhm=5.0 * W.ARCMIN, theta_cut=15.0 * W.ARCMIN, ntab=256,
                      seed=3)
    gplan = A.Plan(gspec.nside, gspec.theta_cut, ntab=gspec.ntab, learnable=True)
    knots = torch.from_numpy(W.gaussian_profile_knots(gspec.fwhm, gspec.theta_cut,
                                                      gspec.ntab).astype(np.float32)).to(dev)
    gplan.set_knots(knots)
    gin = torch.from_numpy(W.white_noise(2048, 13).astype(np.float32)).to(dev)
    g_out = torch.empty_like(x2048)
    g_pairs = gplan.pair_count()

    bspecs = W.batch_specs()
    bplans = [A.Plan(s.nside, s.theta_cut, table(s)) for s in bspecs]
    bx = [torch.from_numpy(W.white_noise(s.nside, s.seed).astype(np.float32)).to(dev)
          for s in bspecs]
    by = [torch.empty_like(x) for x in bx]
    batch = A.Batch(bplans)
    b_pairs = sum(p.pair_count() for p in bplans)
    torch.cuda.synchronize()

    # capture the batched launch in a graph (replayed each step)
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        batch.convolve(bx, by)
    stream.wait_stream(side)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        batch.convolve(bx, by)
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    times = {"fwd": [], "fwdbwd_fwd": [], "fwdbwd_bwd": [], "batch": []}
    fwd_launch_ms = []

    def step(record: bool):
        for p, o, np_ in zip(fwd_plans, fwd_out, fwd_pairs):
            e0, e1 = ev(), ev()
            e0.record(stream)
            p.convolve(x2048, o)
            e1.record(stream)
            if record:
                times["fwd"].append((e0, e1))
        e0, e1, e2 = ev(), ev(), ev()
        e0.record(stream)
        gplan.convolve(x2048, g_out)
        e1.record(stream)
        gplan.backward(gin, x2048, want_map=True, want_knots=True)
        e2.record(stream)
        if record:
            times["fwdbwd_fwd"].append((e0, e1))
            times["fwdbwd_bwd"].append((e1, e2))
        e0, e1 = ev(), ev()
        e0.record(stream)
        graph.replay()
        e1.record(stream)
        if record:
            times["batch"].append((e0, e1))

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    def mean_ms(key):
        return float(np.mean([a.elapsed_time(b) for a, b in times[key]]))

    fwd_ms = [float(np.mean([a.elapsed_time(b) for a, b in times["fwd"][i::3]]))
              for i in range(3)]
    fb_f, fb_b, b_ms = mean_ms("fwdbwd_fwd"), mean_ms("fwdbwd_bwd"), mean_ms("batch")
    step_pairs = sum(fwd_pairs) + 2 * g_pairs + b_pairs
    ms_per_step = 1e3 * wall / args.steps
    value = step_pairs / (wall / args.steps) / 1e9

    plain16_ms = None
    if not args.no_plain_compare:
        log("16 plain launches for comparison")
        e0, e1 = ev(), ev()
        e0.record(stream)
        for p, x, y in zip(bplans, bx, by):
            p.convolve(x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        plain16_ms = e0.elapsed_time(e1)

    # dominant kernel of the step: the batched gather
    parts_ms = {"fwd": sum(fwd_ms), "fwdbwd": fb_f + fb_b, "batch": b_ms}
    dom = max(parts_ms, key=parts_ms.get)
    if dom == "batch":
        kname, dom_pairs, dom_ms = "k_batch", b_pairs, b_ms
    elif dom == "fwd":
        kname, dom_pairs, dom_ms = "k_forward<1>", sum(fwd_pairs) / 3, sum(fwd_ms) / 3
    else:
        kname, dom_pairs, dom_ms = "k_backward<1,1,1>", g_pairs, fb_b
    achieved = FLOP_PER_PAIR * dom_pairs / (dom_ms * 1e-3) / 1e12
    traffic = _traffic(kname)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        s = fwd_specs[2]
        k64 = O.tabulate(O.gaussian_bl(s.fwhm, s.ell_max), s.theta_cut, s.ntab)
        x64 = W.white_noise(s.nside, s.seed)
        pix = np.sort(np.random.default_rng(s.seed + 10_000).choice(
            s.npix, size=args.cpu_sample, replace=False))
        log("oracle on %d pixels" % pix.size)
        t = time.perf_counter()
        _, pairs = O.convolve(s.nside, s.theta_cut, k64, x64, pixels=pix, return_pairs=True)
        dt = time.perf_counter() - t
        cpu = {"value": float(pairs.sum()) / dt / 1e9, "unit": "GPair-evals/s",
               "cores": O.threads(), "kind": "oracle",
               "sample": "Nside 2048, FWHM 5', theta_cut 20', %d random output pixels "
                         "(%d pairs, %.1f s); FP64 C/OpenMP" % (pix.size, int(pairs.sum()), dt)}

    maps_per_step = len(fwd_plans) + 1 + len(bplans)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GPair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "step = Nside-2048 fwd at theta_cut 10/15/20' + Nside-2048 fwd+bwd "
                        "(15', 256 knots) + 16-map batch (Nside 256-2048, FWHM 5-30', 3 FWHM "
                        "cut) in one graph-replayed launch; white-noise FP32 maps",
            "pairs_per_step": int(step_pairs),
            "maps_per_step": maps_per_step,
        },
        "breakdown": {
            "fwd": {"theta_cut_arcmin": [10, 15, 20], "ms": [round(m, 4) for m in fwd_ms],
                    "pairs": fwd_pairs,
                    "gpair_per_s": [round(p / (m * 1e-3) / 1e9, 2) for p, m in zip(fwd_pairs, fwd_ms)],
                    "maps_per_s": [round(1e3 / m, 1) for m in fwd_ms]},
            "fwdbwd": {"ms_fwd": round(fb_f, 4), "ms_bwd": round(fb_b, 4),
                       "pairs": 2 * g_pairs,
                       "gpair_per_s": round(2 * g_pairs / ((fb_f + fb_b) * 1e-3) / 1e9, 2),
                       "maps_per_s": round(1e3 / (fb_f + fb_b), 1)},
            "batch": {"ms": round(b_ms, 4), "pairs": int(b_pairs),
                      "gpair_per_s": round(b_pairs / (b_ms * 1e-3) / 1e9, 2),
                      "maps_per_s": round(16e3 / b_ms, 1),
                      "plain16_ms": None if plain16_ms is None else round(plain16_ms, 4),
                      "speedup_vs_plain16": None if plain16_ms is None else round(plain16_ms / b_ms, 3)},
        },
        "roofline": {
            "kernel": kname,
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic,
            "flop_per_pair": FLOP_PER_PAIR,
            "avg_launch_ms": round(dom_ms, 4),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
