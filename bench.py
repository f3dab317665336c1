#!/usr/bin/env python3
"""Throughput of the real-space spherical convolution on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step is one pass of the whole hot path over synthetic inputs already
resident in HBM (white-noise maps, the flat-spectrum inputs of the paper's
Sec. 3):

  fwd      Nside 2048, one map, Gaussian beam FWHM 5 arcmin, 16384-node table,
           theta_cut swept over 10, 15 and 20 arcmin;
  fwdbwd   Nside 2048, theta_cut 15 arcmin, 256 learnable knots: forward, then
           the adjoint (d/dmap: the same gathers on g) and the knot gradient;
           the knots are bound to the plan before each pass, as the autograd
           function does (node table and circulant weights rebuilt);
  grad     the differentiation workload: Nside 1024, 8 maps, theta_cut
           30 arcmin, 256 learnable knots, forward + adjoint + knot gradient
           with the same knot binding;
  batch    16 maps of Nside 256..2048 and FWHM 5..30 arcmin (cut 3 FWHM) as one
           batch, each of its two gathers one persistent launch replayed from
           a captured graph.

General-gather tile shapes come from the tuning cache the package ships
(python -m paper_1211_3556_amd.autotune); the breakdown says which plans used
tuned shapes.

Every gather launch is bracketed by HIP events on the stream it runs on, so
each kernel's launch time is measured inside the timed region.  The unit of
work is one in-disc pair term (theta_pq < theta_cut), counted exactly by the
plan; `value` is total pairs / total step time, in GPair-evals/s.  One JSON
line is printed.

Beside the step (not part of `value`), the breakdown reports the biased node
table of Sec. 3 against a uniform one, and the split convolution of the
paper's example: the l-space half (GPU spherical-harmonic transforms at
l_cut 1500) and the real-space half (240 arcmin cut) at Nside 2048.
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
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic FP32 work per in-disc pair term:
#   k_circ       one FMA with a precomputed weight (vector ALUs; k_circ_mfma
#                runs the same products on the matrix cores, for plans with
#                long rows);
#   k_general    one FMA, plus a 24-FLOP weight evaluation (longitude, sine
#                series, chord, angle series, table index, interpolation)
#                shared by the 16 quarter-turn, reflection and mirror images;
#   k_knot_circ  one FMA of the ring-pair cross-correlation (circulant rings;
#                the hat weights are applied once per distinct ring pair and
#                tap);
#   k_knot_gen   16 products g x per candidate plus ~44 FLOP of FP64 geometry
#                and hat weights, per 16 images (general rings).
FLOP_PER_PAIR = {"k_circ": 2.0, "k_circ_mfma": 2.0, "k_circ+k_circ_mfma": 2.0,
                 "k_general": 2.0 + 24.0 / 16.0,
                 "k_knot_circ": 2.0, "k_knot_gen": (32.0 + 44.0) / 16.0}
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
    ap.add_argument("--no-biased", action="store_true",
                    help="skip the biased-node-table forwards and the split convolution "
                         "reported beside the step")
    ap.add_argument("--no-large", action="store_true",
                    help="skip the Nside 4096 / 8192 forwards reported beside the step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one plain 256 MiB device-to-device copy, the reference "
                         "for scaling hardware byte counters")
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
    CIRC, GEN = A.PART_CIRCULANT, A.PART_GENERAL

    def log(msg):
        print("[bench] " + msg, file=sys.stderr, flush=True)

    def table(spec):
        return A.tabulate_legendre(A.gaussian_bl(spec.fwhm, spec.ell_max), spec.theta_cut,
                                   spec.ntab)

    def dev_map(nside, seed):
        return torch.from_numpy(W.white_noise(nside, seed).astype(np.float32)).to(dev)

    # ---------------------------------------------------------------- setup --
    log("building plans")
    fwd_specs = list(W.C3)
    fwd_plans = [A.Plan(s.nside, s.theta_cut, table(s)) for s in fwd_specs]
    x2048 = dev_map(2048, fwd_specs[0].seed)
    fwd_out = [torch.empty_like(x2048) for _ in fwd_plans]
    fwd_parts = [p.pair_count_parts() for p in fwd_plans]

    gspec = W.MapSpec(nside=2048, fwhm=5.0 * W.ARCMIN, theta_cut=15.0 * W.ARCMIN, ntab=256,
                      seed=3)
    gplan = A.Plan(gspec.nside, gspec.theta_cut, ntab=gspec.ntab, learnable=True)
    knots = torch.from_numpy(W.gaussian_profile_knots(gspec.fwhm, gspec.theta_cut,
                                                      gspec.ntab).astype(np.float32)).to(dev)
    gplan.set_knots(knots)
    gin = dev_map(2048, 13)
    g_out = torch.empty_like(x2048)
    g_gx = torch.empty_like(x2048)
    g_gk = torch.empty(gspec.ntab, dtype=torch.float32, device=dev)
    g_parts = gplan.pair_count_parts()
    g_pairs = sum(g_parts)

    # the differentiation workload: 8 maps of Nside 1024, 30 arcmin, 256 knots
    c5 = W.C5
    c5plan = A.Plan(c5.nside, c5.theta_cut, ntab=c5.nknots, max_batch=c5.nbatch, learnable=True)
    c5knots = torch.from_numpy(W.gaussian_profile_knots(c5.fwhm, c5.theta_cut,
                                                        c5.nknots).astype(np.float32)).to(dev)
    c5plan.set_knots(c5knots)
    c5x = torch.from_numpy(W.white_noise(c5.nside, c5.seed0, nbatch=c5.nbatch)
                           .astype(np.float32)).to(dev)
    c5g = torch.from_numpy(W.white_noise(c5.nside, c5.seed0 + 100, nbatch=c5.nbatch)
                           .astype(np.float32)).to(dev)
    c5y, c5gx = torch.empty_like(c5x), torch.empty_like(c5x)
    c5gk = torch.empty(c5.nknots, dtype=torch.float32, device=dev)
    c5_parts = c5plan.pair_count_parts()
    c5_pairs = c5.nbatch * sum(c5_parts)

    bspecs = W.batch_specs()
    bplans = [A.Plan(s.nside, s.theta_cut, table(s)) for s in bspecs]
    bx = [dev_map(s.nside, s.seed) for s in bspecs]
    by = [torch.empty_like(x) for x in bx]
    batch = A.Batch(bplans)
    b_parts = [p.pair_count_parts() for p in bplans]
    b_circ, b_gen = sum(c for c, _ in b_parts), sum(g for _, g in b_parts)
    torch.cuda.synchronize()

    # each gather of the batch as one captured graph, replayed every step
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        batch.convolve(bx, by)
    stream.wait_stream(side)
    graphs = {}
    for part in (CIRC, GEN):
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            batch.convolve(bx, by, part=part)
        graphs[part] = g
    torch.cuda.synchronize()

    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    launches = []   # (part of the step, kernel, algorithmic FLOP, start event, end event)

    def timed(record, part, kernel, flop, fn):
        e0, e1 = ev(), ev()
        e0.record(stream)
        fn()
        e1.record(stream)
        if record:
            launches.append((part, kernel, flop, e0, e1))

    def fl(kernel, pairs):
        return FLOP_PER_PAIR[kernel] * pairs

    def circ_kernel(plan):
        """The circulant gather's kernel: vector form or matrix-core form."""
        return "k_circ_mfma" if plan.info()["circ_form"] else "k_circ"

    fwd_ck = [circ_kernel(p) for p in fwd_plans]
    g_ck, c5_ck = circ_kernel(gplan), circ_kernel(c5plan)
    b_forms = {circ_kernel(p) for p in bplans}
    b_ck = "k_circ+k_circ_mfma" if len(b_forms) > 1 else b_forms.pop()

    def step(record: bool):
        for i, (p, o, (pc, pg)) in enumerate(zip(fwd_plans, fwd_out, fwd_parts)):
            timed(record, "fwd%d" % i, fwd_ck[i], fl(fwd_ck[i], pc),
                  lambda: p.convolve_part(x2048, o, CIRC))
            timed(record, "fwd%d" % i, "k_general", fl("k_general", pg),
                  lambda: p.convolve_part(x2048, o, GEN))
        def fwdbwd(part, plan, ck, knots, x, y, g, gx, gk, nb, parts):
            pc, pg = parts
            pc, pg = nb * pc, nb * pg
            # forward with the knots bound to the plan (table + circulant weights)
            timed(record, part, "k_set_knots", 0.0, lambda: plan.set_knots(knots))
            timed(record, part, ck, fl(ck, pc),
                  lambda: plan.convolve_part(x, y, CIRC))
            timed(record, part, "k_general", fl("k_general", pg),
                  lambda: plan.convolve_part(x, y, GEN))
            # backward: knots bound again; the operator is symmetric, so d/dmap
            # is the same two gathers on g
            timed(record, part, "k_set_knots", 0.0, lambda: plan.set_knots(knots))
            timed(record, part, ck, fl(ck, pc),
                  lambda: plan.convolve_part(g, gx, CIRC))
            timed(record, part, "k_general", fl("k_general", pg),
                  lambda: plan.convolve_part(g, gx, GEN))
            # knot gradient: correlation on circulant rings, per pair on general rings
            timed(record, part, "k_knot", fl("k_knot_circ", pc) + fl("k_knot_gen", pg),
                  lambda: plan.backward(g, x, want_map=False, want_knots=True, gk=gk))

        fwdbwd("fwdbwd", gplan, g_ck, knots, x2048, g_out, gin, g_gx, g_gk, 1, g_parts)
        fwdbwd("grad", c5plan, c5_ck, c5knots, c5x, c5y, c5g, c5gx, c5gk, c5.nbatch, c5_parts)
        timed(record, "batch", b_ck, fl(b_ck, b_circ), graphs[CIRC].replay)
        timed(record, "batch", "k_general", fl("k_general", b_gen), graphs[GEN].replay)

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

    ms = [(part, k, fl, a.elapsed_time(b)) for part, k, fl, a, b in launches]

    def part_ms(name):
        return sum(m for part, _, _, m in ms if part == name) / args.steps

    fwd_ms = [part_ms("fwd%d" % i) for i in range(3)]
    fb_ms, b_ms, c5_ms = part_ms("fwdbwd"), part_ms("batch"), part_ms("grad")
    fwd_pairs = [c + g for c, g in fwd_parts]
    step_pairs = sum(fwd_pairs) + 2 * g_pairs + 2 * c5_pairs + b_circ + b_gen
    ms_per_step = 1e3 * wall / args.steps
    value = step_pairs / (wall / args.steps) / 1e9

    # per-kernel totals; the dominant kernel is the one with the most time
    kern = {}
    for _, k, fl, m in ms:
        if k == "k_set_knots":      # no pair work of its own
            continue
        t = kern.setdefault(k, [0.0, 0.0, 0])
        t[0] += fl
        t[1] += m
        t[2] += 1
    dom = max(kern, key=lambda k: kern[k][1])
    flops, total_ms, nl = kern[dom]
    achieved = flops / (total_ms * 1e-3) / 1e12
    kernels = {k: {"launches_per_step": v[2] // args.steps,
                   "avg_launch_ms": round(v[1] / v[2], 4),
                   "tflops": round(v[0] / (v[1] * 1e-3) / 1e12, 2)} for k, v in kern.items()}
    sk = [m for _, k, _, m in ms if k == "k_set_knots"]
    kernels["k_set_knots"] = {"launches_per_step": len(sk) // args.steps,
                              "avg_launch_ms": round(sum(sk) / len(sk), 4)}

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 268435456 bytes read and written")

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

    # Biased node tables (Sec. 3), outside the step: the same split kernel on a
    # biased and on a uniform table, for the 15 arcmin workload and for the
    # paper's split example (240 arcmin).  Each gather timed over `reps` calls.
    biased = None
    if not args.no_biased:
        biased = {}
        reps = 3
        for name, s in (("split_15arcmin", W.C3B), ("split_example_240arcmin", W.SPLIT_EXAMPLE)):
            log("biased-table forwards: %s" % name)
            bl = A.gaussian_bl(s.fwhm, s.ell_max) * W.high_ell_mask(s.ell_max)
            tb, kb = A.paper_bias(s.theta_cut, s.ntab)
            plans = {
                "biased": A.Plan(s.nside, s.theta_cut,
                                 A.tabulate_legendre_at(bl, A.grid_nodes(s.theta_cut, s.ntab,
                                                                         tb, kb)),
                                 theta_break=tb, k_break=kb),
                "uniform": A.Plan(s.nside, s.theta_cut,
                                  A.tabulate_legendre(bl, s.theta_cut, s.ntab)),
            }
            x = dev_map(s.nside, s.seed)
            y = torch.empty_like(x)
            pc, pg = plans["biased"].pair_count_parts()
            rec = {"nside": s.nside, "fwhm_arcmin": round(s.fwhm / W.ARCMIN, 3),
                   "ell_range": [W.SPLIT_ELL + 1, s.ell_max],
                   "theta_cut_arcmin": round(s.theta_cut / W.ARCMIN, 3), "ntab": s.ntab,
                   "theta_break_arcmin": round(tb / W.ARCMIN, 4), "k_break": kb,
                   "pairs": pc + pg}
            for label, p in plans.items():
                for part in (CIRC, GEN):
                    p.convolve_part(x, y, part)
                torch.cuda.synchronize()
                t = {}
                for part, kname in ((CIRC, "k_circ"), (GEN, "k_general")):
                    e0, e1 = ev(), ev()
                    e0.record(stream)
                    for _ in range(reps):
                        p.convolve_part(x, y, part)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    t[kname] = e0.elapsed_time(e1) / reps
                tot = t["k_circ"] + t["k_general"]
                rec[label] = {"ms": round(tot, 4),
                              "k_circ_ms": round(t["k_circ"], 4),
                              "k_general_ms": round(t["k_general"], 4),
                              "circ_kernel": circ_kernel(p),
                              "gpair_per_s": round((pc + pg) / (tot * 1e-3) / 1e9, 2),
                              "k_general_tflops": round(FLOP_PER_PAIR["k_general"] * pg
                                                        / (t["k_general"] * 1e-3) / 1e12, 2)}
            rec["biased_over_uniform"] = round(rec["biased"]["ms"] / rec["uniform"]["ms"], 4)
            biased[name] = rec
            if s is W.SPLIT_EXAMPLE:
                split_real, split_x, split_pairs = plans["biased"], x, pc + pg
            del plans
            torch.cuda.synchronize()

        # The split convolution of the example (Sec. 2, eq. 1): the l-space half
        # Khat_l = b_l, l <= 1500, by GPU spherical-harmonic transforms, plus the
        # real-space half above (the beam's content above l = 1500, cut at 240').
        s = W.SPLIT_EXAMPLE
        L = W.SPLIT_ELL
        log("split convolution: l-space half at l_cut %d" % L)
        harm = A.Harm(s.nside, A.gaussian_bl(s.fwhm, L))
        y = torch.empty_like(split_x)
        harm.convolve(split_x, y)
        A.split_convolve(split_real, harm, split_x, y)
        torch.cuda.synchronize()
        res = {}
        for label, fn in (("l_space_half", lambda: harm.convolve(split_x, y)),
                          ("split_total", lambda: A.split_convolve(split_real, harm, split_x, y))):
            e0, e1 = ev(), ev()
            e0.record(stream)
            for _ in range(reps):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res[label] = e0.elapsed_time(e1) / reps
        npix, nnorth = 12 * s.nside ** 2, 2 * s.nside
        nalm = (L + 1) * (L + 2) // 2
        # algorithmic FP64 FLOP: belt rings of power-of-two length 4 Nside by
        # real FFTs (complex FFT of half the length, 5 M log2 M each way),
        # the other rings by Goertzel and Clenshaw (3 per pixel and m each
        # way); Legendre recurrence 4 plus 2 (analysis) or 4 (synthesis) per
        # (l, m, northern ring)
        nb = 4 * s.nside
        M = nb // 2
        fft = (nb & (nb - 1)) == 0 and 2 <= M <= 8192 and L < M
        belt_rings = 2 * s.nside + 1 if fft else 0
        dft_pix = npix - belt_rings * nb
        flop64 = (6.0 * dft_pix * (L + 1) + belt_rings * 2 * 5.0 * M * np.log2(M)
                  + (6.0 + 8.0) * nnorth * nalm)
        tf = flop64 / (res["l_space_half"] * 1e-3) / 1e12
        biased["split_example"] = {
            "nside": s.nside, "l_cut": L, "theta_cut_arcmin": round(s.theta_cut / W.ARCMIN, 3),
            "l_space_half_ms": round(res["l_space_half"], 4),
            "l_space_fp64_tflops": round(tf, 2),
            "l_space_fp64_frac": round(tf / FP64_VECTOR_PEAK_TFLOPS, 4),
            "real_space_pairs": split_pairs,
            "split_total_ms": round(res["split_total"], 4),
            "maps_per_s": round(1e3 / res["split_total"], 2)}
        del harm, split_real
        torch.cuda.synchronize()

    # All-sky maps at Nside 4096 and 8192 (beyond the paper's single-GPU limit),
    # outside the step; the input is seeded N(0,1) noise drawn on the device.
    large = None
    if not args.no_large:
        large = []
        for s in W.LARGE:
            log("large map: Nside %d" % s.nside)
            p = A.Plan(s.nside, s.theta_cut, table(s))
            gen = torch.Generator(device=dev)
            gen.manual_seed(s.seed)
            x = torch.randn(12 * s.nside ** 2, generator=gen, device=dev)
            y = torch.empty_like(x)
            pc, pg = p.pair_count_parts()
            p.convolve(x, y)
            torch.cuda.synchronize()
            t = {}
            for part, kname in ((CIRC, "k_circ"), (GEN, "k_general")):
                e0, e1 = ev(), ev()
                e0.record(stream)
                for _ in range(3):
                    p.convolve_part(x, y, part)
                e1.record(stream)
                torch.cuda.synchronize()
                t[kname] = e0.elapsed_time(e1) / 3
            tot = t["k_circ"] + t["k_general"]
            large.append({"nside": s.nside, "npix": 12 * s.nside ** 2,
                          "fwhm_arcmin": round(s.fwhm / W.ARCMIN, 3),
                          "theta_cut_arcmin": round(s.theta_cut / W.ARCMIN, 3), "ntab": s.ntab,
                          "pairs": pc + pg, "ms": round(tot, 4),
                          "k_circ_ms": round(t["k_circ"], 4), "k_general_ms": round(t["k_general"], 4),
                          "circ_kernel": circ_kernel(p),
                          "gpair_per_s": round((pc + pg) / (tot * 1e-3) / 1e9, 2),
                          "maps_per_s": round(1e3 / tot, 2)})
            if s.nside == 8192:
                # a ~500 deg^2 polar-cap patch (rings 1..2208, theta <= 12.6 deg):
                # a ring-range plan writes only those rings
                pcap = A.Plan(s.nside, s.theta_cut, table(s), rings=(1, 2208))
                cap_pairs = pcap.pair_count()
                pcap.convolve(x, y)
                torch.cuda.synchronize()
                # a sub-millisecond launch: 20 calls, so that the clock ramp
                # and launch jitter of a few calls do not set the figure
                e0, e1 = ev(), ev()
                e0.record(stream)
                for _ in range(20):
                    pcap.convolve(x, y)
                e1.record(stream)
                torch.cuda.synchronize()
                cms = e0.elapsed_time(e1) / 20
                # the patch's reorientation: an equatorial patch centred on
                # (90 deg, 40 deg) rotated onto those rings of a second map
                rot = A.rotation_to_pole(np.pi / 2, np.radians(40.0))
                xr = torch.zeros_like(x)
                A.rotate_map(s.nside, rot, x, out=xr, rings=(1, 2208))
                torch.cuda.synchronize()
                e0, e1 = ev(), ev()
                e0.record(stream)
                for _ in range(3):
                    A.rotate_map(s.nside, rot, x, out=xr, rings=(1, 2208), stream=stream)
                e1.record(stream)
                torch.cuda.synchronize()
                rms_ = e0.elapsed_time(e1) / 3
                large[-1]["polar_cap_patch"] = {
                    "rings": [1, 2208], "area_deg2": 499, "pairs": cap_pairs,
                    "ms": round(cms, 4), "gpair_per_s": round(cap_pairs / (cms * 1e-3) / 1e9, 2),
                    "rotate_onto_cap_ms": round(rms_, 4),
                    "rotated_pixels": int(2 * 2208 * 2209)}
                del pcap, xr
            del p, x, y
            torch.cuda.synchronize()

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
        rate = float(pairs.sum()) / dt
        cores = O.threads()
        # the same oracle on one thread, over every 16th pixel of the sample
        O.set_threads(1)
        sub = pix[::16]
        t = time.perf_counter()
        _, p1 = O.convolve(s.nside, s.theta_cut, k64, x64, pixels=sub, return_pairs=True)
        dt1 = time.perf_counter() - t
        O.set_threads(cores)
        model = ""
        try:
            with open("/proc/cpuinfo") as f:
                model = next((ln.split(":", 1)[1].strip() for ln in f
                              if ln.startswith("model name")), "")
        except OSError:
            pass
        cpu = {"value": round(rate / 1e9, 4), "unit": "GPair-evals/s",
               "cores": cores, "kind": "oracle",
               "sample": "Nside 2048, FWHM 5', theta_cut 20', %d random output pixels "
                         "(%d pairs, %.1f s); FP64 C/OpenMP" % (pix.size, int(pairs.sum()), dt),
               "cpu_model": model,
               "one_thread_value": round(float(p1.sum()) / dt1 / 1e9, 4),
               "full_map_seconds": round(fwd_pairs[2] / rate, 1)}

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
                        "(15', 256 knots) + Nside-1024 x 8 fwd+bwd (30', 256 knots; knots "
                        "bound before each pass) + 16-map batch (Nside 256-2048, FWHM 5-30', "
                        "3 FWHM cut) replayed from captured graphs; white-noise FP32 maps",
            "pairs_per_step": int(step_pairs),
            "maps_per_step": len(fwd_plans) + 1 + c5.nbatch + len(bplans),
        },
        "breakdown": {
            "fwd": {"theta_cut_arcmin": [10, 15, 20], "ms": [round(m, 4) for m in fwd_ms],
                    "pairs": fwd_pairs,
                    "gpair_per_s": [round(p / (m * 1e-3) / 1e9, 2) for p, m in zip(fwd_pairs, fwd_ms)],
                    "maps_per_s": [round(1e3 / m, 1) for m in fwd_ms]},
            "fwdbwd": {"ms": round(fb_ms, 4), "pairs": 2 * g_pairs,
                       "gpair_per_s": round(2 * g_pairs / (fb_ms * 1e-3) / 1e9, 2),
                       "maps_per_s": round(1e3 / fb_ms, 1)},
            "grad_nside1024x8": {"ms": round(c5_ms, 4), "pairs": 2 * c5_pairs,
                                 "gpair_per_s": round(2 * c5_pairs / (c5_ms * 1e-3) / 1e9, 2),
                                 "maps_per_s": round(c5.nbatch * 1e3 / c5_ms, 1)},
            "tiles": {"tuned_plans": sum(1 for p in fwd_plans + [gplan, c5plan] + bplans
                                         if p.info()["tile_source"] == 1),
                      "plans": len(fwd_plans) + 2 + len(bplans)},
            "batch": {"ms": round(b_ms, 4), "pairs": int(b_circ + b_gen),
                      "gpair_per_s": round((b_circ + b_gen) / (b_ms * 1e-3) / 1e9, 2),
                      "maps_per_s": round(16e3 / b_ms, 1),
                      "plain16_ms": None if plain16_ms is None else round(plain16_ms, 4),
                      "speedup_vs_plain16": None if plain16_ms is None else round(plain16_ms / b_ms, 3)},
            "kernels": kernels,
            "biased_table": biased,
            "large_nside": large,
        },
        "roofline": {
            "kernel": dom,
            "bound": "alu",
            "achieved": round(achieved, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": _traffic(dom),
            "flop_per_pair": FLOP_PER_PAIR.get(dom),
            "avg_launch_ms": round(total_ms / nl, 4),
        },
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
