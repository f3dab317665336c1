"""Tile autotuning of the general gather on the current GPU.

    python -m paper_1211_3556_amd.autotune [--out FILE] [--reps N] [--preset bench]
                                           [NSIDE:ARCMIN[:FIRST-LAST] ...]

For each (Nside, theta_cut) the library's tuner (arkcos_tune) times the
general gather over candidate tile shapes and keeps the fastest; the results
form a tuning cache (one line per device arch, Nside and window class) that
plans created with default tiles read.  The preset `bench` covers the maps of
the benchmark: Nside 2048 at 10, 15, 20, 90 and 240 arcmin, the batch's
Nside 256-2048 maps cut at 3 x {5, 7, 10, 30} arcmin, and Nside 4096 / 8192
at 7.5 / 3.75 arcmin, and the polar-cap patch of the Nside 8192 map (output
rings 1-2208, which keeps cache entries of its own).  Tuning uses a flat table
of NTAB nodes (timing does not depend on the kernel values).
"""
from __future__ import annotations

import argparse
import math
import os
import sys

import paper_1211_3556_amd as A

ARCMIN = math.pi / (180.0 * 60.0)

PRESETS = {
    "bench": [(2048, 10.0), (2048, 15.0), (2048, 20.0), (2048, 240.0), (4096, 7.5),
              (8192, 3.75), (8192, 3.75, (1, 2208))] + [(n, 3.0 * fw) for n in (256, 512, 1024, 2048)
                                                        for fw in (5.0, 7.0, 10.0, 30.0)],
}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--out", default=A._TUNE_CACHE, help="tuning cache to write (replaced)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--ntab", type=int, default=16384)
    ap.add_argument("--preset", choices=sorted(PRESETS))
    ap.add_argument("maps", nargs="*", help="NSIDE:ARCMIN or NSIDE:ARCMIN:FIRST-LAST (rings)")
    args = ap.parse_args(argv)
    todo = list(PRESETS[args.preset]) if args.preset else []
    for m in args.maps:
        f = m.split(":")
        rings = tuple(int(v) for v in f[2].split("-")) if len(f) > 2 else None
        todo.append((int(f[0]), float(f[1])) + ((rings,) if rings else ()))
    if not todo:
        ap.error("give maps or a preset")
    import torch
    if not torch.cuda.is_available():
        print("autotune needs a GPU", file=sys.stderr)
        return 1
    seen = set()
    tmp = args.out + ".tmp"
    with open(tmp, "w") as f:
        f.write("# General-gather tile shapes tuned on this device by arkcos_tune\n"
                "# (python -m paper_1211_3556_amd.autotune); one line per key:\n"
                "# arch nside window_class gen_pixels gen_quad_window gen_pair_window ms\n")
    for item in todo:
        nside, arcmin = item[0], item[1]
        rings = item[2] if len(item) > 2 else None
        tc = arcmin * ARCMIN
        key = (nside,) + A.tune_key(nside, tc, rings)
        if key in seen:
            continue
        seen.add(key)
        r = A.tune(nside, tc, args.ntab, reps=args.reps, cache=tmp, rings=rings)
        print("nside %5d  %7.2f arcmin  class %3d  %s  %.4f ms (defaults %.4f ms)"
              % (nside, arcmin, key[2], r["tiles"], r["ms"], r["default_ms"]), flush=True)
    os.replace(tmp, args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
