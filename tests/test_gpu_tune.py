"""Tile autotuning on the GPU: the tuner returns shapes from its candidate
sets and records them in a cache that later plans read, and every general-
gather tile shape (ring groups of one, two or four, 16 to 128 pixels) gives the
FP64 oracle's result; a batch of plans with tuned shapes equals their plain
launches bit for bit."""
import os

import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import REL_RMS_TOL, assert_tie_free, log, rel_rms, to_dev, to_host

pytestmark = pytest.mark.gpu


def _A():
    import paper_1211_3556_amd as A
    return A


def _sync():
    import torch
    torch.cuda.synchronize()


def test_tuner_writes_a_cache_that_plans_read(tmp_path):
    A = _A()
    nside, tc = 64, np.radians(6.0)
    cache = tmp_path / "tiles.txt"
    log("tune Nside %d" % nside)
    r = A.tune(nside, tc, 4096, reps=2, cache=str(cache))
    t = r["tiles"]
    assert t["gen_pixels"] in (32, 64, 128)
    assert t["gen_quad_window"] in (-1, 32, 64, 96, 128)
    assert t["gen_pair_window"] in (-1, 100, 200, 400, 800)
    assert 0 < r["ms"] <= r["default_ms"] * 1.0000001
    arch, cls = A.tune_key(nside, tc)
    line = cache.read_text().split()
    assert line[:6] == [arch, str(nside), str(cls), str(t["gen_pixels"]),
                        str(t["gen_quad_window"]), str(t["gen_pair_window"])]
    try:
        A.set_tune_cache(str(cache))
        inf = A.Plan(nside, tc, np.ones(64)).info()
        assert inf["tile_source"] == 1 and inf["tile_shapes"] == t
    finally:
        A.set_tune_cache(A._TUNE_CACHE if os.path.exists(A._TUNE_CACHE) else None)
    # a fixed field stays fixed
    r = A.tune(nside, tc, 4096, reps=1, tiles=dict(gen_pixels=16))
    assert r["tiles"]["gen_pixels"] == 16


TILES = [dict(gen_pixels=16, gen_quad_window=-1, gen_pair_window=-1),
         dict(gen_pixels=32, gen_quad_window=1000, gen_pair_window=1000),
         dict(gen_pixels=64, gen_quad_window=-1, gen_pair_window=1000),
         dict(gen_pixels=128, gen_quad_window=32, gen_pair_window=100)]


@pytest.mark.parametrize("nside,tc_deg", [(96, 3.7), (32, 33.3)])
def test_every_tile_shape_matches_the_oracle(nside, tc_deg):
    A = _A()
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    knots = W.gaussian_profile_knots(tc / 3, tc, 3000)
    x = W.white_noise(nside, 950)
    ref = O.convolve(nside, tc, knots, x)
    xd = to_dev(x)
    outs = []
    for t in TILES:
        p = A.Plan(nside, tc, knots, tiles=t)
        assert p.info()["tile_shapes"] == t
        log("tiles %s Nside %d" % (t, nside))
        y = to_host(p.convolve(xd))
        _sync()
        assert rel_rms(y, ref) <= REL_RMS_TOL
        outs.append(y)
    # the circulant rings do not depend on the general tiles
    circ = A.Plan(nside, tc, knots, tiles=TILES[0])
    yc = to_host(circ.convolve_part(xd, xd.new_zeros(xd.shape), A.PART_CIRCULANT))
    _sync()
    mask = yc != 0
    for y in outs[1:]:
        assert np.array_equal(y[mask], outs[0][mask])


def test_batch_with_tuned_shapes_equals_plain():
    A = _A()
    specs = [W.MapSpec(nside=n, fwhm=fw * W.ARCMIN, theta_cut=3 * fw * W.ARCMIN, ntab=2048,
                       seed=960 + k) for k, (n, fw) in enumerate([(64, 60.0), (48, 90.0),
                                                                  (32, 120.0)])]
    plans = [A.Plan(s.nside, s.theta_cut, W.gaussian_profile_knots(s.fwhm, s.theta_cut, s.ntab),
                    tiles=TILES[k % len(TILES)]) for k, s in enumerate(specs)]
    xs = [to_dev(W.white_noise(s.nside, s.seed)) for s in specs]
    log("batch with per-plan tile shapes")
    ys = A.Batch(plans).convolve(xs)
    plain = [p.convolve(x) for p, x in zip(plans, xs)]
    _sync()
    for y, yp in zip(ys, plain):
        assert np.array_equal(to_host(y), to_host(yp))
