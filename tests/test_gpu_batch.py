"""Batched persistent launch: every map of a mixed batch equals its own plain
launch bit for bit, agrees with the oracle, and a captured graph replays it."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import (REL_RMS_TOL, assert_tie_free, gpu_table, log, oracle_table, rel_rms,
                      to_dev, to_host)

pytestmark = pytest.mark.gpu


def _A():
    import paper_1211_3556_amd as A
    return A


def _sync():
    import torch
    torch.cuda.synchronize()


def _small_specs():
    out = []
    # (8, 890 arcmin): a cut of exactly 45 degrees would sit on lattice ties
    for k, (nside, fw) in enumerate([(16, 300.0), (32, 120.0), (64, 60.0), (24, 200.0),
                                     (8, 890.0), (48, 90.0)]):
        out.append(W.MapSpec(nside=nside, fwhm=fw * W.ARCMIN, theta_cut=3 * fw * W.ARCMIN,
                             ntab=2048 + 1000 * k, seed=900 + k))
    return out


def test_mixed_batch_matches_plain_and_oracle():
    A = _A()
    specs = _small_specs()
    for s in specs:
        assert_tie_free(s.nside, s.theta_cut)
    plans = [A.Plan(s.nside, s.theta_cut, gpu_table(s)) for s in specs]
    xs = [to_dev(W.white_noise(s.nside, s.seed)) for s in specs]
    batch = A.Batch(plans)
    log("mixed small batch")
    ys = batch.convolve(xs)
    plain = [p.convolve(x) for p, x in zip(plans, xs)]
    _sync()
    for s, y, yp, x in zip(specs, ys, plain, xs):
        assert np.array_equal(to_host(y), to_host(yp))
        ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), to_host(x))
        assert rel_rms(to_host(y), ref) <= REL_RMS_TOL


def test_batch_parts_compose():
    """The two persistent launches of a batch write disjoint rings: run one
    after the other they equal the full batched call bit for bit."""
    import torch
    A = _A()
    specs = _small_specs()
    plans = [A.Plan(s.nside, s.theta_cut, gpu_table(s)) for s in specs]
    batch = A.Batch(plans)
    xs = [to_dev(W.white_noise(s.nside, s.seed)) for s in specs]
    full = [to_host(y) for y in batch.convolve(xs)]
    outs = [torch.full_like(x, float("nan")) for x in xs]
    batch.convolve(xs, outs, part=A.PART_GENERAL)
    batch.convolve(xs, outs, part=A.PART_CIRCULANT)
    _sync()
    for o, f in zip(outs, full):
        assert np.array_equal(to_host(o), f)


def test_graph_replay():
    """A CUDA/HIP graph of the batched launch replays correctly several times,
    with eager work and synchronisation between replays."""
    import torch
    A = _A()
    specs = _small_specs()[:4]
    plans = [A.Plan(s.nside, s.theta_cut, gpu_table(s)) for s in specs]
    batch = A.Batch(plans)
    xs = [to_dev(W.white_noise(s.nside, s.seed)) for s in specs]
    outs = [torch.empty_like(x) for x in xs]
    eager = [to_host(y) for y in batch.convolve(xs)]
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        batch.convolve(xs, outs)          # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(stream)
    graph = torch.cuda.CUDAGraph()
    log("capture batch graph")
    with torch.cuda.graph(graph):
        batch.convolve(xs, outs)
    for rep in range(4):
        for o in outs:
            o.fill_(float("nan"))
        graph.replay()
        _sync()
        for o, e in zip(outs, eager):
            assert np.array_equal(to_host(o), e), rep
        # eager work between replays
        tmp = plans[0].convolve(xs[0])
        _sync()
        assert np.array_equal(to_host(tmp), eager[0])


def test_c4_full_batch_matches_plain_and_oracle():
    """The 16-map batch (Nside 256..2048, FWHM 5..30 arcmin, cut 3 FWHM) in one
    launch: every map is bitwise equal to its plain launch and agrees with the
    FP64 oracle on 1024 uniform pixels plus the polar, cap/belt and equatorial
    strata."""
    import torch
    A = _A()
    specs = W.batch_specs()
    plans = [A.Plan(s.nside, s.theta_cut, gpu_table(s)) for s in specs]
    xs = [to_dev(W.white_noise(s.nside, s.seed)) for s in specs]
    batch = A.Batch(plans)
    log("c4 batch of 16")
    ys = batch.convolve(xs)
    _sync()
    for k, (s, p, x, y) in enumerate(zip(specs, plans, xs, ys)):
        log("c4 map %d Nside %d" % (k, s.nside))
        yp = p.convolve(x)
        _sync()
        yh = to_host(y)
        assert np.array_equal(yh, to_host(yp))
        pix = W.eval_pixels(s.nside, 1024, s.seed, max_strata_ring_pixels=64)
        ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), to_host(x), pixels=pix)
        err = rel_rms(yh[pix], ref)
        log("c4 map %d rel rms %.3e over %d pixels" % (k, err, pix.size))
        assert err <= REL_RMS_TOL
        del yp
    del ys
    torch.cuda.empty_cache()
