"""GPU parity of ring-range (partial-sky) plans: only the output rings of the
range are written, each as the oracle computes it; every other output pixel
is left as it was.  The last case is a ~500 square-degree polar-cap patch of
an Nside 8192 map, the survey geometry the paper's conclusions (Sec. 4) suggest for
small-area, high-resolution maps."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import REL_RMS_TOL, assert_tie_free, gpu_table, log, oracle_table, rel_rms, to_dev, to_host

pytestmark = pytest.mark.gpu


def _A():
    import paper_1211_3556_amd as A
    return A


def _sync():
    import torch
    torch.cuda.synchronize()


def _ring_pixels(nside, rings):
    lo, _ = W.ring_pixel_range(nside, rings[0])
    _, hi = W.ring_pixel_range(nside, rings[1])
    return lo, hi


@pytest.mark.parametrize("nside,tc_deg,rings", [
    (64, 6.0, (1, 12)),        # polar cap only
    (64, 6.0, (40, 110)),      # across the cap/belt boundary
    (64, 6.0, (120, 136)),     # belt, circulant rings, equator included
    (64, 6.0, (200, 255)),     # southern half only
    (64, 6.0, (128, 128)),     # the equator alone
    (64, 6.0, (30, 221)),      # a tile's two cap rings differ: one has its mirror in range
    (16, 74.7, (3, 50)),       # wide discs, full-range angles
])
def test_ring_range_matches_oracle_and_leaves_the_rest(nside, tc_deg, rings):
    import torch
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = W.gaussian_profile_knots(tc / 3, tc, 1500)
    x = W.white_noise(nside, 77 + rings[0])
    A = _A()
    log("ring range Nside %d rings %d..%d" % (nside, *rings))
    plan = A.Plan(nside, tc, k, rings=rings)
    xd = to_dev(x)
    out = torch.full_like(xd, float("nan"))
    plan.convolve(xd, out)
    full = A.Plan(nside, tc, k).convolve(xd)
    _sync()
    out, full = to_host(out), to_host(full)
    lo, hi = _ring_pixels(nside, rings)
    assert np.all(np.isnan(out[:lo])) and np.all(np.isnan(out[hi:]))
    assert not np.any(np.isnan(out[lo:hi]))
    pix = np.arange(lo, hi)
    ref = O.convolve(nside, tc, k, x, pixels=pix)
    assert rel_rms(out[lo:hi], ref) <= REL_RMS_TOL
    assert rel_rms(out[lo:hi], full[lo:hi]) <= 2e-7


def test_ring_range_batch():
    import torch
    A = _A()
    nside, tc = 32, np.radians(9.0)
    k = W.gaussian_profile_knots(np.radians(3.0), tc, 900)
    pr = A.Plan(nside, tc, k, rings=(5, 60))
    pf = A.Plan(nside, tc, k)
    xs = [to_dev(W.white_noise(nside, 5)), to_dev(W.white_noise(nside, 6))]
    outs = [torch.zeros_like(xs[0]), torch.zeros_like(xs[1])]
    log("ring-range plan in a batch")
    A.Batch([pr, pf]).convolve(xs, outs)
    plain = pr.convolve(xs[0], torch.zeros_like(xs[0]))
    _sync()
    assert np.array_equal(to_host(outs[0]), to_host(plain))


@pytest.mark.parametrize("nside,tc_deg,rings,nb", [
    (32, 9.0, (5, 60), 2),       # cap and belt
    (32, 9.0, (1, 10), 1),       # polar cap only
    (32, 9.0, (60, 68), 1),      # belt around the equator
    (32, 9.0, (100, 127), 2),    # southern cap
    (32, 9.0, (20, 108), 1),     # a tile's ring and its mirror both in range
    (16, 40.3, (2, 9), 1),       # wide discs
])
def test_ring_range_adjoint_and_knot_gradient(nside, tc_deg, rings, nb):
    """The adjoint of a ring-range plan is A^T applied to g restricted to the
    range: the oracle's map gradient of the masked g, zero beyond theta_cut of
    the range; the knot gradient sums over the range's output pixels only."""
    import torch
    A = _A()
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    nk = 96
    knots = W.gaussian_profile_knots(tc / 3, tc, nk)
    x = W.white_noise(nside, 610, nbatch=nb)
    g = W.white_noise(nside, 620, nbatch=nb)
    lo, hi = _ring_pixels(nside, rings)
    gm = np.zeros_like(g)
    gm[:, lo:hi] = g[:, lo:hi]
    plan = A.Plan(nside, tc, ntab=nk, max_batch=nb, learnable=True, rings=rings)
    inf = plan.info()
    plan.set_knots(to_dev(knots))
    log("ring-range adjoint Nside %d rings %d..%d" % (nside, *rings))
    gd = to_dev(g)     # values outside the range must be ignored
    gx = torch.full_like(gd, float("nan"))
    gx, gk = plan.backward(gd, to_dev(x), want_map=True, want_knots=True, gx=gx)
    gx2, gk2 = plan.backward(gd, to_dev(x), want_map=True, want_knots=True)
    _sync()
    gx, gk = to_host(gx), to_host(gk)
    assert np.array_equal(gx, to_host(gx2)) and np.array_equal(gk, to_host(gk2))
    a_lo, a_hi = _ring_pixels(nside, (inf["adjoint_ring_first"], inf["adjoint_ring_last"]))
    assert np.all(gx[:, :a_lo] == 0) and np.all(gx[:, a_hi:] == 0)
    for b in range(nb):
        ref = O.map_grad(nside, tc, knots, gm[b])
        assert np.all(ref[:a_lo] == 0) and np.all(ref[a_hi:] == 0)
        assert rel_rms(gx[b], ref) <= REL_RMS_TOL
    gk_ref = sum(O.knot_grad(nside, tc, nk, x[b], gm[b]) for b in range(nb))
    assert np.max(np.abs(gk - gk_ref)) <= 1e-5 * np.abs(gk_ref).max()
    assert rel_rms(gk, gk_ref) <= REL_RMS_TOL


def test_ring_range_autograd():
    """Through the autograd function: outputs outside the range are zero, and
    the gradients are those of the masked loss."""
    import torch
    A = _A()
    nside, tc, nk, rings = 16, np.radians(30.3), 64, (4, 20)
    assert_tie_free(nside, tc)
    knots = W.gaussian_profile_knots(tc / 3, tc, nk)
    x = W.white_noise(nside, 630)
    t = W.white_noise(nside, 640)
    plan = A.Plan(nside, tc, ntab=nk, learnable=True, rings=rings)
    xd = to_dev(x).requires_grad_(True)
    kd = to_dev(knots).requires_grad_(True)
    y = A.conv(xd, plan, kd)
    loss = ((y - to_dev(t)) ** 2).sum()
    loss.backward()
    _sync()
    lo, hi = _ring_pixels(nside, rings)
    yh = to_host(y)
    assert np.all(yh[:lo] == 0) and np.all(yh[hi:] == 0)
    yr = O.convolve(nside, tc, knots, x, pixels=np.arange(lo, hi))
    gm = np.zeros_like(x)
    gm[lo:hi] = 2 * (yr - t[lo:hi])     # outside the range y is a constant 0
    assert rel_rms(to_host(xd.grad), O.map_grad(nside, tc, knots, gm)) <= 1e-5
    gk_ref = O.knot_grad(nside, tc, nk, x, gm)
    assert np.max(np.abs(to_host(kd.grad) - gk_ref)) <= 1e-5 * np.abs(gk_ref).max()


def test_polar_cap_patch_nside8192_sampled():
    """Rings 1..2208 of an Nside 8192 map: a polar cap of ~500 square degrees
    (theta <= 12.6 deg), FWHM 1.25', theta_cut 3.75', on sampled pixels."""
    s = W.LARGE[1]
    rings = (1, 2208)
    log("polar cap patch Nside 8192 rings 1..2208")
    x = W.white_noise(s.nside, s.seed)
    A = _A()
    plan = A.Plan(s.nside, s.theta_cut, gpu_table(s), rings=rings)
    import torch
    xd = to_dev(x)
    out = torch.zeros_like(xd)
    plan.convolve(xd, out)
    _sync()
    lo, hi = _ring_pixels(s.nside, rings)
    y = to_host(out)
    pix = np.unique(np.concatenate([
        np.random.default_rng(s.seed).integers(lo, hi, 4000),
        np.arange(lo, lo + 400), np.arange(hi - 400, hi)]))
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), x, pixels=pix)
    err = rel_rms(y[pix], ref)
    log("polar cap patch rel rms %.3e over %d pixels" % (err, pix.size))
    assert err <= REL_RMS_TOL
    assert not np.any(y[hi:hi + 100000])
