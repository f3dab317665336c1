"""GPU parity of the polar-cap reorientation (arkcos_rotate_map): the output
pixels are exactly the oracle's (bitwise equal maps, since each output pixel
copies one input pixel chosen in FP64 on both sides), over all rings or a
ring range, for several maps; and the reorientation composed with a
ring-range plan, the partial-sky convolution of Sec. 4 (Conclusions)."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import REL_RMS_TOL, gpu_table, log, oracle_table, rel_rms, to_dev, to_host

pytestmark = pytest.mark.gpu


def _A():
    import paper_1211_3556_amd as A
    return A


def _rotation(a, b, c):
    """R_z(a) R_y(b) R_z(c), built here (neither side's own code)."""
    def rz(t):
        return np.array([[np.cos(t), -np.sin(t), 0.0], [np.sin(t), np.cos(t), 0.0], [0, 0, 1.0]])

    def ry(t):
        return np.array([[np.cos(t), 0.0, np.sin(t)], [0, 1.0, 0], [-np.sin(t), 0.0, np.cos(t)]])
    return rz(a) @ ry(b) @ rz(c)


@pytest.mark.parametrize("nside,angles", [(1, (0.2, 2.5, 1.0)), (2, (1.7, 0.9, -0.4)),
                                          (3, (-2.2, 1.3, 2.6)), (64, (0.3, 1.1, -2.0)),
                                          (100, (2.9, 0.4, 0.7)), (512, (-1.3, 2.2, 0.05))])
def test_rotation_matches_oracle_bitwise(nside, angles):
    import torch
    r = _rotation(*angles)
    x = W.white_noise(nside, 900 + nside)
    log("rotate Nside %d" % nside)
    y = _A().rotate_map(nside, r, to_dev(x))
    torch.cuda.synchronize()
    ref = O.rotate_map(nside, r, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(to_host(y), ref)


def test_ring_range_and_batch():
    import torch
    nside, r = 32, _rotation(0.7, 2.0, 1.9)
    xs = W.white_noise(nside, 950, nbatch=3)
    xd = to_dev(xs)
    out = torch.full_like(xd, float("nan"))
    log("rotate ring range, 3 maps")
    _A().rotate_map(nside, r, xd, out=out, rings=(5, 40))
    torch.cuda.synchronize()
    y = to_host(out)
    lo, _ = W.ring_pixel_range(nside, 5)
    _, hi = W.ring_pixel_range(nside, 40)
    for b in range(3):
        ref = O.rotate_map(nside, r, xs[b].astype(np.float32).astype(np.float64), rings=(5, 40))
        assert np.array_equal(y[b, lo:hi], ref[lo:hi])
        assert np.all(np.isnan(y[b, :lo])) and np.all(np.isnan(y[b, hi:]))


def test_rotation_to_pole_moves_a_patch_to_the_cap():
    """An equatorial disc of radius 10 deg lands within 10 deg of the north
    pole, i.e. on rings 1..k of the rotated map."""
    import torch
    A = _A()
    nside, th0, ph0, rad = 64, 1.4, 0.8, np.radians(10.0)
    r = A.rotation_to_pole(th0, ph0)
    v = O.pix2vec(nside)
    c = np.array([np.sin(th0) * np.cos(ph0), np.sin(th0) * np.sin(ph0), np.cos(th0)])
    x = (v @ c > np.cos(rad)).astype(np.float64)          # indicator of the disc
    log("rotate a patch to the pole")
    y = to_host(A.rotate_map(nside, r, to_dev(x)))
    torch.cuda.synchronize()
    near = v[:, 2] > np.cos(rad - 2.0 / nside)            # well inside the rotated disc
    far = v[:, 2] < np.cos(rad + 2.0 / nside)
    assert np.all(y[near] == 1.0) and np.all(y[far] == 0.0)


def test_partial_sky_convolution_of_a_rotated_patch():
    """Rotate a survey patch onto the north cap, convolve its rings with a
    ring-range plan: equal to the oracle's convolution of the oracle's rotated
    map on those rings (Sec. 4, Conclusions)."""
    import torch
    A = _A()
    nside, tc = 128, np.radians(2.0)
    knots = W.gaussian_profile_knots(tc / 3, tc, 1000)
    r = _rotation(0.4, 1.3, -0.6)                         # patch centre at R^T z
    rings = (1, 60)                                       # cap of ~27 deg
    x = W.white_noise(nside, 960)
    log("rotate then ring-range convolution Nside %d" % nside)
    xr = A.rotate_map(nside, r, to_dev(x))
    plan = A.Plan(nside, tc, knots, rings=rings)
    out = torch.zeros_like(xr)
    plan.convolve(xr, out)
    torch.cuda.synchronize()
    xr_o = O.rotate_map(nside, r, x.astype(np.float32).astype(np.float64))
    assert np.array_equal(to_host(xr), xr_o)
    lo, _ = W.ring_pixel_range(nside, rings[0])
    _, hi = W.ring_pixel_range(nside, rings[1])
    ref = O.convolve(nside, tc, knots, xr_o, pixels=np.arange(lo, hi))
    assert rel_rms(to_host(out)[lo:hi], ref) <= REL_RMS_TOL


def test_large_patch_rotation_sampled():
    """Nside 2048: a patch centre moved to the pole, rings 1..600, checked on
    sampled output pixels against the oracle's point location."""
    import torch
    A = _A()
    nside, rings = 2048, (1, 600)
    r = A.rotation_to_pole(2.0, -1.0)
    x = W.white_noise(nside, 970)
    log("rotate Nside 2048 rings 1..600")
    y = to_host(A.rotate_map(nside, r, to_dev(x), rings=rings))
    torch.cuda.synchronize()
    _, hi = W.ring_pixel_range(nside, rings[1])
    pix = np.random.default_rng(7).integers(0, hi, 20000)
    v = O.pix2vec(nside, pix)
    q = O.vec2pix(nside, v @ r)                            # rows of R^T n_p
    assert np.array_equal(y[pix], x[q].astype(np.float32).astype(np.float64))
