"""GPU parity of the biased node table of Sec. 3 (half of the nodes inside the
first 1/16 of the support) against the FP64 oracle.

The oracle takes the table as an explicit node list and bisects it; the
library builds its own two-piece grid from (theta_break, k_break) and maps
angles to node coordinates in closed form.  Where both sides are given the
same knot values, a grid that differs between them shows up as a parity
failure.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import (REL_RMS_TOL, angle_tolerance, assert_tie_free, log, rel_rms, to_dev,
                      to_host)

pytestmark = pytest.mark.gpu


def _A():
    import paper_1211_3556_amd as A
    return A


def _sync():
    import torch
    torch.cuda.synchronize()


def _conv_gpu(plan, x):
    y = plan.convolve(to_dev(x))
    _sync()
    return to_host(y)


def _knots(fwhm, tc, ntab):
    """Gaussian-profile knots at the oracle's biased nodes (given to both sides)."""
    return W.gaussian_profile_at(fwhm, O.biased_nodes(tc, ntab))


def test_c1_biased_full_map():
    """The Nside-64 workload on a biased table, each side tabulating the beam
    at its own node list."""
    s = W.C1
    A = _A()
    log("biased c1 full map")
    x = W.white_noise(s.nside, s.seed)
    tb, kb = A.paper_bias(s.theta_cut, s.ntab)
    kg = A.tabulate_legendre_at(A.gaussian_bl(s.fwhm, s.ell_max),
                                A.grid_nodes(s.theta_cut, s.ntab, tb, kb))
    y = _conv_gpu(A.Plan(s.nside, s.theta_cut, kg, theta_break=tb, k_break=kb), x)
    nodes = O.biased_nodes(s.theta_cut, s.ntab)
    ko = O.tabulate(O.gaussian_bl(s.fwhm, s.ell_max), s.theta_cut, s.ntab, nodes=nodes)
    ref = O.convolve(s.nside, s.theta_cut, ko, x, nodes=nodes)
    err = rel_rms(y, ref)
    log("biased c1 rel rms %.3e" % err)
    assert err <= REL_RMS_TOL


@pytest.mark.parametrize("nside,tc_deg", [(1, 101.3), (2, 61.7), (3, 41.9), (5, 118.3),
                                          (13, 29.3), (16, 74.7), (64, 6.0), (100, 3.31)])
def test_biased_small_and_ragged_full_maps(nside, tc_deg):
    """Every angle series (theta_cut up to 2 rad), whole-ring windows, ragged
    tiles and both gathers on a biased table."""
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = _knots(tc / 2.5, tc, 1500)
    x = W.white_noise(nside, 1100 + nside)
    log("biased small Nside %d theta_cut %.1f" % (nside, tc_deg))
    y = _conv_gpu(_A().Plan(nside, tc, k, biased=True), x)
    ref = O.convolve(nside, tc, k, x, nodes=O.biased_nodes(tc, k.size))
    assert rel_rms(y, ref) <= REL_RMS_TOL


@pytest.mark.parametrize("nside,q", [(64, 0), (64, 24000), (13, 777)])
def test_biased_impulse_maps(nside, q):
    """x = delta_q with a rapidly oscillating table: y_p = Omega K(theta_pq),
    checked pixel by pixel against the oracle.  Each output is one weight, so
    its error is that of the FP32 node coordinate u (a few eps u, u <= ntab-1)
    times the table's step |K_{i+1} - K_i|, plus the rounding of Omega K."""
    tc = np.radians(6.0 if nside == 64 else 25.0)
    nodes = O.biased_nodes(tc, 2001)
    k = np.cos(40.0 * np.pi * nodes / tc) * np.exp(-nodes / (0.2 * tc)) + 0.1
    x = np.zeros(12 * nside * nside)
    x[q] = 1.0
    log("biased impulse Nside %d q %d" % (nside, q))
    y = _conv_gpu(_A().Plan(nside, tc, k, biased=True), x)
    ref = O.convolve(nside, tc, k, x, nodes=nodes)
    eps = np.finfo(np.float32).eps
    omega = 4 * np.pi / x.size
    bound = omega * (4 * eps * (k.size - 1) * np.abs(np.diff(k)).max() + 4 * eps * np.abs(k).max())
    log("biased impulse max err %.2e bound %.2e" % (np.max(np.abs(y - ref)), bound))
    assert np.max(np.abs(y - ref)) <= bound


def test_biased_grid_that_is_uniform_matches_uniform_plan():
    """theta_break = k_break theta_cut/(ntab-1) puts the two-piece grid on the
    uniform nodes: the biased code path then agrees with the uniform one to
    FP32 rounding of the node coordinate."""
    nside, tc, ntab, kb = 64, np.radians(6.0), 1201, 300
    k = W.gaussian_profile_knots(np.radians(2.0), tc, ntab)
    x = W.white_noise(nside, 5)
    A = _A()
    log("biased grid on uniform nodes")
    yu = _conv_gpu(A.Plan(nside, tc, k), x)
    yb = _conv_gpu(A.Plan(nside, tc, k, theta_break=kb * tc / (ntab - 1), k_break=kb), x)
    assert rel_rms(yb, yu) <= 1e-7


@pytest.mark.parametrize("nside,tc_deg", [(64, 6.0), (16, 74.7)])
def test_biased_int32_numerator_path(monkeypatch, nside, tc_deg):
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = _knots(tc / 3, tc, 2048)
    x = W.white_noise(nside, 92)
    monkeypatch.setenv("ARKCOS_FORCE_INT_NUMERATOR", "1")
    log("biased int32 numerator Nside %d" % nside)
    y = _conv_gpu(_A().Plan(nside, tc, k, biased=True), x)
    ref = O.convolve(nside, tc, k, x, nodes=O.biased_nodes(tc, k.size))
    assert rel_rms(y, ref) <= REL_RMS_TOL


def test_biased_parts_compose_and_determinism():
    import torch
    A = _A()
    nside, tc = 100, np.radians(3.31)
    plan = A.Plan(nside, tc, _knots(tc / 3, tc, 900), biased=True)
    x = to_dev(W.white_noise(nside, 18))
    log("biased parts compose")
    full = plan.convolve(x)
    a = torch.full_like(x, float("nan"))
    plan.convolve_part(x, a, A.PART_GENERAL)
    plan.convolve_part(x, a, A.PART_CIRCULANT)
    again = plan.convolve(x)
    _sync()
    assert np.array_equal(to_host(a), to_host(full))
    assert np.array_equal(to_host(again), to_host(full))


def test_c3b_nside2048_split_kernel_sampled():
    """Nside 2048, theta_cut 15 arcmin, 16384 biased nodes, kernel = the 5
    arcmin beam's content above l = 1500 (an oscillating split real-space
    part), on sampled pixels in the launch configuration the benchmark times."""
    s = W.C3B
    A = _A()
    mask = W.high_ell_mask(s.ell_max)
    tb, kb = A.paper_bias(s.theta_cut, s.ntab)
    kg = A.tabulate_legendre_at(A.gaussian_bl(s.fwhm, s.ell_max) * mask,
                                A.grid_nodes(s.theta_cut, s.ntab, tb, kb))
    x = W.white_noise(s.nside, s.seed)
    log("c3b Nside 2048 biased split kernel")
    y = _conv_gpu(A.Plan(s.nside, s.theta_cut, kg, theta_break=tb, k_break=kb), x)
    nodes = O.biased_nodes(s.theta_cut, s.ntab)
    ko = O.tabulate(O.gaussian_bl(s.fwhm, s.ell_max) * mask, s.theta_cut, s.ntab, nodes=nodes)
    pix = W.eval_pixels(s.nside, 4096, s.seed + 1, max_strata_ring_pixels=512)
    ref = O.convolve(s.nside, s.theta_cut, ko, x, pixels=pix, nodes=nodes)
    err = rel_rms(y[pix], ref)
    log("c3b rel rms %.3e over %d pixels" % (err, pix.size))
    assert err <= REL_RMS_TOL


def test_split_example_240_arcmin_sampled():
    """The split example of Sec. 3 at Nside 2048: 7 arcmin beam above l = 1500
    (l <= 4096), theta_cut 240 arcmin, 16384 biased nodes; about 61000 pairs
    per output pixel, on sampled pixels of every ring class.  This kernel
    oscillates across the whole disc (angle condition ~11, against ~1.4 for
    the Gaussian beams), so it is the hardest case for the FP32 angle and the
    FP32 node coordinate beyond the break; it is held to the same 1e-6 bar as
    the beams, and the FP32-angle bound is logged beside it."""
    s = W.SPLIT_EXAMPLE
    A = _A()
    mask = W.high_ell_mask(s.ell_max)
    tb, kb = A.paper_bias(s.theta_cut, s.ntab)
    kg = A.tabulate_legendre_at(A.gaussian_bl(s.fwhm, s.ell_max) * mask,
                                A.grid_nodes(s.theta_cut, s.ntab, tb, kb))
    x = W.white_noise(s.nside, s.seed)
    log("split example Nside 2048 theta_cut 240 arcmin")
    y = _conv_gpu(A.Plan(s.nside, s.theta_cut, kg, theta_break=tb, k_break=kb), x)
    nodes = O.biased_nodes(s.theta_cut, s.ntab)
    ko = O.tabulate(O.gaussian_bl(s.fwhm, s.ell_max) * mask, s.theta_cut, s.ntab, nodes=nodes)
    pix = W.eval_pixels(s.nside, 768, s.seed + 1, max_strata_ring_pixels=32)
    ref = O.convolve(s.nside, s.theta_cut, ko, x, pixels=pix, nodes=nodes)
    err = rel_rms(y[pix], ref)
    tol = angle_tolerance(s.theta_cut, ko, nodes)
    log("split example rel rms %.3e over %d pixels (angle bound %.2e)" % (err, pix.size, tol))
    assert err <= REL_RMS_TOL


def test_mixed_uniform_and_biased_batch():
    """One persistent launch over plans on both grids: each map equals its
    plain launch bit for bit and the oracle on its own node list."""
    A = _A()
    cases = [(16, 900.0, False), (32, 360.0, True), (24, 600.0, True), (48, 270.0, False),
             (8, 2670.0, True)]
    plans, xs, refs = [], [], []
    for i, (nside, tc_am, biased) in enumerate(cases):
        tc = tc_am * W.ARCMIN
        assert_tie_free(nside, tc)
        ntab = 1024 + 512 * i
        k = _knots(tc / 3, tc, ntab) if biased else W.gaussian_profile_knots(tc / 3, tc, ntab)
        x = W.white_noise(nside, 950 + i)
        plans.append(A.Plan(nside, tc, k, biased=biased))
        xs.append(to_dev(x))
        refs.append(O.convolve(nside, tc, k, x,
                               nodes=O.biased_nodes(tc, ntab) if biased else None))
    batch = A.Batch(plans)
    log("mixed uniform/biased batch")
    ys = batch.convolve(xs)
    plain = [p.convolve(x) for p, x in zip(plans, xs)]
    _sync()
    for y, yp, ref in zip(ys, plain, refs):
        assert np.array_equal(to_host(y), to_host(yp))
        assert rel_rms(to_host(y), ref) <= REL_RMS_TOL


@pytest.mark.parametrize("nside,nb,tc_deg,nk", [(32, 2, 10.3, 64), (16, 3, 99.3, 200)])
def test_biased_gradients_full_maps(nside, nb, tc_deg, nk):
    """Adjoint and knot gradient of a learnable plan on a biased table against
    the oracle's gradients on the same node list."""
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    nodes = O.biased_nodes(tc, nk)
    knots = W.gaussian_profile_at(tc / 3, nodes)
    x = W.white_noise(nside, 610, nbatch=nb)
    g = W.white_noise(nside, 710, nbatch=nb)
    A = _A()
    plan = A.Plan(nside, tc, ntab=nk, max_batch=nb, learnable=True, biased=True)
    plan.set_knots(to_dev(knots))
    log("biased gradients Nside %d batch %d" % (nside, nb))
    gx, gk = plan.backward(to_dev(g), to_dev(x), want_map=True, want_knots=True)
    _sync()
    gx, gk = to_host(gx), to_host(gk)
    gk_ref = sum(O.knot_grad(nside, tc, nk, x[b], g[b], nodes=nodes) for b in range(nb))
    for b in range(nb):
        assert rel_rms(gx[b], O.map_grad(nside, tc, knots, g[b], nodes=nodes)) <= REL_RMS_TOL
    assert np.max(np.abs(gk - gk_ref)) <= 1e-5 * np.abs(gk_ref).max()
    assert rel_rms(gk, gk_ref) <= 1e-6
