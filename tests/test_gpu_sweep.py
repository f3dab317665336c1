"""A seeded sweep of random small configurations against the FP64 oracle.

Each case draws a resolution (odd and even N_side, down to 2), a cut-off from
a fraction of a pixel to ~70 degrees (redrawn until no pixel pair sits on the
cut), a table size, a uniform or two-piece node grid, a smooth but
structured kernel, optionally an output ring range, and the circulant
gather's form (the plan's own choice, or either form forced).  The forward
map is compared with the oracle on every output pixel of the range; pixels
outside the range must be left untouched.  A second sweep checks the map and
knot gradients of learnable plans the same way.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import REL_RMS_TOL, log, rel_rms, to_dev, to_host

pytestmark = pytest.mark.gpu

NSIDES = (2, 3, 5, 8, 12, 13, 16, 21, 32, 40, 48, 64)
NTABS = (16, 100, 257, 1000, 4096)
FORMS = (None, "valu", "mfma")


def _tie_free(nside, tc, rel=1e-7):
    return O.pair_counts(nside, tc * (1 - rel)).sum() == O.pair_counts(nside, tc * (1 + rel)).sum()


def _draw_case(seed):
    rng = np.random.default_rng(seed)
    nside = int(rng.choice(NSIDES))
    pix = np.sqrt(4 * np.pi / (12 * nside * nside))
    while True:
        tc = float(np.exp(rng.uniform(np.log(0.6 * pix), np.log(np.radians(70.0)))))
        if _tie_free(nside, tc):
            break
    ntab = int(rng.choice(NTABS))
    tb, kb = 0.0, 0
    if rng.uniform() < 0.35:
        # two pieces, the first at least as fine as the second
        f = float(rng.uniform(0.05, 0.5))
        kmin = int(np.ceil(f * (ntab - 1))) + 1
        if kmin <= ntab - 2:
            tb, kb = f * tc, int(rng.integers(kmin, ntab - 1))
    nrings = 4 * nside - 1
    rings = None
    if rng.uniform() < 0.3:
        a, b = sorted(int(v) for v in rng.integers(1, nrings + 1, size=2))
        rings = (a, b)
    form = FORMS[int(rng.integers(0, len(FORMS)))]
    # a smooth kernel with some structure: a Gaussian core, a ripple and an offset
    sig = tc * float(rng.uniform(0.15, 0.6))
    ripple = float(rng.uniform(0.0, 0.4))
    return nside, tc, ntab, tb, kb, rings, form, sig, ripple


def _nodes(tc, ntab, tb, kb):
    if kb > 0:
        return O.two_piece_nodes(tc, ntab, tb, kb)
    return np.arange(ntab) * (tc / (ntab - 1))


def _kernel(nodes, tc, sig, ripple):
    return np.exp(-0.5 * (nodes / sig) ** 2) * (1.0 + ripple * np.cos(3.0 * np.pi * nodes / tc)) + 0.05


@pytest.mark.parametrize("seed", range(48))
def test_forward_sweep(monkeypatch, seed):
    import torch
    import paper_1211_3556_amd as A
    nside, tc, ntab, tb, kb, rings, form, sig, ripple = _draw_case(9100 + seed)
    if form is None:
        monkeypatch.delenv("ARKCOS_CIRC_FORM", raising=False)
    else:
        monkeypatch.setenv("ARKCOS_CIRC_FORM", form)
    nodes = _nodes(tc, ntab, tb, kb)
    k = _kernel(nodes, tc, sig, ripple)
    x = W.white_noise(nside, 9200 + seed)
    log("sweep %d: Nside %d cut %.4g rad ntab %d grid (%.3g, %d) rings %s form %s"
        % (seed, nside, tc, ntab, tb, kb, rings, form))
    plan = A.Plan(nside, tc, k, theta_break=tb, k_break=kb, rings=rings)
    xd = to_dev(x)
    out = torch.full_like(xd, float("nan"))
    plan.convolve(xd, out)
    torch.cuda.synchronize()
    out = to_host(out)
    if rings is None:
        lo, hi = 0, x.size
    else:
        lo, _ = W.ring_pixel_range(nside, rings[0])
        _, hi = W.ring_pixel_range(nside, rings[1])
    assert np.all(np.isnan(out[:lo])) and np.all(np.isnan(out[hi:]))
    ref = O.convolve(nside, tc, k, x, pixels=np.arange(lo, hi), nodes=nodes if kb > 0 else None)
    err = rel_rms(out[lo:hi], ref)
    log("sweep %d: rel rms %.3e" % (seed, err))
    assert err <= REL_RMS_TOL


@pytest.mark.parametrize("seed", range(16))
def test_backward_sweep(seed):
    """Map and knot gradients of learnable plans (uniform knots), full sky or a
    ring range, one or two maps."""
    import paper_1211_3556_amd as A
    nside, tc, _, _, _, rings, _, sig, ripple = _draw_case(9300 + seed)
    nside = min(nside, 21)
    while not _tie_free(nside, tc):
        tc *= 1.01
    rng = np.random.default_rng(9400 + seed)
    nk = int(rng.choice((16, 64, 200)))
    nb = int(rng.integers(1, 3))
    if rings is not None:
        nrings = 4 * nside - 1
        rings = (min(rings[0], nrings), min(rings[1], nrings))
    knots = _kernel(np.arange(nk) * (tc / (nk - 1)), tc, sig, ripple)
    x = W.white_noise(nside, 9500 + seed, nbatch=nb)
    g = W.white_noise(nside, 9600 + seed, nbatch=nb)
    gm = np.zeros_like(g)
    if rings is None:
        lo, hi = 0, g.shape[1]
    else:
        lo, _ = W.ring_pixel_range(nside, rings[0])
        _, hi = W.ring_pixel_range(nside, rings[1])
    gm[:, lo:hi] = g[:, lo:hi]
    log("backward sweep %d: Nside %d cut %.4g rad knots %d maps %d rings %s"
        % (seed, nside, tc, nk, nb, rings))
    plan = A.Plan(nside, tc, ntab=nk, max_batch=nb, learnable=True, rings=rings)
    plan.set_knots(to_dev(knots))
    gx, gk = plan.backward(to_dev(g), to_dev(x), want_map=True, want_knots=True)
    import torch
    torch.cuda.synchronize()
    gx, gk = to_host(gx), to_host(gk)
    for b in range(nb):
        err = rel_rms(gx[b], O.map_grad(nside, tc, knots, gm[b]))
        log("backward sweep %d map %d: rel rms %.3e" % (seed, b, err))
        assert err <= REL_RMS_TOL
    gk_ref = sum(O.knot_grad(nside, tc, nk, x[b], gm[b]) for b in range(nb))
    assert np.max(np.abs(gk - gk_ref)) <= 1e-5 * np.abs(gk_ref).max()
