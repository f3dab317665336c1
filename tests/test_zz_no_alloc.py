"""The allocation-free backward entry point (arkcos_convolve_backward_static)
against arkcos_convolve_backward: two calls in a row on one device, the second
with a smaller input, each equal to the plan-workspace call bit for bit and to
the FP64 oracle within the parity bar."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from gpu_util import REL_RMS_TOL, assert_tie_free, log, rel_rms, to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(nside, nb, tc_deg, nk, seed, oracle=True):
    import torch
    import paper_1211_3556_amd as A
    tc = np.radians(tc_deg)
    if oracle:
        assert_tie_free(nside, tc)
    knots = W.gaussian_profile_knots(tc / 3, tc, nk)
    x = W.white_noise(nside, seed, nbatch=nb)
    g = W.white_noise(nside, seed + 1, nbatch=nb)
    plan = A.Plan(nside, tc, ntab=nk, max_batch=nb, learnable=True)
    plan.set_knots(to_dev(knots))
    xd, gd = to_dev(x), to_dev(g)
    log("static-workspace backward: Nside %d, batch %d, %d knots" % (nside, nb, nk))
    gx_s, gk_s = plan.backward(gd, xd, want_map=True, want_knots=True, static_workspace=True)
    gx_p, gk_p = plan.backward(gd, xd, want_map=True, want_knots=True)
    # knot gradient alone through the static workspace
    _, gk_s2 = plan.backward(gd, xd, want_map=False, want_knots=True, static_workspace=True)
    torch.cuda.synchronize()
    gx_s, gk_s, gx_p, gk_p, gk_s2 = (to_host(t) for t in (gx_s, gk_s, gx_p, gk_p, gk_s2))
    assert np.array_equal(gx_s, gx_p)
    assert np.array_equal(gk_s, gk_p)
    assert np.array_equal(gk_s2, gk_p)
    if not oracle:
        plan.close()
        return
    gk_ref = sum(O.knot_grad(nside, tc, nk, x[b], g[b]) for b in range(nb))
    for b in range(nb):
        assert rel_rms(gx_s[b], O.map_grad(nside, tc, knots, g[b])) <= REL_RMS_TOL
    assert np.max(np.abs(gk_s - gk_ref)) <= 1e-5 * np.abs(gk_ref).max()
    assert rel_rms(gk_s, gk_ref) <= REL_RMS_TOL
    plan.close()


def test_static_workspace_backward_two_calls():
    # a larger call, then a smaller one on the same device (the array keeps the
    # first call's partial rows and counters)
    _case(32, 3, 10.3, 256, 810)
    _case(16, 1, 40.3, 64, 820)


def test_static_workspace_rejects_what_the_plan_rejects():
    import torch
    import paper_1211_3556_amd as A
    tc = np.radians(10.3)
    plan = A.Plan(16, tc, ktab=W.gaussian_profile_knots(tc / 3, tc, 64), max_batch=1)
    g = torch.zeros(plan.npix, dtype=torch.float32, device="cuda")
    x = torch.zeros_like(g)
    with pytest.raises(A.ArkcosError) as e:   # knot gradients need a learnable plan
        plan.backward(g, x, want_map=False, want_knots=True, static_workspace=True)
    assert e.value.status == -5
    with pytest.raises(A.ArkcosError) as e:   # nbatch above max_batch
        plan.backward(torch.zeros(2, plan.npix, dtype=torch.float32, device="cuda"),
                      want_map=True, static_workspace=True)
    assert e.value.status == -1


def test_static_workspace_holds_the_largest_knot_table():
    # ntab = ARKCOS_MAX_GRAD_NTAB on a map with more knot-gradient tiles than
    # resident workgroups, so both knot kernels use every partial row they can
    # (bitwise against the plan workspace; the oracle is too slow at this size)
    _case(1024, 1, 1.03, 2048, 830, oracle=False)
    _case(16, 1, 40.3, 2048, 840)
