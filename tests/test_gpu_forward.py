"""GPU parity of the forward real-space convolution against the FP64 oracle.

Every case calls the HIP library through its C ABI (via the ctypes binding)
and compares with the oracle on the same seeded inputs: full maps at small
Nside, sampled pixels (uniform draws plus every pixel of the polar, cap/belt
transition and equatorial rings) at the full workload sizes, in the launch
configuration the benchmark times.
"""
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


def _conv_gpu(plan, x):
    import torch
    y = plan.convolve(to_dev(x))
    torch.cuda.synchronize()
    return to_host(y)


def test_c1_full_map():
    s = W.C1
    log("c1 full map Nside %d" % s.nside)
    x = W.white_noise(s.nside, s.seed)
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    y = _conv_gpu(plan, x)
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), x)
    err = rel_rms(y, ref)
    log("c1 rel rms %.3e" % err)
    assert err <= REL_RMS_TOL


def test_c2_sampled():
    s = W.C2
    log("c2 Nside %d sampled" % s.nside)
    x = W.white_noise(s.nside, s.seed)
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    y = _conv_gpu(plan, x)
    pix = W.eval_pixels(s.nside, s.npix // 100, s.seed)
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), x, pixels=pix)
    err = rel_rms(y[pix], ref)
    log("c2 rel rms %.3e over %d pixels" % (err, pix.size))
    assert err <= REL_RMS_TOL


@pytest.mark.parametrize("k", [0, 1, 2])
def test_c3_nside2048_sampled(k):
    s = W.C3[k]
    log("c3 Nside 2048 theta_cut %.0f arcmin" % (s.theta_cut / W.ARCMIN))
    x = W.white_noise(s.nside, s.seed)
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    y = _conv_gpu(plan, x)
    pix = W.eval_pixels(s.nside, 65536, s.seed, max_strata_ring_pixels=512)
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), x, pixels=pix)
    err = rel_rms(y[pix], ref)
    log("c3 rel rms %.3e over %d pixels" % (err, pix.size))
    assert err <= REL_RMS_TOL


@pytest.mark.parametrize("nside,q", [(64, 0), (64, 8000), (64, 24000), (64, 49151), (13, 777)])
def test_impulse_maps(nside, q):
    """x = delta_q returns Omega K_lin(theta_pq): the table sampled at the true
    separations, element by element."""
    tc = np.radians(6.0 if nside == 64 else 25.0)
    ntab = 4096
    k = W.gaussian_profile_knots(np.radians(2.0 if nside == 64 else 8.0), tc, ntab)
    log("impulse Nside %d q %d" % (nside, q))
    x = np.zeros(12 * nside * nside)
    x[q] = 1.0
    y = _conv_gpu(_A().Plan(nside, tc, k), x)
    ref = O.convolve(nside, tc, k, x)
    nz = ref != 0
    assert np.array_equal(y != 0, nz) or np.sum((y != 0) != nz) <= 2
    err = np.abs(y - ref)
    assert np.all(err <= 2e-6 * np.abs(ref) + 1e-7 * np.abs(ref).max())
    assert rel_rms(y, ref) <= REL_RMS_TOL


def test_constant_map_response():
    s = W.C1
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    log("constant map")
    y = _conv_gpu(plan, np.ones(s.npix))
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), np.ones(s.npix))
    assert rel_rms(y, ref) <= REL_RMS_TOL
    # on a belt ring whose disc stays inside the belt every pixel sees the
    # same disc (rings N+10 and 3N-10 are 10 rings, > 7 degrees, from the caps)
    g = O.ring_geometry(s.nside)
    for i in (s.nside + 10, 2 * s.nside, 3 * s.nside - 10):
        a = g["first"][i - 1]
        ring = y[a:a + g["n"][i - 1]]
        assert np.ptp(ring) <= 1e-6 * np.abs(ring).max()


def _perm(nside, fn):
    g = O.ring_geometry(nside)
    perm = np.empty(12 * nside * nside, dtype=np.int64)
    for i in range(1, 4 * nside):
        n = int(g["n"][i - 1])
        half = not (nside <= i <= 3 * nside and (i - nside) % 2 == 1)
        j = np.arange(n)
        i2, j2 = fn(i, n, half, j)
        perm[g["first"][i - 1] + j] = g["first"][i2 - 1] + j2
    return perm


@pytest.mark.parametrize("which", ["rotation", "reflection", "mirror"])
def test_symmetries(which):
    nside, tc = 32, np.radians(9.0)
    k = W.gaussian_profile_knots(np.radians(3.0), tc, 2048)
    x = W.white_noise(nside, 77)
    fns = {"rotation": lambda i, n, h, j: (i, (j + n // 4) % n),
           "reflection": lambda i, n, h, j: (i, (n - 1 - j) if h else (n - j) % n),
           "mirror": lambda i, n, h, j: (4 * nside - i, j)}
    perm = _perm(nside, fns[which])
    plan = _A().Plan(nside, tc, k)
    log("symmetry %s" % which)
    y = _conv_gpu(plan, x)
    xp = np.empty_like(x)
    xp[perm] = x
    yp = _conv_gpu(plan, xp)
    assert rel_rms(yp[perm], y) <= REL_RMS_TOL


def test_bitwise_deterministic():
    s = W.C2
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    x = W.white_noise(s.nside, 5)
    log("determinism")
    a = _conv_gpu(plan, x)
    b = _conv_gpu(plan, x)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("nside,tc_deg", [(1, 101.3), (2, 61.7), (2, 179.3), (3, 41.9),
                                          (5, 118.3), (13, 29.3), (16, 74.7), (100, 3.31)])
def test_small_and_ragged_full_maps(nside, tc_deg):
    """Tiny rings, whole-ring (pole-crossing) windows, the full-range angle
    path (theta_cut > 0.5 rad), non-power-of-two Nside and ragged tiles, with a
    smooth kernel and a cut-off free of lattice ties."""
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = W.gaussian_profile_knots(tc / 2.5, tc, 1500)
    x = W.white_noise(nside, 1000 + nside)
    log("small Nside %d theta_cut %.1f" % (nside, tc_deg))
    y = _conv_gpu(_A().Plan(nside, tc, k), x)
    ref = O.convolve(nside, tc, k, x)
    assert rel_rms(y, ref) <= REL_RMS_TOL


@pytest.mark.parametrize("nside,tc_deg", [(64, 6.0), (16, 74.7)])
def test_int32_numerator_path(monkeypatch, nside, tc_deg):
    """The general gather carries the longitude numerator m as an exact FP32
    integer and switches to int32 on rings where |m| could reach 2^24 (wide
    windows at Nside >= 1024).  A test hook forces the int32 path everywhere
    at a size the oracle checks in full."""
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = W.gaussian_profile_knots(tc / 3, tc, 2048)
    x = W.white_noise(nside, 91)
    log("int32 numerator path Nside %d cut %.1f deg" % (nside, tc_deg))
    y_f = _conv_gpu(_A().Plan(nside, tc, k), x)
    monkeypatch.setenv("ARKCOS_FORCE_INT_NUMERATOR", "1")
    y_i = _conv_gpu(_A().Plan(nside, tc, k), x)
    ref = O.convolve(nside, tc, k, x)
    assert rel_rms(y_i, ref) <= REL_RMS_TOL
    # same weights up to the sine series, which the int32 path always takes long
    assert rel_rms(y_i, y_f) <= 5e-7


@pytest.mark.parametrize("nside,tc_deg", [(5, 118.3), (100, 3.31)])
def test_rough_table_error_bound(nside, tc_deg):
    """A table of iid random nodes is the worst case for FP32 angles: an error
    du ~ eps u in the table coordinate u = theta/h moves a weight by
    du |K_{i+1} - K_i|.  The error stays within that conditioning bound."""
    tc = np.radians(tc_deg)
    assert_tie_free(nside, tc)
    k = np.random.default_rng(nside).uniform(0.2, 1.0, 300)
    x = W.white_noise(nside, 1000 + nside)
    y = _conv_gpu(_A().Plan(nside, tc, k), x)
    ref = O.convolve(nside, tc, k, x)
    eps = np.finfo(np.float32).eps
    bound = 4 * eps * (k.size - 1) * np.sqrt(np.mean(np.diff(k) ** 2) / np.mean(k ** 2))
    log("rough table rel rms %.2e bound %.2e" % (rel_rms(y, ref), bound))
    assert rel_rms(y, ref) <= bound


def test_tiny_cut_gives_self_pairs_only():
    """theta_cut below the pixel spacing: y = Omega K_0 x."""
    nside = 16
    tc = np.radians(0.5)
    k = np.linspace(3.0, 1.0, 64)
    x = W.white_noise(nside, 3)
    y = _conv_gpu(_A().Plan(nside, tc, k), x)
    omega = 4 * np.pi / (12 * nside * nside)
    np.testing.assert_allclose(y, np.float32(omega * 3.0) * np.float32(x), rtol=1e-6)


def test_map_batches():
    """nbatch maps per call: every map agrees with the oracle, and a map of a
    batch equals the same map convolved alone bit for bit."""
    nside, tc = 40, np.radians(7.0)
    k = W.gaussian_profile_knots(np.radians(2.5), tc, 1000)
    xs = W.white_noise(nside, 11, nbatch=3)
    plan = _A().Plan(nside, tc, k, max_batch=11)
    log("batch of 3 maps")
    ys = _conv_gpu(plan, xs)
    for b in range(3):
        ref = O.convolve(nside, tc, k, xs[b])
        assert rel_rms(ys[b], ref) <= REL_RMS_TOL
    xb = W.white_noise(nside, 50, nbatch=11)
    yb = _conv_gpu(plan, xb)
    one = _conv_gpu(plan, xb[10])
    assert np.array_equal(yb[10], one)
    assert rel_rms(yb[7], O.convolve(nside, tc, k, xb[7])) <= REL_RMS_TOL


@pytest.mark.parametrize("nside,tc_deg", [(64, 6.0), (100, 3.31), (16, 74.7)])
def test_parts_compose_to_full_convolution(nside, tc_deg):
    """The circulant and general gathers write disjoint rings: running them
    one after the other, in either order, equals the full call bit for bit."""
    import torch
    A = _A()
    tc = np.radians(tc_deg)
    plan = A.Plan(nside, tc, W.gaussian_profile_knots(tc / 3, tc, 900))
    x = to_dev(W.white_noise(nside, 17))
    full = plan.convolve(x)
    a = torch.full_like(x, float("nan"))
    plan.convolve_part(x, a, A.PART_CIRCULANT)
    plan.convolve_part(x, a, A.PART_GENERAL)
    b = torch.full_like(x, float("nan"))
    plan.convolve_part(x, b, A.PART_GENERAL)
    plan.convolve_part(x, b, A.PART_CIRCULANT)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(a), to_host(full))
    assert np.array_equal(to_host(b), to_host(full))


def test_rejects_bad_calls():
    import torch
    A = _A()
    plan = A.Plan(8, 0.2, np.ones(16), max_batch=2)
    x = torch.zeros(3, 768, device="cuda")
    with pytest.raises(A.ArkcosError):
        plan.convolve(x)                    # nbatch > max_batch
    x = torch.zeros(768, device="cuda")
    with pytest.raises(A.ArkcosError):
        plan.convolve(x, out=x)             # aliasing
    with pytest.raises(A.ArkcosError):
        plan.backward(x, x, want_map=False, want_knots=True)   # not learnable
    with pytest.raises(TypeError):
        plan.convolve(torch.zeros(768, device="cuda", dtype=torch.float64))


@pytest.mark.parametrize("k", [0, 1])
def test_large_nside_sampled(k):
    """Nside 4096 and 8192 all-sky maps (805 M pixels at 8192) on one GPU,
    on sampled pixels of every ring class, in the launch configuration the
    benchmark times."""
    s = W.LARGE[k]
    log("large Nside %d theta_cut %.2f arcmin" % (s.nside, s.theta_cut / W.ARCMIN))
    x = W.white_noise(s.nside, s.seed)
    plan = _A().Plan(s.nside, s.theta_cut, gpu_table(s))
    y = _conv_gpu(plan, x)
    pix = W.eval_pixels(s.nside, 4096, s.seed, max_strata_ring_pixels=256)
    ref = O.convolve(s.nside, s.theta_cut, oracle_table(s), x, pixels=pix)
    err = rel_rms(y[pix], ref)
    log("large Nside %d rel rms %.3e over %d pixels" % (s.nside, err, pix.size))
    assert err <= REL_RMS_TOL


def test_wide_circulant_rows_split():
    """Belt rings whose rows are wider than one circulant staging pass (256
    taps) stay circulant, their rows split into consecutive passes: Nside 512
    with a 29.8 degree cut (rows up to ~340 taps; the equator's disc stays in
    the belt), against the oracle on sampled pixels."""
    import torch
    A = _A()
    nside, tc = 512, np.radians(29.8)
    knots = W.gaussian_profile_knots(tc / 3, tc, 4096)
    plan = A.Plan(nside, tc, knots)
    inf = plan.info()
    assert inf["circulant_rings"] > 0
    x = W.white_noise(nside, 970)
    log("wide circulant rows Nside %d" % nside)
    xd = to_dev(x)
    yc = torch.zeros_like(xd)
    plan.convolve_part(xd, yc, A.PART_CIRCULANT)
    y = to_host(plan.convolve(xd))
    torch.cuda.synchronize()
    circ = to_host(yc) != 0
    rng = np.random.default_rng(971)
    pix = np.unique(np.concatenate([rng.choice(np.flatnonzero(circ), 160, replace=False),
                                    rng.choice(12 * nside * nside, 40, replace=False)]))
    ref = O.convolve(nside, tc, knots, x, pixels=pix)
    assert rel_rms(y[pix], ref) <= REL_RMS_TOL


@pytest.mark.parametrize("nside,tc_deg,npix_sample", [(13, 40.0, 0), (64, 6.0, 0), (128, 20.0, 0),
                                                       (512, 29.8, 300)])
def test_circulant_vector_and_matrix_forms(monkeypatch, nside, tc_deg, npix_sample):
    """The circulant gather has a vector-FMA form and a matrix-core form (a
    Toeplitz product per row on v_mfma_f32_16x16x4f32), chosen per plan by its
    mean row width.  A test hook forces either form: both match the oracle,
    on ragged ring segments (Nside 13), short rows (Nside 64 at 6 deg), long
    rows (Nside 128 at 20 deg) and rows split over staging passes (Nside 512
    at 29.8 deg, sampled), and they agree with each other to FP32 rounding."""
    import torch
    A = _A()
    tc = np.radians(tc_deg)
    knots = W.gaussian_profile_knots(tc / 3, tc, 2048)
    x = W.white_noise(nside, 880 + nside)
    xd = to_dev(x)
    ys = {}
    for form, code in (("valu", 0), ("mfma", 1)):
        monkeypatch.setenv("ARKCOS_CIRC_FORM", form)
        plan = A.Plan(nside, tc, knots)
        assert plan.info()["circ_form"] == code
        assert plan.info()["circulant_rings"] > 0
        log("circulant %s form Nside %d cut %.1f deg" % (form, nside, tc_deg))
        yc = torch.zeros_like(xd)
        plan.convolve_part(xd, yc, A.PART_CIRCULANT)
        ys[form] = (to_host(yc), to_host(plan.convolve(xd)))
        torch.cuda.synchronize()
    circ = ys["valu"][0] != 0
    if npix_sample:
        rng = np.random.default_rng(881)
        pix = np.unique(rng.choice(np.flatnonzero(circ), npix_sample, replace=False))
    else:
        pix = np.flatnonzero(circ)
    ref = O.convolve(nside, tc, knots, x, pixels=pix)
    for form in ("valu", "mfma"):
        assert rel_rms(ys[form][1][pix], ref) <= REL_RMS_TOL, form
    # the two forms write the same rings and differ only in FP32 summation order
    assert np.array_equal(ys["valu"][0] != 0, ys["mfma"][0] != 0)
    assert rel_rms(ys["mfma"][0], ys["valu"][0]) <= 5e-7

