"""Pins for the FP64 oracle against facts fixed by the paper and by mathematics.

Each test would fail on a plausible slip in the oracle: a wrong pixel centre or
phi offset (golden HEALPix fixtures, symmetries, area identities), a dropped or
wrong pixel area Omega (constant map vs the Legendre transform lambda_0), a
wrong node spacing or interpolation (impulse maps against numpy.interp, the
Funk-Hecke checks), a missing neighbour (exhaustive all-pairs), a Legendre
recurrence slip (closed forms, scipy), a wrong gradient (central finite
differences, which are exact for a quadratic loss), or a misplaced node of the
biased table of Sec. 3 (the paper's printed break angle and node share).
"""
import os

import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load_golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


# ---------------------------------------------------------------- geometry --

def test_golden_nside1_pixel_centres():
    ref = _load_golden("healpix_nside1.txt")
    v = O.pix2vec(1, ref[:, 0].astype(np.int64))
    phi = np.degrees(np.arctan2(v[:, 1], v[:, 0])) % 360.0
    np.testing.assert_allclose(v[:, 2], ref[:, 1], atol=1e-15)
    np.testing.assert_allclose(phi, ref[:, 2], atol=1e-12)


def test_golden_nside2_rings():
    ref = _load_golden("healpix_nside2_rings.txt")
    g = O.ring_geometry(2)
    np.testing.assert_array_equal(g["n"], ref[:, 1].astype(int))
    np.testing.assert_array_equal(g["first"], ref[:, 2].astype(int))
    np.testing.assert_allclose(g["z"], ref[:, 3], atol=1e-15)
    np.testing.assert_allclose(np.degrees(g["phi0"]), ref[:, 4], atol=1e-12)


@pytest.mark.parametrize("nside", [1, 2, 3, 5, 8, 64, 2048])
def test_ring_counts_and_equal_area(nside):
    """Rings tile the map; the area north of each ring centre, 2 pi (1 - z_i),
    equals (pixels in earlier rings + half the ring) times Omega = 4 pi/Npix."""
    g = O.ring_geometry(nside)
    npix = 12 * nside * nside
    assert g["n"].sum() == npix
    np.testing.assert_array_equal(g["first"], np.concatenate([[0], np.cumsum(g["n"])[:-1]]))
    omega = 4.0 * np.pi / npix
    area_north = 2.0 * np.pi * (1.0 - g["z"])
    np.testing.assert_allclose(area_north / omega, g["first"] + 0.5 * g["n"], rtol=1e-12,
                               atol=1e-9)
    # mirror symmetry z_i = -z_{4N-i}, and sin(theta) without cancellation
    np.testing.assert_allclose(g["z"], -g["z"][::-1], atol=1e-15)
    np.testing.assert_allclose(g["s"] ** 2 + g["z"] ** 2, 1.0, atol=4e-16)
    np.testing.assert_allclose(g["theta"], np.arctan2(g["s"], g["z"]), atol=1e-15)


# -------------------------------------------------------------- tabulation --

def test_tabulation_closed_forms():
    th = np.linspace(0.0, np.pi, 33)
    # lmax = 0: K = b_0 / (4 pi)
    np.testing.assert_allclose(O.tabulate([0.7], np.pi, 33), 0.7 / (4 * np.pi), rtol=1e-15)
    # lmax = 1: K = (b_0 + 3 b_1 cos theta) / (4 pi)
    np.testing.assert_allclose(O.tabulate([1.0, 0.4], np.pi, 33),
                               (1.0 + 1.2 * np.cos(th)) / (4 * np.pi), atol=1e-15)
    # b_l = 1: sum_l (2l+1) P_l(x) = (L+1)(P_L(x) - P_{L+1}(x)) / (1 - x), (L+1)^2 at x = 1
    L = 40
    k = O.tabulate(np.ones(L + 1), np.pi, 33)
    x = np.cos(th)
    with np.errstate(divide="ignore", invalid="ignore"):
        cd = (L + 1) * (eval_legendre(L, x) - eval_legendre(L + 1, x)) / (1.0 - x)
    cd[0] = (L + 1) ** 2
    np.testing.assert_allclose(4 * np.pi * k, cd, atol=1e-11 * (L + 1) ** 2)


def test_tabulation_matches_scipy_legendre_sum():
    rng = np.random.default_rng(7)
    bl = rng.uniform(-1, 1, 61)
    tc, ntab = 0.8, 50
    th = np.arange(ntab) * tc / (ntab - 1)
    ref = sum((2 * l + 1) * bl[l] * eval_legendre(l, np.cos(th)) for l in range(61)) / (4 * np.pi)
    np.testing.assert_allclose(O.tabulate(bl, tc, ntab), ref, atol=1e-13 * np.abs(ref).max())


def test_tabulation_orthogonality():
    """With theta_cut = pi the Legendre transform of the table gives back b_l."""
    bl = O.gaussian_bl(np.radians(20.0), 24)
    k = O.tabulate(bl, np.pi, 8001)
    lam = O.legendre_coefficients(k, np.pi, range(25))
    np.testing.assert_allclose(lam, bl, atol=2e-6)


def test_gaussian_beam_half_maximum():
    """The tabulated eq. 5 kernel of a narrow Gaussian beam is, to O(sigma^2),
    the flat-sky profile exp(-theta^2/2 sigma^2)/(2 pi sigma^2): it peaks at
    1/(2 pi sigma^2) and falls to one half at theta = FWHM/2."""
    fw = np.radians(1.0)
    sigma = fw / np.sqrt(8 * np.log(2))
    bl = O.gaussian_bl(fw, 2000)
    k = O.tabulate(bl, fw, 3)                     # nodes at 0, FWHM/2, FWHM
    assert abs(k[0] * 2 * np.pi * sigma ** 2 - 1.0) < 1e-4
    assert abs(k[1] / k[0] - 0.5) < 1e-4
    assert abs(k[2] / k[0] - 1.0 / 16.0) < 1e-4


# ----------------------------------------------------- windows and the sum --

@pytest.mark.parametrize("nside", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("tc_deg", [1.0, 6.0, 30.0, 90.0, 179.0])
def test_windowed_equals_exhaustive(nside, tc_deg):
    rng = np.random.default_rng(nside * 1000 + int(tc_deg))
    x = rng.standard_normal(12 * nside * nside)
    k = rng.standard_normal(37)
    tc = np.radians(tc_deg)
    y1, p1 = O.convolve(nside, tc, k, x, return_pairs=True)
    y2, p2 = O.convolve(nside, tc, k, x, exhaustive=True, return_pairs=True)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_allclose(y1, y2, rtol=0, atol=1e-14 * max(1.0, np.abs(y2).max()))


@pytest.mark.parametrize("tc_deg", [3.0, 25.0])
def test_windowed_equals_exhaustive_nside32(tc_deg):
    nside = 32
    x = np.random.default_rng(3).standard_normal(12 * nside * nside)
    k = np.random.default_rng(4).standard_normal(100)
    pix = W.eval_pixels(nside, 300, 5)
    y1, p1 = O.convolve(nside, np.radians(tc_deg), k, x, pixels=pix, return_pairs=True)
    y2, p2 = O.convolve(nside, np.radians(tc_deg), k, x, pixels=pix, exhaustive=True,
                        return_pairs=True)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_allclose(y1, y2, rtol=0, atol=1e-14 * np.abs(y2).max())


@pytest.mark.parametrize("nside,q", [(8, 0), (8, 300), (16, 1500), (16, 767)])
def test_impulse_map_samples_interpolated_kernel(nside, q):
    """x = delta_q gives y_p = Omega K_lin(theta_pq): the node table linearly
    interpolated (numpy.interp) at the true separation, zero at/after the cut."""
    npix = 12 * nside * nside
    tc = np.radians(40.0)
    k = np.random.default_rng(q).uniform(0.5, 2.0, 29)
    x = np.zeros(npix)
    x[q] = 1.0
    y = O.convolve(nside, tc, k, x)
    v = O.pix2vec(nside)
    cross = np.linalg.norm(np.cross(v, v[q]), axis=1)
    theta = np.arctan2(cross, v @ v[q])
    grid = np.arange(k.size) * tc / (k.size - 1)
    ref = np.where(theta < tc, np.interp(theta, grid, k), 0.0) * 4 * np.pi / npix
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-15)


def _fh_kernel():
    fw, tc = np.radians(6.0), np.radians(15.0)
    k = O.tabulate(O.gaussian_bl(fw, 300), tc, 2048)
    return tc, k


def test_constant_map_gives_legendre_transform_l0():
    """Constant map: y = W_p with W_p -> lambda_0 = 2 pi int K sin theta as the
    pixel quadrature refines (second order in the pixel size)."""
    tc, k = _fh_kernel()
    lam0 = O.legendre_coefficients(k, tc, [0])[0]
    errs = []
    for nside in (16, 32, 64):
        y = O.convolve(nside, tc, k, np.ones(12 * nside * nside))
        errs.append(np.sqrt(np.mean((y / lam0 - 1.0) ** 2)))
    assert errs[2] < 3e-3
    assert errs[1] < errs[0] / 2.5 and errs[2] < errs[1] / 2.5


@pytest.mark.parametrize("ell,m", [(1, 0), (1, 1), (2, 0), (2, 2), (8, 0), (8, 8)])
def test_band_limited_ylm_funk_hecke(ell, m):
    """Funk-Hecke: a Y_lm comes back scaled by lambda_l, the Legendre transform
    (eq. 1's operator) of the truncated interpolated kernel; the pixel-sum
    error falls as Nside grows."""
    tc, k = _fh_kernel()
    lam = O.legendre_coefficients(k, tc, [ell])[0]
    errs = []
    for nside in (16, 32, 64):
        v = O.pix2vec(nside)
        f = O.real_ylm(ell, m, v)
        y = O.convolve(nside, tc, k, f)
        errs.append(np.sqrt(np.mean((y - lam * f) ** 2) / np.mean((lam * f) ** 2)))
    assert errs[2] < 2e-3
    assert errs[1] < errs[0] / 2.0 and errs[2] < errs[1] / 2.0


# --------------------------------------------------------------- symmetry --

def _ring_perm(nside, fn):
    """Pixel permutation built ring by ring from the HEALPix layout: fn(i, n,
    half_offset, j) -> (i', j')."""
    g = O.ring_geometry(nside)
    perm = np.empty(12 * nside * nside, dtype=np.int64)
    for i in range(1, 4 * nside):
        n = int(g["n"][i - 1])
        half = not (nside <= i <= 3 * nside and (i - nside) % 2 == 1)
        j = np.arange(n)
        i2, j2 = fn(i, n, half, j)
        perm[g["first"][i - 1] + j] = g["first"][i2 - 1] + j2
    return perm


@pytest.mark.parametrize("nside,tc_deg", [(4, 50.0), (8, 20.0), (16, 8.0)])
def test_exact_symmetries(nside, tc_deg):
    """Rotation by pi/2, reflection phi -> -phi and the N-S mirror map pixel
    centres onto pixel centres, so they commute with the operator."""
    rng = np.random.default_rng(11)
    x = rng.standard_normal(12 * nside * nside)
    k = rng.uniform(0.1, 1.0, 57)
    tc = np.radians(tc_deg)
    y = O.convolve(nside, tc, k, x)
    rot = _ring_perm(nside, lambda i, n, h, j: (i, (j + n // 4) % n))
    refl = _ring_perm(nside, lambda i, n, h, j: (i, (n - 1 - j) if h else (n - j) % n))
    mirr = _ring_perm(nside, lambda i, n, h, j: (4 * nside - i, j))
    for perm in (rot, refl, mirr):
        xp = np.empty_like(x)
        xp[perm] = x
        yp = O.convolve(nside, tc, k, xp)
        np.testing.assert_allclose(yp[perm], y, rtol=0, atol=1e-13 * np.abs(y).max())


def test_belt_one_pixel_shift():
    """Shifting every belt ring by one pixel is a rotation by pi/(2N); outputs
    on rings whose disc stays inside the belt commute with it."""
    nside, tc = 16, np.radians(6.0)
    g = O.ring_geometry(nside)
    x = np.random.default_rng(5).standard_normal(12 * nside * nside)
    k = np.random.default_rng(6).uniform(0.1, 1.0, 40)
    shift = _ring_perm(nside, lambda i, n, h, j: (i, (j + 1) % n if nside <= i <= 3 * nside else j))
    xs = np.empty_like(x)
    xs[shift] = x
    y, ys = O.convolve(nside, tc, k, x), O.convolve(nside, tc, k, xs)
    zb = 2.0 / 3.0
    th_edge = np.arccos(zb)
    checked = 0
    for i in range(nside, 3 * nside + 1):
        th = g["theta"][i - 1]
        if th - tc > th_edge + 1e-9 and th + tc < np.pi - th_edge - 1e-9:
            sl = slice(g["first"][i - 1], g["first"][i - 1] + g["n"][i - 1])
            np.testing.assert_allclose(ys[sl][shift[sl] - g["first"][i - 1]], y[sl], rtol=0,
                                       atol=1e-12 * np.abs(y).max())
            checked += 1
    assert checked > 20


def test_self_adjoint():
    nside, tc = 16, np.radians(12.0)
    rng = np.random.default_rng(9)
    x, y = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(-1, 1, 80)
    ax, ay = O.convolve(nside, tc, k, x), O.convolve(nside, tc, k, y)
    assert abs(ax @ y - x @ ay) < 1e-13 * np.abs(ax).max() * np.abs(y).sum()


def test_total_pairs_match_disc_area():
    """Sum of in-disc pairs ~ Npix^2 (1 - cos theta_cut)/2."""
    for nside, tc in ((32, np.radians(10.0)), (64, np.radians(6.0))):
        npix = 12 * nside * nside
        tot = O.pair_counts(nside, tc).sum()
        expect = npix * npix * (1 - np.cos(tc)) / 2
        assert abs(tot / expect - 1) < 0.03


# --------------------------------------------------------------- gradients --

def _loss(y, t):
    return float(np.sum((y - t) ** 2))


def test_map_gradient_central_differences():
    """L = sum (A x - t)^2 is quadratic in x, so central differences are exact
    up to rounding: dL/dx_q = (A g)_q with g = 2 (A x - t)."""
    nside, tc = 8, np.radians(25.0)
    rng = np.random.default_rng(21)
    x, t = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(0.2, 1.0, 64)
    y = O.convolve(nside, tc, k, x)
    grad = O.map_grad(nside, tc, k, 2.0 * (y - t))
    h = 1e-3
    for q in (0, 5, 100, 383, 767):
        e = np.zeros_like(x)
        e[q] = h
        fd = (_loss(O.convolve(nside, tc, k, x + e), t) - _loss(O.convolve(nside, tc, k, x - e), t)) / (2 * h)
        assert abs(fd - grad[q]) < 1e-8 * max(1.0, abs(grad[q]))


def test_knot_gradient_central_differences():
    nside, tc = 8, np.radians(25.0)
    rng = np.random.default_rng(22)
    x, t = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(0.2, 1.0, 32)
    y = O.convolve(nside, tc, k, x)
    gk = O.knot_grad(nside, tc, k.size, x, 2.0 * (y - t))
    h = 1e-3 * np.abs(k).max()
    for kk in range(0, 32, 3):
        e = np.zeros_like(k)
        e[kk] = h
        fd = (_loss(O.convolve(nside, tc, k + e, x), t) - _loss(O.convolve(nside, tc, k - e, x), t)) / (2 * h)
        assert abs(fd - gk[kk]) < 1e-8 * max(1.0, np.abs(gk).max())


def test_gradient_euler_identities():
    """y is linear in the knots and in x: <K, dL/dK> = <g, y> = <x, dL/dx>."""
    nside, tc = 16, np.radians(10.0)
    rng = np.random.default_rng(23)
    x, t = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(0.2, 1.0, 48)
    y = O.convolve(nside, tc, k, x)
    g = 2.0 * (y - t)
    gk = O.knot_grad(nside, tc, k.size, x, g)
    gx = O.map_grad(nside, tc, k, g)
    gy = g @ y
    assert abs(k @ gk - gy) < 1e-12 * np.abs(g).sum() * np.abs(y).max()
    assert abs(x @ gx - gy) < 1e-12 * np.abs(g).sum() * np.abs(y).max()


# ------------------------------------------------------ biased node table --
# Sec. 3 places half of the nodes inside the first 1/16 of the support.  The
# oracle takes such a table as an explicit node list (two_piece_nodes) and
# finds node intervals by bisection; these pins fix the placement from the
# paper's printed figures and the sums on it from numpy.interp, brute force,
# the uniform special case, Funk-Hecke and finite differences.

def test_biased_nodes_match_paper_figures():
    frac_support, frac_nodes, break_arcmin = _load_golden("biased_grid_sec3.txt")
    tc = break_arcmin / frac_support * W.ARCMIN            # 120 arcmin
    for ntab in (4, 5, 257, 4096, 16384):
        nodes = O.biased_nodes(tc, ntab)
        tb, kb = O.paper_bias(tc, ntab)
        assert nodes.size == ntab and nodes[0] == 0.0 and nodes[-1] == tc
        assert np.all(np.diff(nodes) > 0)
        assert nodes[kb] == tb
        assert abs(tb / W.ARCMIN - break_arcmin) < 1e-12
        inside = int(np.count_nonzero(nodes <= tb))
        assert inside == -(-ntab // 2)                    # half of the nodes, rounded up
        assert abs(inside / ntab - frac_nodes) <= 0.5 / ntab + 1e-15
        # uniform on each piece, finer on the first
        d = np.diff(nodes)
        np.testing.assert_allclose(d[:kb], tb / kb, rtol=1e-9)
        np.testing.assert_allclose(d[kb:], (tc - tb) / (ntab - 1 - kb), rtol=1e-9)
        assert d[0] < d[-1]


def test_two_piece_nodes_rejects_bad_breaks():
    for tb, kb in ((0.0, 3), (1.0, 3), (0.5, 0), (0.5, 9)):
        with pytest.raises(ValueError):
            O.two_piece_nodes(1.0, 10, tb, kb)


@pytest.mark.parametrize("nside,q", [(8, 0), (8, 300), (16, 1500), (16, 767)])
def test_biased_impulse_map_samples_interpolated_kernel(nside, q):
    """x = delta_q on a biased table: y_p = Omega numpy.interp(theta_pq, nodes, K)."""
    npix = 12 * nside * nside
    tc = np.radians(40.0)
    k = np.random.default_rng(q + 1).uniform(0.5, 2.0, 29)
    nodes = O.biased_nodes(tc, k.size)
    x = np.zeros(npix)
    x[q] = 1.0
    y = O.convolve(nside, tc, k, x, nodes=nodes)
    v = O.pix2vec(nside)
    cross = np.linalg.norm(np.cross(v, v[q]), axis=1)
    theta = np.arctan2(cross, v @ v[q])
    ref = np.where(theta < tc, np.interp(theta, nodes, k), 0.0) * 4 * np.pi / npix
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(O.kernel_eval(tc, k, theta, nodes=nodes) * 4 * np.pi / npix, ref,
                               rtol=1e-12, atol=1e-15)


def test_kernel_eval_is_piecewise_linear_interpolation():
    tc = 0.3
    rng = np.random.default_rng(31)
    k = rng.standard_normal(40)
    nodes = O.two_piece_nodes(tc, k.size, 0.07, 25)
    th = np.concatenate([rng.uniform(0, tc, 5000), nodes, [tc, 0.4, np.pi]])
    ref = np.where(th < tc, np.interp(th, nodes, k), 0.0)
    np.testing.assert_allclose(O.kernel_eval(tc, k, th, nodes=nodes), ref, rtol=1e-13,
                               atol=1e-14)
    uni = tc * np.arange(k.size) / (k.size - 1)
    np.testing.assert_allclose(O.kernel_eval(tc, k, th),
                               np.where(th < tc, np.interp(th, uni, k), 0.0),
                               rtol=0, atol=1e-13)


def test_uniform_node_list_reduces_to_uniform_table():
    nside, tc = 16, np.radians(12.0)
    rng = np.random.default_rng(32)
    x, g = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(0.2, 1.0, 41)
    uni = tc * (np.arange(k.size) / (k.size - 1))
    uni[-1] = tc
    y0, y1 = O.convolve(nside, tc, k, x), O.convolve(nside, tc, k, x, nodes=uni)
    np.testing.assert_allclose(y1, y0, rtol=0, atol=1e-13 * np.abs(y0).max())
    g0, g1 = O.knot_grad(nside, tc, k.size, x, g), O.knot_grad(nside, tc, k.size, x, g, nodes=uni)
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-13 * np.abs(g0).max())


@pytest.mark.parametrize("nside,tc_deg", [(4, 60.0), (8, 20.0), (16, 9.0)])
def test_biased_windowed_equals_exhaustive(nside, tc_deg):
    rng = np.random.default_rng(nside + 77)
    x = rng.standard_normal(12 * nside * nside)
    k = rng.standard_normal(64)
    tc = np.radians(tc_deg)
    nodes = O.biased_nodes(tc, k.size)
    y1, p1 = O.convolve(nside, tc, k, x, return_pairs=True, nodes=nodes)
    y2, p2 = O.convolve(nside, tc, k, x, exhaustive=True, return_pairs=True, nodes=nodes)
    np.testing.assert_array_equal(p1, p2)
    np.testing.assert_allclose(y1, y2, rtol=0, atol=1e-14 * max(1.0, np.abs(y2).max()))


def test_biased_tabulation_matches_scipy_legendre_sum():
    rng = np.random.default_rng(33)
    bl = rng.uniform(-1, 1, 61)
    tc, ntab = 0.8, 50
    nodes = O.biased_nodes(tc, ntab)
    ref = sum((2 * l + 1) * bl[l] * eval_legendre(l, np.cos(nodes)) for l in range(61)) / (4 * np.pi)
    np.testing.assert_allclose(O.tabulate(bl, tc, ntab, nodes=nodes), ref,
                               atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("ell,m", [(2, 1), (8, 0)])
def test_biased_band_limited_ylm_funk_hecke(ell, m):
    """Funk-Hecke on a biased table: Y_lm comes back scaled by the Legendre
    transform of that table's interpolated kernel."""
    fw, tc = np.radians(6.0), np.radians(15.0)
    nodes = O.biased_nodes(tc, 2048)
    k = O.tabulate(O.gaussian_bl(fw, 300), tc, 2048, nodes=nodes)
    lam = O.legendre_coefficients(k, tc, [ell], nodes=nodes)[0]
    errs = []
    for nside in (16, 32, 64):
        v = O.pix2vec(nside)
        f = O.real_ylm(ell, m, v)
        y = O.convolve(nside, tc, k, f, nodes=nodes)
        errs.append(np.sqrt(np.mean((y - lam * f) ** 2) / np.mean((lam * f) ** 2)))
    assert errs[2] < 2e-3
    assert errs[1] < errs[0] / 2.0 and errs[2] < errs[1] / 2.0


def test_biased_knot_gradient_central_differences_and_euler():
    nside, tc = 8, np.radians(25.0)
    rng = np.random.default_rng(34)
    x, t = rng.standard_normal((2, 12 * nside * nside))
    k = rng.uniform(0.2, 1.0, 32)
    nodes = O.biased_nodes(tc, k.size)
    y = O.convolve(nside, tc, k, x, nodes=nodes)
    g = 2.0 * (y - t)
    gk = O.knot_grad(nside, tc, k.size, x, g, nodes=nodes)
    h = 1e-3 * np.abs(k).max()
    for kk in range(0, 32, 3):
        e = np.zeros_like(k)
        e[kk] = h
        fd = (_loss(O.convolve(nside, tc, k + e, x, nodes=nodes), t)
              - _loss(O.convolve(nside, tc, k - e, x, nodes=nodes), t)) / (2 * h)
        assert abs(fd - gk[kk]) < 1e-8 * max(1.0, np.abs(gk).max())
    assert abs(k @ gk - g @ y) < 1e-12 * np.abs(g).sum() * np.abs(y).max()


def test_bias_trades_outer_for_inner_interpolation_error():
    """What the bias of Sec. 3 buys: with the same node count the fine piece
    is 8x finer than a uniform table, so the linear-interpolation error of a
    smooth profile (h^2 |K''| / 8) inside theta_cut/16 falls ~64-fold, while
    the coarse piece is 15/8 as wide, raising the error there ~(15/8)^2."""
    tc, ntab = np.radians(2.0), 1025
    sig = tc / 5.0
    f = lambda th: np.exp(-0.5 * (th / sig) ** 2)   # noqa: E731
    uni = tc * np.arange(ntab) / (ntab - 1)
    bia = O.biased_nodes(tc, ntab)
    th_in = np.linspace(0.0, tc / 16, 20001)[:-1]
    th_out = np.linspace(tc / 8, tc, 20001)[:-1]
    err = {}
    for name, nodes in (("uni", uni), ("bia", bia)):
        k = f(nodes)
        err[name] = [np.abs(O.kernel_eval(tc, k, th, nodes=nodes) - f(th)).max()
                     for th in (th_in, th_out)]
    assert err["bia"][0] < err["uni"][0] / 50.0
    assert err["bia"][1] < err["uni"][1] * (15 / 8) ** 2 * 1.05
    assert err["bia"][1] > err["uni"][1] * 3.0


# ------------------------------------------------ harmonic-space half (SHT) --
# The l-space half of the split applies Khat_l, l <= lcut, by analysis with the
# pixel quadrature and synthesis.  By the addition theorem
#     sum_m Y_lm(p) conj(Y_lm(q)) = (2l+1)/(4 pi) P_l(cos theta_pq),
# that operator is exactly the all-pairs sum with the untruncated Legendre
# kernel Omega sum_l (2l+1)/(4 pi) Khat_l P_l(cos theta_pq): a closed form
# the pins below evaluate with scipy, independently of the transforms.

@pytest.mark.parametrize("theta", [0.0, 0.3, 1.1, np.pi / 2, 2.9])
def test_legendre_lm_matches_scipy(theta):
    from scipy.special import sph_harm_y
    L = 40
    lam = O.legendre_lm(L, theta)
    for l in range(L + 1):
        for m in range(l + 1):
            ref = sph_harm_y(l, m, theta, 0.0).real
            assert abs(lam[l, m] - ref) < 1e-13 * max(1.0, abs(ref)), (l, m)


def _addition_theorem(nside, khat, x):
    v = O.pix2vec(nside)
    c = np.clip(v @ v.T, -1.0, 1.0)
    kern = sum((2 * l + 1) / (4 * np.pi) * khat[l] * eval_legendre(l, c)
               for l in range(khat.size))
    return (4 * np.pi / x.size) * kern @ x


@pytest.mark.parametrize("nside,lcut", [(1, 0), (1, 9), (2, 5), (2, 30), (4, 11), (4, 23),
                                        (8, 23), (8, 40)])
def test_harmonic_equals_addition_theorem_sum(nside, lcut):
    """lcut below, at and above 3 Nside - 1 (longitude frequencies above the
    ring lengths included): the transform pair equals the all-pairs sum."""
    rng = np.random.default_rng(100 * nside + lcut)
    x = rng.standard_normal(12 * nside * nside)
    khat = rng.uniform(-1.0, 1.0, lcut + 1)
    y = O.harmonic(nside, khat, x)
    ref = _addition_theorem(nside, khat, x)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_harmonic_monopole_closed_form():
    """lcut = 0: y = Khat_0 (Omega sum x) / (4 pi) on every pixel."""
    nside = 16
    x = np.random.default_rng(5).standard_normal(12 * nside * nside)
    y = O.harmonic(nside, [2.5], x)
    np.testing.assert_allclose(y, 2.5 * (4 * np.pi / x.size) * x.sum() / (4 * np.pi),
                               rtol=1e-12)


def test_harmonic_band_limited_quadrature_convergence():
    """A band-limited Y_lm input with l <= lcut comes back scaled by Khat_l up
    to the HEALPix quadrature error, which falls as Nside grows."""
    ell, m = 5, 3
    khat = np.linspace(1.0, 2.0, 12)
    errs = []
    for nside in (8, 16, 32):
        f = O.real_ylm(ell, m, O.pix2vec(nside))
        y = O.harmonic(nside, khat, f)
        errs.append(np.sqrt(np.mean((y - khat[ell] * f) ** 2) / np.mean((khat[ell] * f) ** 2)))
    assert errs[2] < 1e-2
    assert errs[1] < errs[0] / 2.0 and errs[2] < errs[1] / 2.0


# ------------------------------------------------------ point location and map rotation --
def _healpix_projection(vec):
    """The HEALPix projection (Gorski et al. 2005; Calabretta & Roukema 2007)
    of unit vectors: x = phi, y = 3 pi z / 8 in the equatorial zone, and with
    sigma = sqrt(3 (1 - |z|)), x = phi_c + sigma (phi - phi_c),
    y = sign(z) pi (2 - sigma) / 4 in the caps (phi_c the centre of the
    longitude quadrant).  Pixels at resolution N are the squares
    |dx| + |dy| <= pi/(4N)."""
    v = np.asarray(vec, dtype=np.float64)
    z = v[:, 2] / np.linalg.norm(v, axis=1)
    phi = np.mod(np.arctan2(v[:, 1], v[:, 0]), 2 * np.pi)
    x = phi.copy()
    y = 3 * np.pi * z / 8
    cap = np.abs(z) > 2.0 / 3.0
    sig = np.sqrt(3 * (1 - np.abs(z[cap])))
    phc = phi[cap] - np.mod(phi[cap], np.pi / 2) + np.pi / 4
    x[cap] = phc + sig * (phi[cap] - phc)
    y[cap] = np.sign(z[cap]) * np.pi * (2 - sig) / 4
    return x, y


@pytest.mark.parametrize("nside", [1, 2, 3, 8, 33, 64, 100])
def test_vec2pix_returns_every_pixel_centre(nside):
    pix = np.arange(O.npix(nside))
    assert np.array_equal(O.vec2pix(nside, O.pix2vec(nside)), pix)


@pytest.mark.parametrize("nside", [1, 2, 5, 16, 64])
def test_vec2pix_point_lies_in_its_pixel_square(nside):
    """Random directions: in the HEALPix projection the point lies in the
    square of the pixel it is assigned to (an independent description of the
    pixel boundaries, by the projection instead of the ring formulae)."""
    rng = np.random.default_rng(31 + nside)
    v = rng.standard_normal((20000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    p = O.vec2pix(nside, v)
    x, y = _healpix_projection(v)
    xc, yc = _healpix_projection(O.pix2vec(nside, p))
    dx = np.abs(np.mod(x - xc + np.pi, 2 * np.pi) - np.pi)
    d = dx + np.abs(y - yc)
    assert np.all(d <= np.pi / (4 * nside) * (1 + 1e-9) + 1e-12)


def test_rotation_to_pole_and_rotated_maps():
    """R(theta, phi) takes (theta, phi) to the pole; the identity rotation
    copies a map; a quarter turn about z is the exact in-ring shift by n/4;
    only the requested rings are written."""
    th, ph = 1.1, 2.3
    r = O.rotation_to_pole(th, ph)
    n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    np.testing.assert_allclose(r @ n, [0, 0, 1], atol=1e-15)
    np.testing.assert_allclose(r @ r.T, np.eye(3), atol=1e-15)
    assert abs(np.linalg.det(r) - 1) < 1e-14
    nside = 16
    x = np.random.default_rng(3).standard_normal(O.npix(nside))
    assert np.array_equal(O.rotate_map(nside, np.eye(3), x), x)
    # R = rotation by +pi/2 about z: out(n) = x(R^T n), so out at pixel j of a
    # ring reads pixel j - n/4 of the same ring
    rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    y = O.rotate_map(nside, rz, x)
    g = O.ring_geometry(nside)
    for i in range(4 * nside - 1):
        f, nr = g["first"][i], g["n"][i]
        j = np.arange(nr)
        assert np.array_equal(y[f + j], x[f + (j - nr // 4) % nr])
    z = O.rotate_map(nside, rz, x, rings=(3, 5), out=np.full_like(x, 7.0))
    lo, hi = g["first"][2], g["first"][4] + g["n"][4]
    assert np.array_equal(z[lo:hi], y[lo:hi]) and np.all(z[:lo] == 7.0) and np.all(z[hi:] == 7.0)
