"""Host-side checks of libarkcos (no GPU needed): exported symbols, status
codes, and the plan's FP64 geometry, node table, longitude windows and exact
pair counts against the independent oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_1211_3556_amd as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "arkcos.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(arkcos_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = A.load_library()
    names = _declared_functions()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    # and nothing outside the header is exported with the prefix
    out = os.popen("nm -D --defined-only %s" % A.library_path()).read()
    exported = set(re.findall(r"\bT (arkcos_\w+)", out))
    assert exported == set(names)


def test_status_strings_and_version():
    lib = A.load_library()
    for code in (0, -1, -2, -3, -4, -5):
        assert lib.arkcos_status_string(code).startswith(b"ARKCOS")
    assert lib.arkcos_version() == 10000


@pytest.mark.parametrize("kw,msg", [
    (dict(nside=0), "nside"), (dict(nside=8193), "nside"),
    (dict(theta_cut=0.0), "theta_cut"), (dict(theta_cut=3.2), "theta_cut"),
    (dict(ntab=1, ktab=None), "ntab"), (dict(max_batch=0), "max_batch"),
    (dict(tiles=dict(gen_pixels=100)), "gen_pixels"),
    (dict(tiles=dict(gen_quad_window=-2)), "window"),
    (dict(tiles=dict(gen_pair_window=2000000)), "window"),
])
def test_plan_argument_errors(kw, msg):
    args = dict(nside=8, theta_cut=0.1, ktab=np.ones(16), max_batch=1, host_only=True)
    args.update(kw)
    if "ntab" in kw:
        args["ktab"] = np.ones(kw["ntab"])
        del args["ntab"]
    with pytest.raises(A.ArkcosError) as e:
        A.Plan(**args)
    assert e.value.status == -1 and msg in str(e.value)


def test_null_knots_need_learnable_and_bad_flags():
    lib = A.load_library()
    desc = A._PlanDesc(8, 0.1, 16, None, 1, A._tiles(None), 1)
    h = ctypes.c_void_p()
    assert lib.arkcos_plan_create(ctypes.byref(desc), ctypes.byref(h)) == -1
    assert b"learnable" in lib.arkcos_last_error()
    assert not h.value
    desc = A._PlanDesc(8, 0.1, 16, None, 1, A._tiles(None), 1 | 2 | 64)
    assert lib.arkcos_plan_create(ctypes.byref(desc), ctypes.byref(h)) == -1
    assert lib.arkcos_plan_create(None, ctypes.byref(h)) == -1
    assert lib.arkcos_plan_create(ctypes.byref(desc), None) == -1


def test_compute_calls_on_host_only_plan_are_rejected():
    lib = A.load_library()
    p = A.Plan(8, 0.2, np.ones(16), host_only=True, learnable=True)
    buf = ctypes.c_void_p(0x1000)
    out = ctypes.c_void_p(0x100000)
    assert lib.arkcos_convolve(p.handle, buf, out, 1, None) == -5
    assert lib.arkcos_convolve(p.handle, None, out, 1, None) == -1
    assert lib.arkcos_convolve_backward(p.handle, buf, None, None, None, 1, None) == -1
    assert lib.arkcos_plan_set_kernel(p.handle, buf, None) == -5
    assert lib.arkcos_plan_set_kernel_host(p.handle, np.ones(16).ctypes.data_as(A._dp)) == -5
    assert lib.arkcos_batch_create(None, 0, ctypes.byref(ctypes.c_void_p())) == -1
    arr = (ctypes.c_void_p * 1)(p.handle)
    assert lib.arkcos_batch_create(arr, 1, ctypes.byref(ctypes.c_void_p())) == -5
    # destroying NULL objects is a no-op
    assert lib.arkcos_plan_destroy(None) == 0
    assert lib.arkcos_batch_destroy(None) == 0


def test_forced_allocation_failure(monkeypatch):
    monkeypatch.setenv("ARKCOS_FAULT", "alloc")
    with pytest.raises(A.ArkcosError) as e:
        A.Plan(8, 0.2, np.ones(16))
    assert e.value.status == -2


def test_tabulate_argument_errors():
    lib = A.load_library()
    b = np.ones(4)
    out = np.empty(4)
    f = lib.arkcos_tabulate_legendre
    assert f(b.ctypes.data_as(A._dp), -1, 0.1, 4, out.ctypes.data_as(A._dp)) == -1
    assert f(b.ctypes.data_as(A._dp), 3, 0.0, 4, out.ctypes.data_as(A._dp)) == -1
    assert f(b.ctypes.data_as(A._dp), 3, 0.1, 1, out.ctypes.data_as(A._dp)) == -1
    assert f(None, 3, 0.1, 4, out.ctypes.data_as(A._dp)) == -1


@pytest.mark.parametrize("nside", [1, 2, 3, 7, 64, 2048])
def test_ring_geometry_matches_oracle(nside):
    g = O.ring_geometry(nside)
    rings = range(1, 4 * nside) if nside < 100 else list(range(1, 40)) + list(
        range(nside - 5, nside + 6)) + list(range(2 * nside - 3, 2 * nside + 4)) + list(
        range(4 * nside - 40, 4 * nside))
    for i in rings:
        r = A.ring_info(nside, i)
        assert r["n"] == g["n"][i - 1] and r["first"] == g["first"][i - 1]
        assert abs(r["z"] - g["z"][i - 1]) < 5e-16
        assert abs(r["sin_theta"] - g["s"][i - 1]) < 5e-16
        assert abs(r["phi0"] - g["phi0"][i - 1]) < 1e-15


@pytest.mark.parametrize("fwhm_arcmin,lmax,tc_arcmin,ntab", [
    (120.0, 191, 360.0, 4096), (30.0, 1535, 90.0, 8192), (5.0, 6143, 20.0, 2049),
])
def test_tabulation_matches_oracle(fwhm_arcmin, lmax, tc_arcmin, ntab):
    am = np.pi / 180 / 60
    bl = O.gaussian_bl(fwhm_arcmin * am, lmax)
    np.testing.assert_allclose(A.gaussian_bl(fwhm_arcmin * am, lmax), bl, rtol=1e-15)
    ko = O.tabulate(bl, tc_arcmin * am, ntab)
    ka = A.tabulate_legendre(bl, tc_arcmin * am, ntab)
    # two different FP64 summation algorithms (forward recurrence in the oracle,
    # Clenshaw in the plan); rounding grows like lmax * eps * max|K|
    assert np.max(np.abs(ka - ko)) < max(1e-13, 2e-14 * lmax) * np.abs(ko).max()


@pytest.mark.parametrize("nside,tc_deg", [
    (1, 30.0), (1, 179.0), (2, 50.0), (4, 1.0), (4, 89.7), (8, 20.0), (8, 179.3),
    (16, 6.0), (16, 44.9), (16, 71.7), (32, 17.3), (64, 6.0), (64, 2.5), (128, 1.5),
])
def test_exact_pair_count_matches_oracle(nside, tc_deg):
    """Cut-offs are chosen off lattice ties: at e.g. 45 or 90 degrees whole
    families of HEALPix pairs sit exactly on the cut, where the strict test
    theta < theta_cut is decided by the last bit of either computation."""
    tc = np.radians(tc_deg)
    p = A.Plan(nside, tc, np.ones(8), host_only=True)
    counts = O.pair_counts(nside, tc)
    assert p.pair_count() == int(counts.sum())
    circ, gen = p.pair_count_parts()
    assert circ + gen == p.pair_count()
    # general rings comprise both polar caps, so at least their pairs
    g = O.ring_geometry(nside)
    caps = np.zeros(counts.size, bool)
    for i in list(range(1, nside)) + list(range(3 * nside + 1, 4 * nside)):
        caps[g["first"][i - 1]:g["first"][i - 1] + g["n"][i - 1]] = True
    assert gen >= int(counts[caps].sum())


def _in_disc_pairs(nside, tc):
    v = O.pix2vec(nside)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    th = 2 * np.arcsin(np.minimum(1.0, d / 2))
    return np.nonzero(th < tc)


def _ring_index(nside):
    g = O.ring_geometry(nside)
    ring = np.repeat(np.arange(1, 4 * nside), g["n"])
    j = np.arange(12 * nside * nside) - np.repeat(g["first"], g["n"])
    return ring, j, g


@pytest.mark.parametrize("nside,tc_deg", [(4, 40.0), (8, 12.0), (8, 100.0), (16, 7.0),
                                          (16, 160.0), (24, 5.0)])
def test_windows_cover_every_in_disc_pair(nside, tc_deg):
    """Every pair the oracle finds inside the disc lies in a window the kernels
    scan, and every window stays within one wrap of its ring."""
    tc = np.radians(tc_deg)
    plan = A.Plan(nside, tc, np.ones(8), host_only=True)
    ring, jj, g = _ring_index(nside)
    P, Q = _in_disc_pairs(nside, tc)
    win = {}
    for r in range(1, 4 * nside):
        for s in range(1, 4 * nside):
            w0 = plan.window(r, s, 0)
            if w0 is None:
                continue
            n_s = g["n"][s - 1]
            for j in range(g["n"][r - 1]):
                lo, hi = plan.window(r, s, j)
                assert -n_s < lo and hi < 2 * n_s and hi - lo + 1 <= n_s
                win[(r, s, j)] = (lo, hi)
    for p, q in zip(P, Q):
        r, j, s, jq = ring[p], jj[p], ring[q], jj[q]
        lo, hi = win[(r, s, j)]
        n_s = g["n"][s - 1]
        assert any(lo <= jq + k * n_s <= hi for k in (-1, 0, 1)), (r, j, s, jq, lo, hi)


def test_plan_info_is_consistent():
    p = A.Plan(32, np.radians(5.0), np.ones(100), host_only=True, tiles=dict(gen_pixels=64))
    inf = p.info()
    assert inf["nside"] == 32 and inf["nrings"] == 127 and inf["npix"] == 12288
    assert inf["tile_shapes"] == dict(gen_pixels=64, gen_quad_window=64, gen_pair_window=200)
    assert inf["tile_source"] == 2
    assert inf["ntab"] == 100 and inf["device_bytes"] == 0
    assert abs(inf["omega"] - 4 * np.pi / 12288) < 1e-18
    assert inf["tiles"] == inf["circulant_tiles"] + inf["general_tiles"]
    assert inf["candidates"] >= p.pair_count()


@pytest.mark.parametrize("nside,tc_deg", [(1, 5.0), (8, 3.0), (64, 6.0), (100, 3.31), (512, 1.5),
                                          (2048, 20.0 / 60), (16, 75.0), (300, 100.0)])
def test_ring_classes_cover_every_ring(nside, tc_deg):
    """Every ring is gathered by exactly one kernel: circulant belt rings
    (whose whole disc stays in the belt) or general rings (caps, belt edges),
    mirror-symmetric.  General tiles cover the pixels j <= jbar = n/4 - 2o - j
    of the first quadrant of each northern general ring (the reflection
    phi -> pi/2 - phi supplies the rest), up to 128 pixels per tile."""
    p = A.Plan(nside, np.radians(tc_deg), np.ones(8), host_only=True)
    inf = p.info()
    assert inf["circulant_rings"] + inf["general_rings"] == 4 * nside - 1
    assert inf["general_rings"] >= min(2 * (nside - 1), 4 * nside - 1)
    assert inf["general_rings"] % 2 == 1 or inf["circulant_rings"] % 2 == 1
    g = O.ring_geometry(nside)
    if inf["general_rings"] == 4 * nside - 1:
        tiles = 0
        for n, phi0 in zip(g["n"][:2 * nside], g["phi0"][:2 * nside]):
            q = int(n) // 4
            lanes = ((q - 1) // 2 if phi0 > 0 else q // 2) + 1
            tiles += -(-lanes // 128)
        assert inf["general_tiles"] == tiles
    if inf["circulant_rings"]:
        assert inf["weights"] > 0 and inf["circulant_tiles"] > 0


# ---------------------------------------------------------- biased grid --

@pytest.mark.parametrize("tc,ntab,tb_frac,kb", [
    (np.radians(2.0), 16384, 1 / 16, 8191), (0.3, 257, 1 / 16, 128), (0.3, 4, 0.1, 1),
    (np.pi, 1000, 0.25, 700), (0.01, 3, 0.4, 1),
])
def test_grid_nodes_match_oracle(tc, ntab, tb_frac, kb):
    tb = tb_frac * tc
    a = A.grid_nodes(tc, ntab, tb, kb)
    o = O.two_piece_nodes(tc, ntab, tb, kb)
    assert a[0] == 0.0 and a[-1] == tc and a[kb] == tb
    np.testing.assert_allclose(a, o, rtol=4e-16, atol=0)
    u = A.grid_nodes(tc, ntab)
    np.testing.assert_allclose(u, tc * np.arange(ntab) / (ntab - 1), rtol=4e-16, atol=0)
    assert u[-1] == tc


def test_paper_bias_matches_oracle():
    for ntab in (2 + 1, 4, 4096, 16384, 16385):
        assert A.paper_bias(0.2, ntab) == O.paper_bias(0.2, ntab)


@pytest.mark.parametrize("tb,kb,msg", [
    (0.01, 0, "k_break"), (0.0, 3, "theta_break"), (0.2, 3, "theta_break"),
    (-0.01, 3, "theta_break"), (0.01, 15, "k_break"), (0.01, -1, "k_break"),
    (0.15, 1, "fine"),
])
def test_grid_argument_errors(tb, kb, msg):
    with pytest.raises(A.ArkcosError) as e:
        A.Plan(8, 0.2, np.ones(16), host_only=True, theta_break=tb, k_break=kb)
    assert e.value.status == -1 and msg in str(e.value)
    with pytest.raises(A.ArkcosError) as e:
        A.grid_nodes(0.2, 16, tb, kb)
    assert e.value.status == -1


def test_biased_plan_info_and_nodes():
    tc = np.radians(3.0)
    p = A.Plan(16, tc, np.ones(101), host_only=True, biased=True)
    inf = p.info()
    assert inf["k_break"] == 50 and inf["theta_break"] == tc / 16
    nodes = p.nodes()
    assert nodes[50] == tc / 16 and nodes[-1] == tc
    with pytest.raises(ValueError):
        A.Plan(16, tc, np.ones(101), host_only=True, biased=True, k_break=3)
    # the grid changes neither the geometry nor the pair count
    q = A.Plan(16, tc, np.ones(101), host_only=True)
    assert q.pair_count() == p.pair_count() and q.info()["tiles"] == inf["tiles"]


def test_tabulate_at_nodes_matches_oracle():
    am = np.pi / 180 / 60
    bl = O.gaussian_bl(5.0 * am, 6143)
    tc = 15.0 * am
    nodes = O.biased_nodes(tc, 2049)
    ko = O.tabulate(bl, tc, nodes.size, nodes=nodes)
    ka = A.tabulate_legendre_at(bl, A.grid_nodes(tc, 2049, *A.paper_bias(tc, 2049)))
    assert np.max(np.abs(ka - ko)) < 2e-14 * 6143 * np.abs(ko).max()
    lib = A.load_library()
    th = np.array([0.1, 3.5])
    out = np.empty(2)
    f = lib.arkcos_tabulate_legendre_at
    assert f(bl.ctypes.data_as(A._dp), 10, th.ctypes.data_as(A._dp), 2,
             out.ctypes.data_as(A._dp)) == -1                       # angle above pi
    assert f(bl.ctypes.data_as(A._dp), 10, th.ctypes.data_as(A._dp), 0,
             out.ctypes.data_as(A._dp)) == -1
    assert f(None, 10, th.ctypes.data_as(A._dp), 1, out.ctypes.data_as(A._dp)) == -1


@pytest.mark.parametrize("nside,lcut,kind,status", [
    (0, 10, "ok", -1), (8193, 10, "ok", -1), (8, -1, "ok", -1), (8, 4096, "ok", -4),
    (8, 10, "null", -1), (8, 10, "batch", -1),
])
def test_harm_argument_errors(nside, lcut, kind, status):
    lib = A.load_library()
    k = np.ones(max(lcut, 0) + 1)
    h = ctypes.c_void_p()
    rc = lib.arkcos_harm_create(nside, lcut, None if kind == "null" else k.ctypes.data_as(A._dp),
                                0 if kind == "batch" else 1, ctypes.byref(h))
    assert rc == status and not h.value
    assert lib.arkcos_harm_destroy(None) == 0
    assert lib.arkcos_harm_convolve(None, None, None, 1, 0, None) == -1


# ------------------------------------------------------ ring-range plans --

@pytest.mark.parametrize("nside,tc_deg,rings", [(16, 7.0, (1, 10)), (16, 7.0, (12, 40)),
                                                (16, 30.0, (31, 31)), (16, 7.0, (50, 63)),
                                                (8, 100.0, (2, 29))])
def test_ring_range_pair_count_and_info(nside, tc_deg, rings):
    """A ring-range plan counts the in-disc pairs of its output rings only:
    the oracle's per-pixel counts summed over those rings."""
    tc = np.radians(tc_deg)
    p = A.Plan(nside, tc, np.ones(8), host_only=True, rings=rings)
    pc = O.pair_counts(nside, tc)
    g = O.ring_geometry(nside)
    lo, hi = g["first"][rings[0] - 1], g["first"][rings[1] - 1] + g["n"][rings[1] - 1]
    assert p.pair_count() == int(pc[lo:hi].sum())
    inf = p.info()
    assert (inf["ring_first"], inf["ring_last"]) == rings
    assert inf["circulant_rings"] + inf["general_rings"] == rings[1] - rings[0] + 1
    full = A.Plan(nside, tc, np.ones(8), host_only=True)
    assert inf["tiles"] <= full.info()["tiles"]


@pytest.mark.parametrize("rings", [(0, 5), (5, 0), (6, 5), (1, 64), (-1, 3)])
def test_ring_range_errors(rings):
    with pytest.raises(A.ArkcosError) as e:
        A.Plan(16, 0.1, np.ones(8), host_only=True, rings=rings)
    assert e.value.status == -1 and "ring range" in str(e.value)


@pytest.mark.parametrize("nside,tc_deg,rings", [(32, 9.0, (5, 60)), (32, 9.0, (1, 10)),
                                                (64, 6.0, (120, 136)), (16, 40.3, (2, 9))])
def test_ring_range_adjoint_rings(nside, tc_deg, rings):
    """The adjoint of a ring range writes every ring within theta_cut of it."""
    tc = np.radians(tc_deg)
    inf = A.Plan(nside, tc, np.ones(8), host_only=True, rings=rings).info()
    th = np.arccos(O.ring_geometry(nside)["z"])
    near = [s + 1 for s in range(4 * nside - 1)
            if np.min(np.abs(th[s] - th[rings[0] - 1:rings[1]])) < tc]
    assert (inf["adjoint_ring_first"], inf["adjoint_ring_last"]) == (near[0], near[-1])
    assert A.Plan(nside, tc, np.ones(8), host_only=True).info()["adjoint_ring_first"] == 0


def test_plan_log_line():
    """ARKCOS_LOG=1 prints one line of plan statistics per plan to stderr."""
    import subprocess
    import sys
    code = ("import numpy as np, paper_1211_3556_amd as A; "
            "A.Plan(32, np.radians(5.0), np.ones(64), host_only=True)")
    env = dict(os.environ, ARKCOS_LOG="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    assert r.returncode == 0, r.stderr
    lines = [l for l in r.stderr.splitlines() if l.startswith("[arkcos] plan")]
    assert len(lines) == 1
    p = A.Plan(32, np.radians(5.0), np.ones(64), host_only=True)
    inf = p.info()
    assert "nside 32" in lines[0] and "ring pairs %d" % inf["ring_pairs"] in lines[0]
    assert "rings %d circulant / %d general" % (inf["circulant_rings"], inf["general_rings"]) \
        in lines[0]


def test_rotation_to_pole_host():
    """The library's rotation takes (theta, phi) to the pole, equals
    R_y(-theta) R_z(-phi) built here, and rejects bad arguments; rotate_map
    rejects matrices that are not rotations before touching the device."""
    th, ph = 0.9, -2.4
    r = A.rotation_to_pole(th, ph)
    n = np.array([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)])
    np.testing.assert_allclose(r @ n, [0, 0, 1], atol=1e-15)
    rz = np.array([[np.cos(ph), np.sin(ph), 0], [-np.sin(ph), np.cos(ph), 0], [0, 0, 1.0]])
    ry = np.array([[np.cos(th), 0, -np.sin(th)], [0, 1.0, 0], [np.sin(th), 0, np.cos(th)]])
    np.testing.assert_allclose(r, ry @ rz, atol=1e-15)
    lib = A.load_library()
    dp = ctypes.POINTER(ctypes.c_double)
    EINVAL = -1
    assert lib.arkcos_rotation_to_pole(float("nan"), 0.0, np.zeros(9).ctypes.data_as(dp)) == EINVAL
    fake = ctypes.c_void_p(0x1000)
    far = ctypes.c_void_p(0x1000 + 12 * 16 * 16 * 4 * 8)
    bad = np.eye(3) * 1.01
    refl = np.diag([1.0, 1.0, -1.0])
    for m in (bad, refl):
        assert lib.arkcos_rotate_map(16, np.ascontiguousarray(m).ctypes.data_as(dp), fake, far, 1,
                                     0, 0, None) == EINVAL
    eye = np.eye(3)
    assert lib.arkcos_rotate_map(16, eye.ctypes.data_as(dp), fake, far, 1, 0, 70,
                                 None) == EINVAL
    assert lib.arkcos_rotate_map(16, eye.ctypes.data_as(dp), fake, fake, 1, 0, 0,
                                 None) == EINVAL


def test_circulant_form_follows_row_width(monkeypatch):
    """Plans with short circulant rows take the vector form of the circulant
    gather, plans whose rows average 9 taps or more the matrix-core form;
    ARKCOS_CIRC_FORM at plan creation forces either.  The log line names it."""
    import workloads as W
    def plan(tc_arcmin):
        tc = tc_arcmin * W.ARCMIN
        return A.Plan(2048, tc, W.gaussian_profile_knots(tc / 3, tc, 512), host_only=True)
    assert plan(10.0).info()["circ_form"] == 0
    assert plan(90.0).info()["circ_form"] == 1
    monkeypatch.setenv("ARKCOS_CIRC_FORM", "mfma")
    assert plan(10.0).info()["circ_form"] == 1
    monkeypatch.setenv("ARKCOS_CIRC_FORM", "valu")
    assert plan(90.0).info()["circ_form"] == 0
