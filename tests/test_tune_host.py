"""Host side of the tile autotuner: the tuning-cache key, cache lookup and its
precedence, and general-gather tilings that cover every general pixel exactly
once for any tile shapes."""
import os

import numpy as np
import pytest

import oracle as O
import paper_1211_3556_amd as A


def _restore_cache():
    A.set_tune_cache(A._TUNE_CACHE if os.path.exists(A._TUNE_CACHE) else None)


@pytest.mark.parametrize("nside,arcmin", [(2048, 10.0), (2048, 90.0), (256, 15.0), (8192, 3.75),
                                          (1, 600.0)])
def test_tune_key(nside, arcmin):
    tc = np.radians(arcmin / 60.0)
    arch, cls = A.tune_key(nside, tc)
    assert arch.startswith("gfx")
    pix = np.sqrt(4 * np.pi / (12.0 * nside * nside))
    assert cls == int(np.floor(2 * np.log2(tc / pix) + 0.5))
    with pytest.raises(A.ArkcosError):
        A.tune_key(0, tc)
    with pytest.raises(A.ArkcosError):
        A.tune_key(nside, 0.0)


def test_tune_cache_lookup_and_precedence(tmp_path):
    tc = np.radians(6.0)
    arch, cls = A.tune_key(64, tc)
    path = tmp_path / "tiles.txt"
    path.write_text(
        "# arch nside class gen_pixels quad pair ms\n"
        "%s 64 %d 32 -1 100 1.5\n"
        "%s 64 %d 64 32 400 1.2   # a later line for the same key wins\n"
        "%s 64 %d 16 16 16 0.1\n"
        "not a cache line\n"
        "%s 64 %d 100 32 400 0.1\n"          # invalid tile shapes are skipped
        "otherarch 64 %d 16 -1 -1 1.0\n" % (arch, cls, arch, cls, arch, cls + 1, arch, cls, cls))
    try:
        A.set_tune_cache(str(path))
        inf = A.Plan(64, tc, np.ones(8), host_only=True).info()
        assert inf["tile_source"] == 1
        assert inf["tile_shapes"] == dict(gen_pixels=64, gen_quad_window=32, gen_pair_window=400)
        # another window class has its own entry; an unknown key takes the defaults
        inf = A.Plan(64, tc * 1.45, np.ones(8), host_only=True).info()
        assert A.tune_key(64, tc * 1.45)[1] == cls + 1 and inf["tile_source"] == 1
        assert inf["tile_shapes"] == dict(gen_pixels=16, gen_quad_window=16, gen_pair_window=16)
        inf = A.Plan(32, tc, np.ones(8), host_only=True).info()
        assert inf["tile_source"] == 0
        assert inf["tile_shapes"] == dict(gen_pixels=128, gen_quad_window=64, gen_pair_window=200)
        # descriptor fields win over the cache; unset fields take the defaults
        inf = A.Plan(64, tc, np.ones(8), host_only=True, tiles=dict(gen_quad_window=-1)).info()
        assert inf["tile_source"] == 2
        assert inf["tile_shapes"] == dict(gen_pixels=128, gen_quad_window=-1, gen_pair_window=200)
        # no cache: defaults
        A.set_tune_cache(None)
        inf = A.Plan(64, tc, np.ones(8), host_only=True).info()
        assert inf["tile_source"] == 0
    finally:
        _restore_cache()


def test_ring_range_plans_keep_their_own_cache_entries(tmp_path):
    """A plan restricted to a ring range reads the entry of its window class
    plus TUNE_RANGE_CLASS; the whole sky, also when given as the full ring
    range, reads the plain class."""
    tc = np.radians(6.0)
    arch, cls = A.tune_key(64, tc)
    assert A.tune_key(64, tc, (1, 40)) == (arch, cls + A.TUNE_RANGE_CLASS)
    assert A.tune_key(64, tc, (1, 255)) == (arch, cls)
    path = tmp_path / "tiles.txt"
    path.write_text("%s 64 %d 64 32 400 1.0\n%s 64 %d 32 96 800 0.5\n"
                    % (arch, cls, arch, cls + A.TUNE_RANGE_CLASS))
    try:
        A.set_tune_cache(str(path))
        whole = dict(gen_pixels=64, gen_quad_window=32, gen_pair_window=400)
        part = dict(gen_pixels=32, gen_quad_window=96, gen_pair_window=800)
        for rings, want in ((None, whole), ((1, 255), whole), ((1, 40), part), ((30, 200), part)):
            inf = A.Plan(64, tc, np.ones(8), host_only=True, rings=rings).info()
            assert inf["tile_source"] == 1 and inf["tile_shapes"] == want, rings
    finally:
        _restore_cache()


def _general_north_rings(nside):
    g = O.ring_geometry(nside)
    out = {}
    for r in range(1, 2 * nside + 1):
        q = int(g["n"][r - 1]) // 4
        out[r] = ((q - 1) // 2 if g["phi0"][r - 1] > 0 else q // 2) + 1
    return out


@pytest.mark.parametrize("nside,tc_deg", [(16, 75.0), (64, 6.0), (100, 3.31), (512, 1.5),
                                          (2048, 90.0 / 60)])
@pytest.mark.parametrize("tiles", [dict(), dict(gen_pixels=16), dict(gen_pixels=32,
                                                                      gen_quad_window=-1),
                                   dict(gen_pixels=64, gen_quad_window=1000, gen_pair_window=-1),
                                   dict(gen_quad_window=-1, gen_pair_window=-1),
                                   dict(gen_quad_window=32, gen_pair_window=1000000)])
def test_gen_tiles_cover_every_general_pixel_once(nside, tc_deg, tiles):
    p = A.Plan(nside, np.radians(tc_deg), np.ones(8), host_only=True, tiles=tiles or None)
    inf = p.info()
    seg = inf["tile_shapes"]["gen_pixels"]
    t = p.gen_tiles()
    lanes = _general_north_rings(nside)
    rings = sorted(set(t[:, 2].tolist()))
    # every general northern ring is tiled, and the ring classes are mirror-symmetric
    nr_general = 2 * len(rings) - (1 if 2 * nside in rings else 0)
    assert nr_general == inf["general_rings"]
    cover = {r: np.zeros(lanes[r], dtype=int) for r in rings}
    for tile in np.unique(t[:, 0]):
        rows = t[t[:, 0] == tile]
        nr = rows[0, 1]
        assert nr in (1, 2, 4) and len(rows) <= nr and np.all(rows[:, 1] == nr)
        assert len(set(rows[:, 3].tolist())) == 1                  # one segment of each ring
        rs = rows[:, 2]     # adjacent rings (a ring may have no pixel in the last segment)
        assert np.all(np.diff(rs) >= 1) and rs[-1] - rs[0] < nr
        for _, _, r, j0, ln in rows:
            assert 1 <= ln <= seg and j0 % seg == 0
            cover[r][j0:j0 + ln] += 1
    for r in rings:
        assert np.all(cover[r] == 1), r
