"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the convolution itself: only workload
descriptions (sizes, beams, cut-offs, seeds) and random inputs drawn from
``numpy.random.default_rng``.  The GPU library and the CPU oracle each compute
geometry, kernel tables and sums on their own.

Maps are iid N(0, 1) white noise in RING order.  White noise is the flat
C_l ~ 1 input spectrum the paper assumes for its kernels (Sec. 3, eq. 5 with
C_l ~ 1) and its "uniform-noise" test maps; no sky data is used.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

ARCMIN = np.pi / (180.0 * 60.0)
DEG = np.pi / 180.0


@dataclass(frozen=True)
class MapSpec:
    """One convolution: Nside, Gaussian beam FWHM, cut-off, table size, seed."""
    nside: int
    fwhm: float          # radians
    theta_cut: float     # radians
    ntab: int
    seed: int
    lmax: int = -1       # band limit of the beam; -1 means 3*Nside - 1

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def ell_max(self) -> int:
        return self.lmax if self.lmax >= 0 else 3 * self.nside - 1


# Nside 64, 2 degree beam, 6 degree cut, 4096 nodes: the small full-map case.
C1 = MapSpec(nside=64, fwhm=2.0 * DEG, theta_cut=6.0 * DEG, ntab=4096, seed=1, lmax=191)
# Nside 512, 30 arcmin beam, 1.5 degree cut, 8192 nodes.
C2 = MapSpec(nside=512, fwhm=30.0 * ARCMIN, theta_cut=1.5 * DEG, ntab=8192, seed=2, lmax=1535)
# Nside 2048, 5 arcmin beam, cut-off swept over 10/15/20 arcmin, 16384 nodes.
C3 = tuple(MapSpec(nside=2048, fwhm=5.0 * ARCMIN, theta_cut=tc * ARCMIN, ntab=16384, seed=3,
                   lmax=6143) for tc in (10.0, 15.0, 20.0))


def batch_specs() -> list[MapSpec]:
    """16 maps: Nside {256, 512, 1024, 2048} x FWHM {5, 7, 10, 30} arcmin, each
    Nside group taking every FWHM once; cut-off 3 FWHM, 16384 nodes; map k
    (ordered by Nside then FWHM) uses seed 400 + k."""
    out = []
    k = 0
    for nside in (256, 512, 1024, 2048):
        for fw in (5.0, 7.0, 10.0, 30.0):
            out.append(MapSpec(nside=nside, fwhm=fw * ARCMIN, theta_cut=3.0 * fw * ARCMIN,
                               ntab=16384, seed=400 + k))
            k += 1
    return out


@dataclass(frozen=True)
class GradSpec:
    """Learnable-knot workload: a batch of maps, knots on [0, theta_cut]."""
    nside: int = 1024
    nbatch: int = 8
    fwhm: float = 10.0 * ARCMIN
    target_fwhm: float = 9.0 * ARCMIN
    theta_cut: float = 30.0 * ARCMIN
    nknots: int = 256
    seed0: int = 500

    @property
    def npix(self) -> int:
        return 12 * self.nside * self.nside

    @property
    def ell_max(self) -> int:
        return 3 * self.nside - 1


C5 = GradSpec()


def white_noise(nside: int, seed: int, nbatch: int | None = None) -> np.ndarray:
    """iid N(0,1) FP64 map(s) of 12 Nside^2 pixels in RING order."""
    n = 12 * nside * nside
    if nbatch is None:
        return np.random.default_rng(seed).standard_normal(n)
    return np.stack([np.random.default_rng(seed + b).standard_normal(n) for b in range(nbatch)])


def ring_pixel_range(nside: int, ring: int) -> tuple[int, int]:
    """[first, last+1) RING indices of ring `ring` (1-based), for choosing
    evaluation pixels only."""
    n = nside
    if ring < n:
        first, cnt = 2 * ring * (ring - 1), 4 * ring
    elif ring <= 3 * n:
        first, cnt = 2 * n * (n - 1) + 4 * n * (ring - n), 4 * n
    else:
        k = 4 * n - ring
        first, cnt = 12 * n * n - 2 * k * (k + 1), 4 * k
    return first, first + cnt


def strata_rings(nside: int) -> list[int]:
    """Rings every evaluation subset includes: the poles, the cap/belt
    transitions and the equator, which a uniform sample almost never hits."""
    n = nside
    rings = set(range(1, 5)) | {n - 1, n, n + 1, 2 * n, 3 * n - 1, 3 * n, 3 * n + 1}
    rings |= set(range(4 * n - 4, 4 * n))
    return sorted(r for r in rings if 1 <= r <= 4 * n - 1)


def eval_pixels(nside: int, size: int, seed: int, max_strata_ring_pixels: int | None = None
                ) -> np.ndarray:
    """Sorted pixel subset: `size` uniform draws (seed + 10000) plus the strata
    rings.  Rings longer than max_strata_ring_pixels are subsampled evenly."""
    npix = 12 * nside * nside
    rng = np.random.default_rng(seed + 10_000)
    pick = set(rng.choice(npix, size=min(size, npix), replace=False).tolist())
    for r in strata_rings(nside):
        a, b = ring_pixel_range(nside, r)
        idx = np.arange(a, b)
        if max_strata_ring_pixels is not None and idx.size > max_strata_ring_pixels:
            idx = idx[:: int(np.ceil(idx.size / max_strata_ring_pixels))]
        pick.update(idx.tolist())
    return np.array(sorted(pick), dtype=np.int64)


def gaussian_profile_at(fwhm: float, theta) -> np.ndarray:
    """Synthetic node values: the small-angle Gaussian profile
    exp(-theta^2 / (2 sigma^2)) / (2 pi sigma^2) at the given angles."""
    sigma = fwhm / np.sqrt(8.0 * np.log(2.0))
    theta = np.asarray(theta, dtype=np.float64)
    return np.exp(-0.5 * (theta / sigma) ** 2) / (2.0 * np.pi * sigma * sigma)


def gaussian_profile_knots(fwhm: float, theta_cut: float, ntab: int) -> np.ndarray:
    """gaussian_profile_at sampled at k theta_cut/(ntab-1).  Used where both
    sides must start from byte-identical knots."""
    return gaussian_profile_at(fwhm, np.arange(ntab) * (theta_cut / (ntab - 1)))


# The ell at which the split example of Sec. 3 truncates its harmonic-space
# kernel.  The real-space part of such a split carries the beam's content
# above it and oscillates at small angles, which is what the biased table of
# Sec. 3 is for.
SPLIT_ELL = 1500

# Biased-table workload: Nside 2048, 5 arcmin beam restricted to
# SPLIT_ELL < l <= 6143, theta_cut 15 arcmin, 16384 nodes with half of them
# inside theta_cut / 16.
C3B = MapSpec(nside=2048, fwhm=5.0 * ARCMIN, theta_cut=15.0 * ARCMIN, ntab=16384, seed=3,
              lmax=6143)


# The split example of Sec. 3 at the paper's map size: a 7 arcmin beam with
# l <= 4096, the harmonic part truncated at l = 1500, the real-space part cut
# at 240 arcmin, on a 16384-node biased table.
SPLIT_EXAMPLE = MapSpec(nside=2048, fwhm=7.0 * ARCMIN, theta_cut=240.0 * ARCMIN, ntab=16384,
                        seed=7, lmax=4096)


# All-sky maps beyond the single-GPU limit of the paper's time (its
# conclusions, Sec. 4, put l ~ 8000-16000 on several GPUs): Nside 4096 and
# 8192, with the beam and cut scaled to the pixel size so that a disc holds as
# many pixels as in the 15 arcmin Nside-2048 workload (about 240 pairs per pixel).
LARGE = (MapSpec(nside=4096, fwhm=2.5 * ARCMIN, theta_cut=7.5 * ARCMIN, ntab=16384, seed=41),
         MapSpec(nside=8192, fwhm=1.25 * ARCMIN, theta_cut=3.75 * ARCMIN, ntab=16384, seed=42))


def high_ell_mask(lmax: int, ell_split: int = SPLIT_ELL) -> np.ndarray:
    """0/1 weights over l = 0..lmax keeping l > ell_split: applied to a beam's
    b_l it gives the real-space part of a sharp harmonic split."""
    return (np.arange(lmax + 1) > ell_split).astype(np.float64)
