"""FP64 CPU oracle for the real-space half of the split spherical convolution.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this package.  It shares no code
with the HIP library in ``paper_1211_3556_amd``; neither imports the other.

The heavy loops live in ``arkcos_oracle.c`` (plain C, FP64, OpenMP), loaded
through ctypes.  This module adds:

* ``gaussian_bl`` -- the beam of the eq. 5 kernel family with C_l = 1,
  b_l = exp(-l(l+1) sigma^2 / 2), sigma = FWHM / sqrt(8 ln 2) (Sec. 3);
* ``legendre_coefficients`` -- the Legendre transform operator of eq. 1,
  lambda_l = 2 pi int_0^theta_cut K(theta) P_l(cos theta) sin theta dtheta,
  applied to the interpolated, truncated real-space kernel (Gauss-Legendre on
  every linear segment of the table);
* ``real_ylm`` -- real spherical harmonics for the Funk-Hecke checks;
* ``harmonic`` -- the harmonic-space half of the split: the truncated
  l-space kernel applied by spherical-harmonic analysis (pixel quadrature)
  and synthesis, written out as plain sums;
* ``two_piece_nodes`` / ``paper_bias`` -- the biased node placement of Sec. 3
  (half of the nodes inside the first 1/16 of the support) as an explicit
  node list, which every kernel-table function here accepts as ``nodes``.

Parity pins for every function here are in ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "arkcos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math) into liboracle.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-fno-fast-math", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        lib.orc_ring.argtypes = [ctypes.c_long, ctypes.c_long, _dp, _dp, _dp, _lp, _lp, _dp]
        lib.orc_pix2vec.argtypes = [ctypes.c_long, ctypes.c_long, _lp, _dp]
        lib.orc_vec2pix.argtypes = [ctypes.c_long, ctypes.c_long, _dp, _lp]
        lib.orc_rotate_map.argtypes = [ctypes.c_long, _dp, ctypes.c_long, ctypes.c_long, _dp,
                                       _dp]
        lib.orc_tabulate.argtypes = [_dp, ctypes.c_long, ctypes.c_double, ctypes.c_long, _dp,
                                     _dp]
        for name in ("orc_convolve", "orc_convolve_exhaustive"):
            getattr(lib, name).argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_long, _dp,
                                           _dp, _dp, ctypes.c_long, _lp, _dp, _lp]
        lib.orc_knot_grad.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_long,
                                      _dp, _dp, _dp, _dp]
        lib.orc_kernel_eval.argtypes = [ctypes.c_double, ctypes.c_long, _dp, _dp, ctypes.c_long,
                                        _dp, _dp]
        lib.orc_harmonic.argtypes = [ctypes.c_long, ctypes.c_long, _dp, _dp, _dp]
        lib.orc_legendre_lm.argtypes = [ctypes.c_long, ctypes.c_double, _dp]
        lib.orc_threads.restype = ctypes.c_int
        lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _nodes(nodes, ntab):
    """(pointer, keep-alive array) of an optional explicit node list."""
    if nodes is None:
        return None, None
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    if nodes.size != ntab:
        raise ValueError("%d node angles for a table of %d values" % (nodes.size, ntab))
    return _d(nodes), nodes


def _l(a):
    return a.ctypes.data_as(_lp)


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with status %d" % (what, rc))


def threads() -> int:
    """OpenMP threads the oracle runs with."""
    return int(_load().orc_threads())


def set_threads(n: int) -> None:
    """Run the oracle's parallel loops on n OpenMP threads."""
    _check(_load().orc_set_threads(int(n)), "set_threads")


def npix(nside: int) -> int:
    return 12 * nside * nside


def ring_geometry(nside: int) -> dict:
    """Per-ring HEALPix RING geometry, rings 1..4N-1 (Gorski et al. 2005)."""
    lib = _load()
    nr = 4 * nside - 1
    out = {k: np.empty(nr) for k in ("z", "s", "theta", "phi0")}
    out["n"] = np.empty(nr, dtype=np.int64)
    out["first"] = np.empty(nr, dtype=np.int64)
    z, s, th, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n, f = ctypes.c_long(), ctypes.c_long()
    for i in range(1, nr + 1):
        _check(lib.orc_ring(nside, i, ctypes.byref(z), ctypes.byref(s), ctypes.byref(th),
                            ctypes.byref(n), ctypes.byref(f), ctypes.byref(p0)), "ring")
        out["z"][i - 1], out["s"][i - 1], out["theta"][i - 1] = z.value, s.value, th.value
        out["phi0"][i - 1], out["n"][i - 1], out["first"][i - 1] = p0.value, n.value, f.value
    return out


def pix2vec(nside: int, pix=None) -> np.ndarray:
    """Unit vectors (npix, 3) of RING pixels (all pixels if pix is None)."""
    if pix is None:
        pix = np.arange(npix(nside), dtype=np.int64)
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    out = np.empty((pix.size, 3))
    _check(_load().orc_pix2vec(nside, pix.size, _l(pix), _d(out)), "pix2vec")
    return out


def vec2pix(nside: int, vec) -> np.ndarray:
    """RING pixels containing the directions of the rows of `vec` (n, 3),
    from the HEALPix pixel boundaries (Gorski et al. 2005)."""
    v = np.ascontiguousarray(np.atleast_2d(vec), dtype=np.float64)
    out = np.empty(v.shape[0], dtype=np.int64)
    _check(_load().orc_vec2pix(nside, v.shape[0], _d(v), _l(out)), "vec2pix")
    return out


def rotation_to_pole(theta: float, phi: float) -> np.ndarray:
    """The rotation R_y(-theta) R_z(-phi), which takes the direction
    (theta, phi) to the north pole."""
    ct, st, cp, sp = np.cos(theta), np.sin(theta), np.cos(phi), np.sin(phi)
    rz = np.array([[cp, sp, 0.0], [-sp, cp, 0.0], [0.0, 0.0, 1.0]])
    ry = np.array([[ct, 0.0, -st], [0.0, 1.0, 0.0], [st, 0.0, ct]])
    return ry @ rz


def rotate_map(nside: int, rot, x, rings=None, out=None) -> np.ndarray:
    """out[p] = x[pixel containing R^T n_p] for the pixels of `rings`
    (1-based, inclusive; all by default): the map rotated by R, resampled at
    the nearest pixel.  Other pixels of `out` (zeros if not given) are kept."""
    r = np.ascontiguousarray(rot, dtype=np.float64).reshape(3, 3)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x) if out is None else np.array(out, dtype=np.float64, copy=True)
    lo, hi = (1, 4 * nside - 1) if rings is None else rings
    _check(_load().orc_rotate_map(nside, _d(r), lo, hi, _d(x), _d(y)), "rotate_map")
    return y


def gaussian_bl(fwhm_rad: float, lmax: int) -> np.ndarray:
    """Gaussian beam b_l, l = 0..lmax (eq. 5 with C_l = 1)."""
    sigma = fwhm_rad / np.sqrt(8.0 * np.log(2.0))
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma * sigma)


def two_piece_nodes(theta_cut: float, ntab: int, theta_break: float, k_break: int
                    ) -> np.ndarray:
    """Node angles of a table that is uniform on each of two pieces: nodes
    0..k_break evenly spaced on [0, theta_break], nodes k_break..ntab-1 evenly
    spaced on [theta_break, theta_cut] (node k_break sits on the break)."""
    if not (0.0 < theta_break < theta_cut) or not (1 <= k_break <= ntab - 2):
        raise ValueError("need 0 < theta_break < theta_cut and 1 <= k_break <= ntab - 2")
    fine = theta_break * (np.arange(k_break + 1) / k_break)
    coarse = theta_break + (theta_cut - theta_break) * (
        np.arange(1, ntab - k_break) / (ntab - 1 - k_break))
    nodes = np.concatenate([fine, coarse])
    nodes[k_break] = theta_break
    nodes[-1] = theta_cut
    return nodes


def paper_bias(theta_cut: float, ntab: int) -> tuple[float, int]:
    """The bias of Sec. 3: half of the nodes (ceil(ntab/2) of them, nodes
    0..k_break) inside the first 1/16 of the support [0, theta_cut]."""
    return theta_cut / 16.0, (ntab - 1) // 2


def biased_nodes(theta_cut: float, ntab: int) -> np.ndarray:
    """Node angles of the Sec. 3 biased table."""
    tb, kb = paper_bias(theta_cut, ntab)
    return two_piece_nodes(theta_cut, ntab, tb, kb)


def tabulate(bl, theta_cut: float, ntab: int, nodes=None) -> np.ndarray:
    """Node table K(theta_k) = sum_l (2l+1)/(4 pi) b_l P_l(cos theta_k) at the
    uniform nodes, or at `nodes` when given."""
    bl = np.ascontiguousarray(bl, dtype=np.float64)
    out = np.empty(ntab)
    nptr, _keep = _nodes(nodes, ntab)
    _check(_load().orc_tabulate(_d(bl), bl.size - 1, float(theta_cut), ntab, nptr, _d(out)),
           "tabulate")
    return out


def kernel_eval(theta_cut: float, ktab, theta, nodes=None) -> np.ndarray:
    """The interpolated, truncated kernel K(theta) of a node table."""
    ktab = np.ascontiguousarray(ktab, dtype=np.float64)
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(theta.size)
    nptr, _keep = _nodes(nodes, ktab.size)
    _check(_load().orc_kernel_eval(float(theta_cut), ktab.size, nptr, _d(ktab), theta.size,
                                   _d(theta), _d(out)), "kernel_eval")
    return out


def convolve(nside: int, theta_cut: float, ktab, x, pixels=None, exhaustive=False,
             return_pairs=False, nodes=None):
    """y[p] = Omega sum_{theta_pq < theta_cut} K(theta_pq) x[q] at `pixels`
    (K on the uniform nodes, or on `nodes` when given)."""
    lib = _load()
    ktab = np.ascontiguousarray(ktab, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != npix(nside):
        raise ValueError("map has %d pixels, Nside %d needs %d" % (x.size, nside, npix(nside)))
    if pixels is None:
        pix_ptr, neval = None, npix(nside)
    else:
        pixels = np.ascontiguousarray(pixels, dtype=np.int64)
        pix_ptr, neval = _l(pixels), pixels.size
    y = np.empty(neval)
    pairs = np.empty(neval, dtype=np.int64)
    fn = lib.orc_convolve_exhaustive if exhaustive else lib.orc_convolve
    nptr, _keep = _nodes(nodes, ktab.size)
    _check(fn(nside, float(theta_cut), ktab.size, nptr, _d(ktab), _d(x), neval, pix_ptr, _d(y),
              _l(pairs)), "convolve")
    return (y, pairs) if return_pairs else y


def pair_counts(nside: int, theta_cut: float, pixels=None, exhaustive=False) -> np.ndarray:
    """In-disc pair count per output pixel."""
    _, pairs = convolve(nside, theta_cut, np.ones(2), np.zeros(npix(nside)), pixels,
                        exhaustive, return_pairs=True)
    return pairs


def map_grad(nside: int, theta_cut: float, ktab, g, nodes=None) -> np.ndarray:
    """dL/dx = A^T g.  The operator is symmetric (theta_pq = theta_qp and Omega
    is the same for every pixel), so A^T g is the same direct sum applied to g."""
    return convolve(nside, theta_cut, ktab, g, nodes=nodes)


def knot_grad(nside: int, theta_cut: float, ntab: int, x, g, nodes=None) -> np.ndarray:
    """dL/dK_k = Omega sum_p g[p] sum_q Lambda_k(theta_pq) x[q] (hat basis)."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.empty(ntab)
    nptr, _keep = _nodes(nodes, ntab)
    _check(_load().orc_knot_grad(nside, float(theta_cut), ntab, nptr, _d(x), _d(g), _d(out)),
           "knot_grad")
    return out


def legendre_coefficients(ktab, theta_cut: float, ells, order: int = 12, nodes=None
                          ) -> np.ndarray:
    """lambda_l = 2 pi int_0^theta_cut K_lin(theta) P_l(cos theta) sin(theta) dtheta.

    This is the Legendre transform operator of eq. 1 applied to the truncated,
    linearly interpolated real-space kernel.  By the Funk-Hecke theorem a
    band-limited Y_lm comes back from the continuous convolution scaled by
    lambda_l.  Quadrature: Gauss-Legendre of `order` points on each segment.
    """
    from scipy.special import eval_legendre

    ktab = np.asarray(ktab, dtype=np.float64)
    ntab = ktab.size
    if nodes is None:
        nodes = theta_cut * (np.arange(ntab) / (ntab - 1))
    nodes = np.asarray(nodes, dtype=np.float64)
    width = np.diff(nodes)[:, None]                 # segment widths
    xg, wg = np.polynomial.legendre.leggauss(order)
    tt = 0.5 * (xg + 1.0)                           # quadrature points on [0, 1]
    ww = 0.5 * wg
    theta = nodes[:-1, None] + tt[None, :] * width  # (ntab-1, order)
    kval = (1.0 - tt[None, :]) * ktab[:-1, None] + tt[None, :] * ktab[1:, None]
    base = 2.0 * np.pi * width * ww[None, :] * kval * np.sin(theta)
    ct = np.cos(theta)
    return np.array([np.sum(base * eval_legendre(int(l), ct)) for l in np.atleast_1d(ells)])


def harmonic(nside: int, khat, x) -> np.ndarray:
    """The harmonic-space half of the split (Sec. 2, eq. 1): Khat_l, l <= lcut =
    len(khat) - 1, applied by spherical-harmonic analysis with the pixel
    quadrature a_lm = Omega sum_p x_p conj(Y_lm(p)) and synthesis
    y_p = sum_l Khat_l sum_m a_lm Y_lm(p)."""
    khat = np.ascontiguousarray(khat, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if x.size != npix(nside):
        raise ValueError("map has %d pixels, Nside %d needs %d" % (x.size, nside, npix(nside)))
    y = np.empty_like(x)
    _check(_load().orc_harmonic(nside, khat.size - 1, _d(khat), _d(x), _d(y)), "harmonic")
    return y


def legendre_lm(lmax: int, theta: float) -> np.ndarray:
    """Orthonormal lambda_lm(cos theta), 0 <= m <= l <= lmax, as an
    (lmax+1, lmax+1) array indexed [l, m] (zero above the diagonal)."""
    out = np.zeros((lmax + 1, lmax + 1))
    _check(_load().orc_legendre_lm(lmax, float(theta), _d(out)), "legendre_lm")
    return out


def real_ylm(ell: int, m: int, vec) -> np.ndarray:
    """Unnormalised real spherical harmonic P_l^m(z) cos(m phi) at unit vectors."""
    from scipy.special import lpmv

    vec = np.asarray(vec, dtype=np.float64)
    z = np.clip(vec[:, 2], -1.0, 1.0)
    phi = np.arctan2(vec[:, 1], vec[:, 0])
    return lpmv(m, ell, z) * np.cos(m * phi)
