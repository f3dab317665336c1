"""Real-space spherical convolution on MI355X (gfx950).

Python binding of ``libarkcos.so`` (C ABI in ``include/arkcos.h``).  This layer
only marshals arguments: every step of the computation runs in the library's
HIP kernels.  PyTorch supplies device memory and the current stream.  There is
no CPU fallback: if the library is not built, importing the binding succeeds
but every call raises.

The operation is the real-space half of the split convolution of Sutter,
Wandelt & Elsner (2012), Sec. 2 (eq. 1, the ARKCoS term of eq. 3):

    out[p] = Omega * sum_{q : theta(p,q) < theta_cut} K(theta(p,q)) in[q]

on HEALPix RING maps, with K linear in theta between ntab nodes on
[0, theta_cut] (Sec. 3): uniform nodes, or the biased two-piece table of Sec. 3
(``paper_bias``, ``grid_nodes``).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = ["ArkcosError", "Plan", "Batch", "Harm", "split_convolve", "ArkcosConvFn", "conv",
           "tabulate_legendre",
           "tabulate_legendre_at", "grid_nodes", "paper_bias", "tune", "tune_key", "set_tune_cache", "ring_info", "gaussian_bl", "library_path", "load_library", "PLAN_HOST_ONLY",
           "PLAN_LEARNABLE", "PART_CIRCULANT", "PART_GENERAL", "PART_ALL", "MAX_GRAD_NTAB",
           "MAX_NSIDE"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libarkcos.so")
_TUNE_CACHE = os.path.join(_HERE, "tiles_gfx950.txt")

PLAN_HOST_ONLY = 1
PLAN_LEARNABLE = 2
PART_CIRCULANT = 1
PART_GENERAL = 2
PART_ALL = 3
MAX_NSIDE = 8192
MAX_GRAD_NTAB = 2048
MAX_LCUT = 4095

_STATUS = {0: "ARKCOS_OK", -1: "ARKCOS_EINVAL", -2: "ARKCOS_ENOMEM", -3: "ARKCOS_EDEVICE",
           -4: "ARKCOS_EUNSUPPORTED", -5: "ARKCOS_ESTATE"}


class ArkcosError(RuntimeError):
    """A libarkcos call returned a negative status."""

    def __init__(self, status: int, fn: str, detail: str):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (fn, _STATUS.get(status, status), detail))


class _Tiles(ctypes.Structure):
    _fields_ = [("gen_pixels", ctypes.c_int), ("gen_quad_window", ctypes.c_int),
                ("gen_pair_window", ctypes.c_int), ("reserved", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"gen_pixels": self.gen_pixels, "gen_quad_window": self.gen_quad_window,
                "gen_pair_window": self.gen_pair_window}


def _tiles(tiles) -> _Tiles:
    """arkcos_tiles from None (all 0: tuned or default) or a dict with any of
    gen_pixels, gen_quad_window, gen_pair_window."""
    if tiles is None:
        return _Tiles(0, 0, 0, 0)
    if isinstance(tiles, _Tiles):
        return tiles
    unknown = set(tiles) - {"gen_pixels", "gen_quad_window", "gen_pair_window"}
    if unknown:
        raise ValueError("unknown tile fields %s" % sorted(unknown))
    return _Tiles(int(tiles.get("gen_pixels", 0)), int(tiles.get("gen_quad_window", 0)),
                  int(tiles.get("gen_pair_window", 0)), 0)


class _PlanDesc(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("theta_cut", ctypes.c_double), ("ntab", ctypes.c_int),
                ("ktab", ctypes.POINTER(ctypes.c_double)), ("max_batch", ctypes.c_int),
                ("tiles", _Tiles), ("flags", ctypes.c_uint),
                ("theta_break", ctypes.c_double), ("k_break", ctypes.c_int),
                ("ring_first", ctypes.c_int), ("ring_last", ctypes.c_int)]


class _PlanInfo(ctypes.Structure):
    _fields_ = [("nside", ctypes.c_int), ("nrings", ctypes.c_int), ("npix", ctypes.c_longlong),
                ("ring_pairs", ctypes.c_longlong), ("tiles", ctypes.c_longlong),
                ("candidates", ctypes.c_longlong), ("omega", ctypes.c_double),
                ("ntab", ctypes.c_int), ("tile_shapes", _Tiles), ("tile_source", ctypes.c_int),
                ("flags", ctypes.c_uint),
                ("threads_per_block", ctypes.c_int), ("device_bytes", ctypes.c_longlong),
                ("circulant_rings", ctypes.c_int), ("general_rings", ctypes.c_int),
                ("circulant_tiles", ctypes.c_longlong), ("general_tiles", ctypes.c_longlong),
                ("weights", ctypes.c_longlong), ("theta_break", ctypes.c_double),
                ("k_break", ctypes.c_int), ("ring_first", ctypes.c_int),
                ("ring_last", ctypes.c_int), ("adjoint_ring_first", ctypes.c_int),
                ("adjoint_ring_last", ctypes.c_int), ("circ_form", ctypes.c_int)]


_lib = None
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libarkcos.so (built in-tree by ``python -m paper_1211_3556_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libarkcos.so is not built (%s); run `python -m "
                          "paper_1211_3556_amd.build` -- there is no CPU fallback" % _LIB_PATH)
    lib = ctypes.CDLL(_LIB_PATH)
    sig = {
        "arkcos_tabulate_legendre": [_dp, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp],
        "arkcos_tabulate_legendre_at": [_dp, ctypes.c_int, _dp, ctypes.c_int, _dp],
        "arkcos_grid_nodes": [ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp],
        "arkcos_ring_info": [ctypes.c_int, ctypes.c_int, _dp, _dp, _ip,
                             ctypes.POINTER(ctypes.c_longlong), _dp],
        "arkcos_plan_create": [ctypes.POINTER(_PlanDesc), ctypes.POINTER(_vp)],
        "arkcos_plan_destroy": [_vp],
        "arkcos_plan_get_info": [_vp, ctypes.POINTER(_PlanInfo)],
        "arkcos_plan_pair_count": [_vp, ctypes.POINTER(ctypes.c_ulonglong)],
        "arkcos_plan_window": [_vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip, _ip],
        "arkcos_plan_set_kernel_host": [_vp, _dp],
        "arkcos_plan_gen_tiles": [_vp, _ip, ctypes.c_longlong, ctypes.POINTER(ctypes.c_longlong)],
        "arkcos_plan_set_kernel": [_vp, _vp, _vp],
        "arkcos_convolve": [_vp, _vp, _vp, ctypes.c_int, _vp],
        "arkcos_convolve_part": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
        "arkcos_plan_pair_count_parts": [_vp, ctypes.POINTER(ctypes.c_ulonglong),
                                         ctypes.POINTER(ctypes.c_ulonglong)],
        "arkcos_convolve_backward": [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp],
        "arkcos_convolve_backward_static": [_vp, _vp, _vp, _vp, _vp, ctypes.c_int, _vp],
        "arkcos_batch_create": [ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp)],
        "arkcos_batch_convolve": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp],
        "arkcos_batch_convolve_part": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.c_int,
                                       _vp],
        "arkcos_batch_destroy": [_vp],
        "arkcos_harm_create": [ctypes.c_int, ctypes.c_int, _dp, ctypes.c_int, ctypes.POINTER(_vp)],
        "arkcos_harm_destroy": [_vp],
        "arkcos_harm_set_kernel": [_vp, _dp],
        "arkcos_harm_get_info": [_vp, _ip, _ip, ctypes.POINTER(ctypes.c_longlong),
                                 ctypes.POINTER(ctypes.c_longlong)],
        "arkcos_harm_convolve": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp],
        "arkcos_split_convolve": [_vp, _vp, _vp, _vp, ctypes.c_int, _vp],
        "arkcos_set_tune_cache": [ctypes.c_char_p],
        "arkcos_tune_key": [ctypes.c_int, ctypes.c_double, ctypes.c_char_p, ctypes.c_int, _ip],
        "arkcos_tune": [ctypes.POINTER(_PlanDesc), ctypes.c_int, ctypes.c_char_p,
                        ctypes.POINTER(_Tiles), _dp, _dp],
        "arkcos_rotation_to_pole": [ctypes.c_double, ctypes.c_double, _dp],
        "arkcos_rotate_map": [ctypes.c_int, _dp, _vp, _vp, ctypes.c_int, ctypes.c_int,
                              ctypes.c_int, _vp],
        "arkcos_status_string": [ctypes.c_int],
        "arkcos_last_error": [],
        "arkcos_version": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("arkcos_status_string", "arkcos_last_error") \
            else ctypes.c_int
    # plans with all-zero tiles read the tuning cache: ARKCOS_TUNE_CACHE if set,
    # else the cache measured for this package's target
    if "ARKCOS_TUNE_CACHE" not in os.environ and os.path.exists(_TUNE_CACHE):
        lib.arkcos_set_tune_cache(_TUNE_CACHE.encode())
    _lib = lib
    return lib


def _call(name: str, *args) -> None:
    lib = load_library()
    rc = getattr(lib, name)(*args)
    if rc != 0:
        detail = lib.arkcos_last_error().decode(errors="replace")
        raise ArkcosError(rc, name, detail)


def _stream_ptr(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(t, name: str):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != torch.float32:
        raise TypeError("%s must be float32, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t


def gaussian_bl(fwhm: float, lmax: int) -> np.ndarray:
    """Legendre coefficients b_l = exp(-l(l+1) sigma^2/2), sigma = FWHM/sqrt(8 ln 2), of the
    Gaussian beam of the paper's eq. 5 kernels with C_l = 1 (Sec. 3)."""
    sigma = fwhm / np.sqrt(8.0 * np.log(2.0))
    ell = np.arange(lmax + 1, dtype=np.float64)
    return np.exp(-0.5 * ell * (ell + 1.0) * sigma * sigma)


def tabulate_legendre(b_l, theta_cut: float, ntab: int) -> np.ndarray:
    """Host FP64 node table sum_l (2l+1)/(4 pi) b_l P_l(cos theta_k) (arkcos_tabulate_legendre)."""
    b = np.ascontiguousarray(b_l, dtype=np.float64)
    out = np.empty(ntab, dtype=np.float64)
    _call("arkcos_tabulate_legendre", b.ctypes.data_as(_dp), b.size - 1, float(theta_cut), ntab,
          out.ctypes.data_as(_dp))
    return out


def paper_bias(theta_cut: float, ntab: int) -> tuple[float, int]:
    """(theta_break, k_break) of the biased table of Sec. 3: half of the nodes
    (nodes 0..(ntab-1)//2) inside the first 1/16 of the support."""
    return theta_cut / 16.0, (ntab - 1) // 2


def grid_nodes(theta_cut: float, ntab: int, theta_break: float = 0.0, k_break: int = 0
               ) -> np.ndarray:
    """Node angles of a table (arkcos_grid_nodes): uniform for (0, 0), else two
    pieces, each uniform, meeting at node k_break = theta_break."""
    out = np.empty(ntab, dtype=np.float64)
    _call("arkcos_grid_nodes", float(theta_cut), int(ntab), float(theta_break), int(k_break),
          out.ctypes.data_as(_dp))
    return out


def tabulate_legendre_at(b_l, theta) -> np.ndarray:
    """sum_l (2l+1)/(4 pi) b_l P_l(cos theta) at the given angles (arkcos_tabulate_legendre_at)."""
    b = np.ascontiguousarray(b_l, dtype=np.float64)
    th = np.ascontiguousarray(theta, dtype=np.float64)
    out = np.empty(th.size, dtype=np.float64)
    _call("arkcos_tabulate_legendre_at", b.ctypes.data_as(_dp), b.size - 1,
          th.ctypes.data_as(_dp), th.size, out.ctypes.data_as(_dp))
    return out


def ring_info(nside: int, ring: int) -> dict:
    """Geometry of ring `ring` (1-based) as the library's plan computes it."""
    z, s, p0 = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    n, f = ctypes.c_int(), ctypes.c_longlong()
    _call("arkcos_ring_info", nside, ring, ctypes.byref(z), ctypes.byref(s), ctypes.byref(n),
          ctypes.byref(f), ctypes.byref(p0))
    return {"z": z.value, "sin_theta": s.value, "n": n.value, "first": f.value, "phi0": p0.value}


def set_tune_cache(path) -> None:
    """Tuning cache read by plans created with all-zero tiles (None: none)."""
    _call("arkcos_set_tune_cache", None if path is None else str(path).encode())


TUNE_RANGE_CLASS = 100   # ARKCOS_TUNE_RANGE_CLASS


def tune_key(nside: int, theta_cut: float, rings=None) -> tuple[str, int]:
    """(arch, window class) of the tuning-cache key of (nside, theta_cut); a
    ring range other than the whole sky adds TUNE_RANGE_CLASS."""
    buf = ctypes.create_string_buffer(64)
    cls = ctypes.c_int()
    _call("arkcos_tune_key", int(nside), float(theta_cut), buf, 64, ctypes.byref(cls))
    whole = rings is None or (rings[0] <= 1 and rings[1] >= 4 * int(nside) - 1)
    return buf.value.decode(), cls.value + (0 if whole else TUNE_RANGE_CLASS)


def tune(nside: int, theta_cut: float, ntab: int, ktab=None, reps: int = 5, cache=None,
         tiles=None, theta_break: float = 0.0, k_break: int = 0, rings=None) -> dict:
    """Autotune the general-gather tiles of a plan on the current device
    (arkcos_tune); appends the result to ``cache`` if given.  Returns the best
    tiles with their time and the defaults' time (ms per launch)."""
    k = None if ktab is None else np.ascontiguousarray(ktab, dtype=np.float64)
    desc = _PlanDesc(int(nside), float(theta_cut), int(ntab),
                     k.ctypes.data_as(_dp) if k is not None else None, 1, _tiles(tiles),
                     PLAN_LEARNABLE if k is None else 0, float(theta_break), int(k_break),
                     *((0, 0) if rings is None else (int(rings[0]), int(rings[1]))))
    best = _Tiles()
    bms, dms = ctypes.c_double(), ctypes.c_double()
    _call("arkcos_tune", ctypes.byref(desc), int(reps),
          None if cache is None else str(cache).encode(), ctypes.byref(best), ctypes.byref(bms),
          ctypes.byref(dms))
    return {"tiles": best.as_dict(), "ms": bms.value, "default_ms": dms.value}


class Plan:
    """A plan for one (Nside, theta_cut, node table) on the current device.

    ``ktab`` is a host FP64 node table of ``ntab`` values (copied); with
    ``learnable=True`` it may be omitted and knots set later with ``set_knots``.
    ``theta_break``/``k_break`` choose the node grid (0, 0: uniform; see
    ``grid_nodes`` and ``paper_bias``); ``biased=True`` is the Sec. 3 bias.
    ``rings=(first, last)`` (1-based, inclusive) restricts the output to a
    ring range (partial sky); other output pixels are left untouched.
    ``tiles`` (a dict of arkcos_tiles fields) fixes general-gather tile
    shapes; by default they come from the tuning cache (see ``tune``).
    """

    def __init__(self, nside: int, theta_cut: float, ktab=None, ntab: int | None = None,
                 max_batch: int = 1, tiles=None, learnable: bool = False,
                 host_only: bool = False, theta_break: float = 0.0, k_break: int = 0,
                 biased: bool = False, rings=None):
        if ktab is not None:
            ktab = np.ascontiguousarray(ktab, dtype=np.float64)
            ntab = ktab.size if ntab is None else ntab
            if ktab.size != ntab:
                raise ValueError("ktab has %d values, ntab is %d" % (ktab.size, ntab))
        if ntab is None:
            raise ValueError("give ktab or ntab")
        if biased:
            if theta_break or k_break:
                raise ValueError("give biased=True or theta_break/k_break, not both")
            theta_break, k_break = paper_bias(theta_cut, ntab)
        flags = (PLAN_LEARNABLE if learnable else 0) | (PLAN_HOST_ONLY if host_only else 0)
        desc = _PlanDesc(int(nside), float(theta_cut), int(ntab),
                         ktab.ctypes.data_as(_dp) if ktab is not None else None,
                         int(max_batch), _tiles(tiles), flags, float(theta_break), int(k_break),
                         *((0, 0) if rings is None else (int(rings[0]), int(rings[1]))))
        h = _vp()
        _call("arkcos_plan_create", ctypes.byref(desc), ctypes.byref(h))
        self._h = h
        self.nside = int(nside)
        self.theta_cut = float(theta_cut)
        self.ntab = int(ntab)
        self.theta_break = float(theta_break)
        self.k_break = int(k_break)
        self.max_batch = int(max_batch)
        self.learnable = learnable
        self.host_only = host_only
        self.rings = None if rings is None else (int(rings[0]), int(rings[1]))
        self.npix = 12 * self.nside * self.nside

    # -- lifetime -------------------------------------------------------------
    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().arkcos_plan_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- queries --------------------------------------------------------------
    def info(self) -> dict:
        inf = _PlanInfo()
        _call("arkcos_plan_get_info", self._h, ctypes.byref(inf))
        d = {k: getattr(inf, k) for k, _ in _PlanInfo._fields_}
        d["tile_shapes"] = inf.tile_shapes.as_dict()
        return d

    def nodes(self) -> np.ndarray:
        """Node angles of the plan's table."""
        return grid_nodes(self.theta_cut, self.ntab, self.theta_break, self.k_break)

    def pair_count(self) -> int:
        c = ctypes.c_ulonglong()
        _call("arkcos_plan_pair_count", self._h, ctypes.byref(c))
        return int(c.value)

    def pair_count_parts(self):
        """(pairs of circulant output rings, pairs of general output rings)."""
        c, g = ctypes.c_ulonglong(), ctypes.c_ulonglong()
        _call("arkcos_plan_pair_count_parts", self._h, ctypes.byref(c), ctypes.byref(g))
        return int(c.value), int(g.value)

    def gen_tiles(self) -> np.ndarray:
        """General-gather tiles: rows (tile, rings in tile, ring, first pixel, pixels)."""
        n = ctypes.c_longlong()
        _call("arkcos_plan_gen_tiles", self._h, None, 0, ctypes.byref(n))
        out = np.zeros((max(n.value, 1), 5), dtype=np.int32)
        _call("arkcos_plan_gen_tiles", self._h, out.ctypes.data_as(_ip), n.value, ctypes.byref(n))
        return out[:n.value]

    def window(self, ring_out: int, ring_src: int, j: int):
        lo, hi, cov = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _call("arkcos_plan_window", self._h, ring_out, ring_src, j, ctypes.byref(lo),
              ctypes.byref(hi), ctypes.byref(cov))
        return (lo.value, hi.value) if cov.value else None

    # -- kernel table ---------------------------------------------------------
    def set_ktab(self, ktab) -> None:
        k = np.ascontiguousarray(ktab, dtype=np.float64)
        if k.size != self.ntab:
            raise ValueError("expected %d node values" % self.ntab)
        _call("arkcos_plan_set_kernel_host", self._h, k.ctypes.data_as(_dp))

    def set_knots(self, knots, stream=None) -> None:
        """Stream-ordered replacement of the node table from device FP32 knots."""
        k = _dev_f32(knots, "knots")
        if k.numel() != self.ntab:
            raise ValueError("expected %d knots" % self.ntab)
        _call("arkcos_plan_set_kernel", self._h, _vp(k.data_ptr()), _stream_ptr(stream))

    # -- compute --------------------------------------------------------------
    def _shape(self, x):
        if x.dim() == 1 and x.numel() == self.npix:
            return 1
        if x.dim() == 2 and x.shape[1] == self.npix:
            return x.shape[0]
        raise ValueError("map must have shape (Npix,) or (B, Npix) with Npix = %d" % self.npix)

    def convolve(self, x, out=None, stream=None):
        """Forward convolution of a (Npix,) or (B, Npix) FP32 device tensor."""
        import torch
        x = _dev_f32(x, "x")
        nb = self._shape(x)
        if out is None:
            # a ring-range plan leaves the other rings as they are: zero here
            out = torch.zeros_like(x) if self.rings is not None else torch.empty_like(x)
        else:
            _dev_f32(out, "out")
            if out.shape != x.shape:
                raise ValueError("out must have the shape of x")
        _call("arkcos_convolve", self._h, _vp(x.data_ptr()), _vp(out.data_ptr()), nb,
              _stream_ptr(stream))
        return out

    def convolve_part(self, x, out, part: int, stream=None):
        """Run one gather (PART_CIRCULANT or PART_GENERAL) into `out`; the other
        gather's rings are left as they are."""
        x = _dev_f32(x, "x")
        nb = self._shape(x)
        _dev_f32(out, "out")
        if out.shape != x.shape:
            raise ValueError("out must have the shape of x")
        _call("arkcos_convolve_part", self._h, _vp(x.data_ptr()), _vp(out.data_ptr()), nb,
              int(part), _stream_ptr(stream))
        return out

    def backward(self, grad_out, x=None, want_map: bool = True, want_knots: bool = False,
                 stream=None, gx=None, gk=None, static_workspace: bool = False):
        """(dL/dx, dL/dknots) for dL/d(out) = grad_out; either may be None.

        ``gx``/``gk`` may be given as preallocated outputs.  With
        ``static_workspace=True`` the call goes to arkcos_convolve_backward_static,
        whose workspace is the library's per-device static array."""
        import torch
        g = _dev_f32(grad_out, "grad_out")
        nb = self._shape(g)
        if want_map:
            gx = torch.empty_like(g) if gx is None else _dev_f32(gx, "gx")
            if gx.shape != g.shape:
                raise ValueError("gx must have the shape of grad_out")
        else:
            gx = None
        if want_knots:
            gk = torch.empty(self.ntab, dtype=torch.float32, device=g.device) if gk is None \
                else _dev_f32(gk, "gk")
            if gk.numel() != self.ntab:
                raise ValueError("gk must hold ntab values")
        else:
            gk = None
        xp = _vp(_dev_f32(x, "x").data_ptr()) if x is not None else _vp()
        if want_knots and x is None:
            raise ValueError("knot gradients need the input map x")
        fn = "arkcos_convolve_backward_static" if static_workspace else "arkcos_convolve_backward"
        _call(fn, self._h, _vp(g.data_ptr()), xp,
              _vp(gx.data_ptr()) if gx is not None else _vp(),
              _vp(gk.data_ptr()) if gk is not None else _vp(), nb, _stream_ptr(stream))
        return gx, gk


def _make_conv_fn():
    import torch

    class ArkcosConvFn(torch.autograd.Function):
        """y = conv(x; knots) with the plan's geometry.  Backward gives dL/dx (the
        transposed gather) and dL/dknots (hat-basis gather), both on the GPU.  The
        knots are re-bound to the plan in backward, so optimiser steps between
        forward calls are safe."""

        @staticmethod
        def forward(ctx, x, knots, plan):
            plan.set_knots(knots.detach().contiguous())
            ctx.save_for_backward(x, knots)
            ctx.plan = plan
            return plan.convolve(x.contiguous())

        @staticmethod
        def backward(ctx, gy):
            x, knots = ctx.saved_tensors
            plan = ctx.plan
            want_x, want_k = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            if not (want_x or want_k):
                return None, None, None
            plan.set_knots(knots.detach().contiguous())
            gx, gk = plan.backward(gy.contiguous(), x.detach().contiguous() if want_k else None,
                                   want_map=want_x, want_knots=want_k)
            return gx, gk, None

    return ArkcosConvFn


_conv_fn = None


def __getattr__(name):
    # the autograd Function is created on first use so that importing the
    # binding does not import torch
    global _conv_fn
    if name == "ArkcosConvFn":
        if _conv_fn is None:
            _conv_fn = _make_conv_fn()
        return _conv_fn
    raise AttributeError(name)


def conv(x, plan: Plan, knots=None):
    """Convolve x with the plan's kernel; with ``knots`` (learnable plan), differentiable in
    both x and knots."""
    if knots is None:
        return plan.convolve(x)
    return __getattr__("ArkcosConvFn").apply(x, knots, plan)


class Batch:
    """Several plans (one map each) convolved in one persistent launch."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (_vp * len(self.plans))(*[p.handle for p in self.plans])
        h = _vp()
        _call("arkcos_batch_create", arr, len(self.plans), ctypes.byref(h))
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().arkcos_batch_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def convolve(self, xs, outs=None, stream=None, part: int = PART_ALL):
        """Convolve map k with plan k; `part` selects one of the two gathers."""
        import torch
        if len(xs) != len(self.plans):
            raise ValueError("need one map per plan")
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for p, x, o in zip(self.plans, xs, outs):
            _dev_f32(x, "x")
            _dev_f32(o, "out")
            if x.numel() != p.npix or o.numel() != p.npix:
                raise ValueError("map size does not match its plan")
        n = len(self.plans)
        ins = (_vp * n)(*[x.data_ptr() for x in xs])
        ous = (_vp * n)(*[o.data_ptr() for o in outs])
        _call("arkcos_batch_convolve_part", self._h, ins, ous, int(part), _stream_ptr(stream))
        return outs


class Harm:
    """The harmonic-space half of a split convolution (arkcos_harm_*): Khat_l,
    l <= lcut = len(khat) - 1, applied by spherical-harmonic analysis (pixel
    quadrature) and synthesis on the GPU."""

    def __init__(self, nside: int, khat, max_batch: int = 1):
        k = np.ascontiguousarray(khat, dtype=np.float64)
        if k.ndim != 1 or k.size < 1:
            raise ValueError("khat must be a 1-D array of lcut + 1 values")
        h = _vp()
        _call("arkcos_harm_create", int(nside), k.size - 1, k.ctypes.data_as(_dp), int(max_batch),
              ctypes.byref(h))
        self._h = h
        self.nside = int(nside)
        self.lcut = k.size - 1
        self.npix = 12 * self.nside * self.nside
        self.max_batch = int(max_batch)

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            load_library().arkcos_harm_destroy(self._h)
            self._h = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n, lc = ctypes.c_int(), ctypes.c_int()
        na, db = ctypes.c_longlong(), ctypes.c_longlong()
        _call("arkcos_harm_get_info", self._h, ctypes.byref(n), ctypes.byref(lc),
              ctypes.byref(na), ctypes.byref(db))
        return {"nside": n.value, "lcut": lc.value, "nalm": na.value, "device_bytes": db.value}

    def set_kernel(self, khat) -> None:
        k = np.ascontiguousarray(khat, dtype=np.float64)
        if k.size != self.lcut + 1:
            raise ValueError("khat must have lcut + 1 = %d values" % (self.lcut + 1))
        _call("arkcos_harm_set_kernel", self._h, k.ctypes.data_as(_dp))

    def _shape(self, x):
        if x.dim() == 1 and x.numel() == self.npix:
            return 1
        if x.dim() == 2 and x.shape[1] == self.npix:
            return x.shape[0]
        raise ValueError("map must have shape (Npix,) or (B, Npix) with Npix = %d" % self.npix)

    def convolve(self, x, out=None, accumulate: bool = False, stream=None):
        """The l-space half of a (Npix,) or (B, Npix) FP32 device tensor, written
        to `out` or (accumulate=True) added to it."""
        import torch
        x = _dev_f32(x, "x")
        nb = self._shape(x)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs an out tensor")
            out = torch.empty_like(x)
        else:
            _dev_f32(out, "out")
            if out.shape != x.shape:
                raise ValueError("out must have the shape of x")
        _call("arkcos_harm_convolve", self._h, _vp(x.data_ptr()), _vp(out.data_ptr()), nb,
              1 if accumulate else 0, _stream_ptr(stream))
        return out


def split_convolve(plan: Plan, harm: Harm, x, out=None, stream=None):
    """The full split convolution (arkcos_split_convolve): the real-space half
    of `plan` plus the l-space half of `harm`."""
    import torch
    x = _dev_f32(x, "x")
    nb = plan._shape(x)
    if out is None:
        out = torch.empty_like(x)
    else:
        _dev_f32(out, "out")
        if out.shape != x.shape:
            raise ValueError("out must have the shape of x")
    _call("arkcos_split_convolve", plan.handle, harm.handle, _vp(x.data_ptr()),
          _vp(out.data_ptr()), nb, _stream_ptr(stream))
    return out


def rotation_to_pole(theta: float, phi: float) -> np.ndarray:
    """The 3x3 rotation taking the direction (theta, phi) to the north pole
    (arkcos_rotation_to_pole)."""
    r = np.empty(9)
    _call("arkcos_rotation_to_pole", float(theta), float(phi), r.ctypes.data_as(_dp))
    return r.reshape(3, 3)


def rotate_map(nside: int, rot, x, out=None, rings=None, stream=None):
    """Rotated copy of FP32 RING map(s) on the GPU, resampled at the nearest
    pixel (arkcos_rotate_map): out[p] = x[pixel containing R^T n_p] for the
    pixels of ``rings`` (1-based, inclusive; all by default)."""
    import torch
    x = _dev_f32(x, "x")
    npix = 12 * nside * nside
    if x.shape[-1] != npix or x.dim() > 2:
        raise ValueError("x must hold one or more maps of 12 nside^2 pixels")
    nb = 1 if x.dim() == 1 else x.shape[0]
    if out is None:
        out = torch.zeros_like(x)
    else:
        _dev_f32(out, "out")
        if out.shape != x.shape:
            raise ValueError("out must have the shape of x")
    r = np.ascontiguousarray(rot, dtype=np.float64).reshape(9)
    lo, hi = (0, 0) if rings is None else (int(rings[0]), int(rings[1]))
    _call("arkcos_rotate_map", int(nside), r.ctypes.data_as(_dp), _vp(x.data_ptr()),
          _vp(out.data_ptr()), nb, lo, hi, _stream_ptr(stream))
    return out
