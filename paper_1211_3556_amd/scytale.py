"""Kernel splitting for the split convolution: the scytale tool of Sec. 2, on MI355X.

The paper splits a radial kernel K_l into a truncated harmonic-space part
Khat_l (l <= l_cut) and a truncated real-space part Khat_theta
(theta < theta_cut), so that (eq. 1)

    Ktilde_l = Khat_l + P_{l theta} Khat_theta,

estimates the error of the approximation by a fractional rms (eq. 2) and
chooses (l_cut, theta_cut) that meet an error bound at the lowest cost, with
the cost of each half measured on the hardware (eq. 3, eq. 4).  This module
does the same for the two halves built here:

* ``legendre_matrix`` -- P_{l theta} of the hat basis of a node table:
  column k holds 2 pi int Lambda_k(theta) P_l(cos theta) sin(theta) dtheta;
* ``split_kernel`` -- a split for given (l_cut, theta_cut).  The paper does not
  say how its splits were made; here Khat_theta is the kernel's content above
  l_cut as a real-space profile on a biased table, cut at theta_cut, and
  Khat_l = K_l - P_{l theta} Khat_theta below l_cut absorbs the rest exactly,
  so only the theta truncation leaves an error (above l_cut).  Applied to
  band-limited noise by the two GPU halves, the map error of such a split is
  the eq. 2 estimate divided by alpha, to a few per cent;
* ``error_estimate`` -- eq. 2 with C_l = 1 input power:
  sigma = alpha sqrt(sum (2l+1)(Ktilde_l - K_l)^2 / sum (2l+1) K_l^2);
* ``CostModel`` -- the two halves' times on MI355X from measurements
  (``measure_costs``): the real-space half interpolated in theta_cut, the
  harmonic half fitted to t_harm = c + d (l_cut + 1) Npix + e n_alm Nside;
  ``PaperCostModel`` holds the paper's own eq. 3 and eq. 4;
* ``optimise`` -- the cheapest (l_cut, theta_cut) on a grid whose estimated
  error meets the bound (both halves run on the GPU, one after the other, so
  the cost is their sum).

Everything here is host-side planning in FP64 numpy; the two halves
themselves run in the library's GPU kernels (``Plan``, ``Harm``,
``split_convolve``).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

COST_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cost_mi355x.json")


def legendre_matrix(nodes, lmax: int, order: int = 4) -> np.ndarray:
    """(lmax+1, ntab) matrix T with T[l, k] = 2 pi int Lambda_k P_l(cos) sin:
    the Legendre transform (eq. 1's P_{l theta}) of the hat function of node
    k of a piecewise-linear table on `nodes`.  Gauss-Legendre with `order`
    points on every node interval; P_l by the three-term recurrence."""
    nodes = np.asarray(nodes, dtype=np.float64)
    xg, wg = np.polynomial.legendre.leggauss(order)
    t = 0.5 * (xg + 1.0)
    w = 0.5 * wg
    h = np.diff(nodes)
    th = nodes[:-1, None] + t[None, :] * h[:, None]
    a = 2.0 * np.pi * w[None, :] * h[:, None] * np.sin(th)
    wl = a * (1.0 - t)[None, :]      # weight of the interval's left node
    wr = a * t[None, :]              # and of its right node
    x = np.cos(th)
    T = np.zeros((lmax + 1, nodes.size))
    pm1, p = np.ones_like(x), x.copy()
    for l in range(lmax + 1):
        if l == 0:
            P = pm1
        elif l == 1:
            P = p
        else:
            P = ((2 * l - 1) * x * p - (l - 1) * pm1) / l
            pm1, p = p, P
        T[l, :-1] += (P * wl).sum(axis=1)
        T[l, 1:] += (P * wr).sum(axis=1)
    return T


def error_estimate(K, Ktilde, alpha: float = 5.0) -> float:
    """Eq. 2 with flat input power (C_l = 1): alpha times the fractional rms of
    Ktilde_l - K_l, each l weighted by its 2l+1 modes.  alpha = 5 is the
    paper's empirical factor for single precision and interpolation."""
    K = np.asarray(K, dtype=np.float64)
    Kt = np.asarray(Ktilde, dtype=np.float64)
    w = 2.0 * np.arange(K.size) + 1.0
    return float(alpha * np.sqrt(np.sum(w * (Kt - K) ** 2) / np.sum(w * K * K)))


@dataclass
class Split:
    """A split of K_l: the real-space table on `nodes` and the l-space part."""
    lcut: int
    theta_cut: float
    nodes: np.ndarray            # node angles of Khat_theta (radians), biased table
    khat_theta: np.ndarray       # table values at the nodes
    khat_l: np.ndarray           # Khat_l, l = 0..lcut
    ktilde: np.ndarray           # eq. 1's approximate kernel, l = 0..lmax
    sigma: float                 # eq. 2 estimate
    low_l_share: float           # rms of P_{l theta} Khat_theta over rms of K_l, l <= lcut
    theta_break: float = 0.0
    k_break: int = 0


def biased_grid(theta_cut: float, ntab: int) -> tuple[np.ndarray, float, int]:
    """Node angles of the Sec. 3 biased table (half of the nodes within
    theta_cut/16) and its (theta_break, k_break)."""
    from . import grid_nodes, paper_bias
    tb, kb = paper_bias(theta_cut, ntab)
    return grid_nodes(theta_cut, ntab, tb, kb), tb, kb


def split_kernel(K, lcut: int, theta_cut: float, ntab: int = 2049, alpha: float = 5.0,
                 T=None) -> Split:
    """Split K_l (l = 0..lmax) at (lcut, theta_cut).  The real-space part is
    the kernel's content above lcut, sum_{l > lcut} (2l+1)/(4 pi) K_l
    P_l(cos theta), tabulated on a biased table and cut at theta_cut; the
    l-space part Khat_l = K_l - (P_{l theta} Khat_theta)_l, l <= lcut, makes
    Ktilde_l = K_l exactly below the cut, so the error is what the truncation
    in theta leaves above it."""
    from . import tabulate_legendre_at
    K = np.asarray(K, dtype=np.float64)
    lmax = K.size - 1
    if not (0 <= lcut < lmax):
        raise ValueError("need 0 <= lcut < lmax")
    nodes, tb, kb = biased_grid(theta_cut, ntab)
    high = np.where(np.arange(lmax + 1) > lcut, K, 0.0)
    table = tabulate_legendre_at(high, nodes)
    if T is None:
        T = legendre_matrix(nodes, lmax)
    real_l = T @ table
    khat_l = K[:lcut + 1] - real_l[:lcut + 1]
    ktilde = real_l.copy()
    ktilde[:lcut + 1] += khat_l
    w = 2.0 * np.arange(lmax + 1) + 1.0
    low = float(np.sqrt(np.sum((w * real_l ** 2)[:lcut + 1]) / np.sum((w * K ** 2)[:lcut + 1])))
    return Split(lcut=lcut, theta_cut=theta_cut, nodes=nodes, khat_theta=table, khat_l=khat_l,
                 ktilde=ktilde, sigma=error_estimate(K, ktilde, alpha), low_l_share=low,
                 theta_break=tb, k_break=kb)


# ------------------------------------------------------------------ costs --

@dataclass
class CostModel:
    """Measured times of the two halves on one MI355X (ms), at one Nside.
    The real-space half is interpolated in theta_cut between the measured
    cuts (log-log, extrapolated with the end slopes): its time is not linear
    in the pair count, since larger discs turn more rings general.  The
    harmonic half is fitted as t_harm = c + d (l_cut + 1) Npix + e n_alm Nside,
    n_alm = (l_cut+1)(l_cut+2)/2 (longitude and Legendre steps).  Both halves
    run on the GPU one after the other, so a split costs their sum."""
    nside: int
    real: list          # [(theta_cut_arcmin, pairs, ms)], increasing theta_cut
    c: float
    d: float
    e: float
    harm: list = field(default_factory=list)   # [(l_cut, ms)] measured

    def t_real(self, theta_cut: float) -> float:
        am = theta_cut * 180.0 * 60.0 / np.pi
        lx = np.log([r[0] for r in self.real])
        ly = np.log([r[2] for r in self.real])
        v = np.log(am)
        if v <= lx[0]:
            i = 0
        elif v >= lx[-1]:
            i = len(lx) - 2
        else:
            i = int(np.searchsorted(lx, v)) - 1
        slope = (ly[i + 1] - ly[i]) / (lx[i + 1] - lx[i])
        return float(np.exp(ly[i] + slope * (v - lx[i])))

    def t_harm(self, lcut: int) -> float:
        npix = 12.0 * self.nside ** 2
        nalm = (lcut + 1.0) * (lcut + 2.0) / 2.0
        return self.c + self.d * (lcut + 1.0) * npix + self.e * nalm * self.nside

    def total(self, lcut: int, theta_cut: float) -> float:
        return self.t_real(theta_cut) + self.t_harm(lcut)

    @staticmethod
    def fit(nside: int, real: list, harm: list) -> "CostModel":
        """real: [(theta_cut_arcmin, pairs, ms)], harm: [(l_cut, ms)]."""
        npix = 12.0 * nside ** 2
        ph = np.array([[1.0, (l + 1.0) * npix, (l + 1.0) * (l + 2.0) / 2.0 * nside]
                       for l, _ in harm])
        c, d, e = np.linalg.lstsq(ph, np.array([m for _, m in harm]), rcond=None)[0]
        return CostModel(nside, sorted([list(map(float, r)) for r in real]), float(c), float(d),
                         float(e), [list(map(float, r)) for r in harm])

    def save(self, path: str = COST_FILE) -> None:
        with open(path, "w") as f:
            json.dump(self.__dict__, f, indent=1)

    @staticmethod
    def load(path: str = COST_FILE) -> "CostModel":
        with open(path) as f:
            return CostModel(**json.load(f))


@dataclass
class PaperCostModel:
    """The paper's cost models (eq. 3: a GTX 480 for the real-space half,
    theta_cut in arcmin; eq. 4: one 2.8 GHz core with libpsht for the
    l-space half, l_max the map band limit), in ms; the halves run in
    parallel, so a split costs the slower one."""
    lmax: int = 4096

    def t_real(self, theta_cut: float) -> float:
        return 1e3 * (0.0232 * theta_cut * 180.0 * 60.0 / np.pi + 2.428)

    def t_harm(self, lcut: int) -> float:
        return 1e3 * 160.0 * lcut ** 2 * self.lmax / 4096.0 ** 3

    def total(self, lcut: int, theta_cut: float) -> float:
        return max(self.t_real(theta_cut), self.t_harm(lcut))


def measure_costs(nside: int = 2048, theta_cuts_arcmin=(30, 60, 120, 240, 390),
                  lcuts=(250, 500, 1000, 1500, 2000, 3000), ntab: int = 16384,
                  reps: int = 3) -> CostModel:
    """Time both halves on the current GPU (HIP events on the current stream)
    and fit the cost model.  The tables are placeholders of the right size
    (costs do not depend on the values)."""
    import torch
    from . import Harm, Plan
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(0)
    x = torch.randn(12 * nside * nside, generator=gen, device="cuda")
    y = torch.empty_like(x)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    real = []
    for tc_am in theta_cuts_arcmin:
        tc = tc_am * np.pi / 180.0 / 60.0
        p = Plan(nside, tc, np.exp(-np.linspace(0.0, 3.0, ntab)), biased=True)
        real.append((float(tc_am), float(p.pair_count()), timed(lambda: p.convolve(x, y))))
        del p
    harm = []
    for lc in lcuts:
        h = Harm(nside, np.ones(lc + 1))
        harm.append((lc, timed(lambda: h.convolve(x, y))))
        del h
    return CostModel.fit(nside, real, harm)


def optimise(K, cost, bound: float = 1e-5, lcuts=None, theta_cuts=None,
             ntab: int = 2049, alpha: float = 5.0) -> dict:
    """The cheapest (l_cut, theta_cut) on the grid whose eq. 2 estimate meets
    `bound` under `cost` (a CostModel, or the paper's PaperCostModel);
    returns the choice, its split, and every grid point scanned."""
    K = np.asarray(K, dtype=np.float64)
    lmax = K.size - 1
    if lcuts is None:
        lcuts = list(range(250, lmax, 250))
    if theta_cuts is None:
        theta_cuts = [m * np.pi / 180.0 / 60.0 for m in range(30, 481, 30)]
    rows = []
    best = None
    for tc in theta_cuts:
        nodes, _, _ = biased_grid(tc, ntab)
        T = legendre_matrix(nodes, lmax)
        for lc in lcuts:
            s = split_kernel(K, lc, tc, ntab, alpha, T=T)
            t = cost.total(lc, tc)
            rows.append({"lcut": lc, "theta_cut_arcmin": tc * 180.0 * 60.0 / np.pi,
                         "sigma": s.sigma, "low_l_share": s.low_l_share, "ms": t})
            if s.sigma <= bound and (best is None or t < best[0]):
                best = (t, s)
    out = {"grid": rows, "bound": bound}
    if best is not None:
        out.update({"ms": best[0], "lcut": best[1].lcut,
                    "theta_cut_arcmin": best[1].theta_cut * 180.0 * 60.0 / np.pi,
                    "sigma": best[1].sigma, "split": best[1]})
    return out


def cmb_like_cl(lmax: int, l_damp: float = 1400.0) -> np.ndarray:
    """A synthetic stand-in for a CMB power spectrum (the paper uses a WMAP
    7-year spectrum, not available here): scale invariant, C_l ~ 1/(l(l+1)),
    with a Gaussian damping tail at l_damp; C_0 = C_1 = C_2."""
    ell = np.arange(lmax + 1, dtype=np.float64)
    c = np.empty(lmax + 1)
    c[2:] = 110.0 / (ell[2:] * (ell[2:] + 1.0)) * np.exp(-(ell[2:] / l_damp) ** 2)
    c[:2] = c[2]
    return c


def main(argv=None) -> int:
    import argparse
    ap = argparse.ArgumentParser(description="kernel splitting on MI355X")
    sub = ap.add_subparsers(dest="cmd", required=True)
    me = sub.add_parser("measure", help="time both halves on the GPU and write the cost model")
    me.add_argument("--out", default=COST_FILE)
    op = sub.add_parser("optimise", help="optimum splits of Gaussian-beam kernels")
    op.add_argument("--fwhm", type=float, nargs="+", default=[5, 7, 10, 15])
    op.add_argument("--lmax", type=int, default=4096)
    op.add_argument("--bound", type=float, default=1e-5)
    op.add_argument("--paper-costs", action="store_true",
                    help="use the paper's eq. 3 / eq. 4 costs (halves in parallel)")
    args = ap.parse_args(argv)
    if args.cmd == "measure":
        m = measure_costs()
        m.save(args.out)
        print(json.dumps(m.__dict__, indent=1))
        return 0
    cost = PaperCostModel(args.lmax) if args.paper_costs else CostModel.load()
    ell = np.arange(args.lmax + 1)
    for fw in args.fwhm:
        sig = fw * np.pi / 180.0 / 60.0 / np.sqrt(8.0 * np.log(2.0))
        K = np.sqrt(cmb_like_cl(args.lmax)) * np.exp(-0.5 * ell * (ell + 1.0) * sig * sig)
        r = optimise(K, cost, args.bound)
        if "lcut" in r:
            print("FWHM %4.1f': l_cut %4d theta_cut %5.0f' sigma %.2e cost %.1f ms"
                  % (fw, r["lcut"], r["theta_cut_arcmin"], r["sigma"], r["ms"]))
        else:
            print("FWHM %4.1f': no split meets %.0e on the grid" % (fw, args.bound))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
