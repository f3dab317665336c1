"""Helpers shared by the GPU parity tests."""
import sys

import numpy as np

import oracle as O
import workloads as W


def log(msg: str) -> None:
    """Name the case before a GPU step, flushed, so a fault still identifies it."""
    sys.stdout.write("[gpu] %s\n" % msg)
    sys.stdout.flush()


def rel_rms(got, ref) -> float:
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.sqrt(np.sum((got - ref) ** 2) / np.sum(ref ** 2)))


def oracle_table(spec: W.MapSpec) -> np.ndarray:
    """Node table of a Gaussian-beam workload, from the oracle's own tabulation."""
    return O.tabulate(O.gaussian_bl(spec.fwhm, spec.ell_max), spec.theta_cut, spec.ntab)


def gpu_table(spec: W.MapSpec) -> np.ndarray:
    """Node table of a Gaussian-beam workload, from the library's own tabulation."""
    import paper_1211_3556_amd as A
    return A.tabulate_legendre(A.gaussian_bl(spec.fwhm, spec.ell_max), spec.theta_cut, spec.ntab)


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


# Relative rms error bar of a GPU output against the FP64 oracle on the same
# pixels (the accuracy target of the real-space path, well inside the
# 1e-5 fractional error budget of the paper's split method).
REL_RMS_TOL = 1e-6


def angle_condition(theta_cut: float, ktab, nodes=None, samples: int = 200001) -> float:
    """kappa = rms(theta K'(theta)) / rms(K(theta)) over the disc (area weight
    sin theta), from the oracle's interpolated kernel.  An FP32 angle with
    relative error e moves a weight by e theta K', so a direct sum over white
    noise carries a relative rms error of about e kappa."""
    th = np.linspace(0.0, theta_cut, samples)[:-1]
    k = O.kernel_eval(theta_cut, ktab, th, nodes=nodes)
    dk = np.gradient(k, th)
    w = np.sin(th)
    return float(np.sqrt(np.sum((th * dk) ** 2 * w) / np.sum(k * k * w)))


def angle_tolerance(theta_cut: float, ktab, nodes=None) -> float:
    """Relative rms error bar of a GPU output for a kernel of angle condition
    kappa: REL_RMS_TOL, or 2 eps_32 kappa where that is larger.  The FP32 chord
    and angle series of the general gather round about six times, each within
    eps_32/2, so the angle's relative rms error stays below 2 eps_32."""
    eps = float(np.finfo(np.float32).eps)
    return max(REL_RMS_TOL, 2.0 * eps * angle_condition(theta_cut, ktab, nodes))


def assert_tie_free(nside: int, theta_cut: float, rel: float = 1e-7) -> None:
    """No pixel pair sits on the cut: at such lattice ties the strict test
    theta < theta_cut is decided by the last bit of either computation."""
    lo = O.pair_counts(nside, theta_cut * (1 - rel)).sum()
    hi = O.pair_counts(nside, theta_cut * (1 + rel)).sum()
    assert lo == hi, "cut-off %.6g rad has lattice ties at Nside %d" % (theta_cut, nside)
