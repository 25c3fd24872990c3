"""Seeded synthetic inputs for IBMI: covariance matrices, batches and request streams.

This module builds inputs only.  It holds none of the arithmetic of the IBMI method
(no factorisation, no block update, no residual), so both the CPU oracle and the HIP
path may draw their inputs from it.

Covariance kernels follow Table 1 of the paper (exponential, RBF / squared exponential,
inverse quadratic, Matern 3/2, Matern 5/2), with the length scale written ``ell``.
Points are drawn uniformly in [0, 1]^d and sorted along the first coordinate before the
matrix is built, which keeps most of the weight near the diagonal (the paper's advice in
its section on properties affecting convergence; its red-black experiment shows that
scattering neighbours hurts).  A nugget ``tau * I`` is added to the diagonal afterwards.

Every generator takes an explicit seed and draws from NumPy's PCG64 ``default_rng``
in a fixed, documented order, so the same call always yields the same bits.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "sorted_points", "pairwise_distance", "kernel_matrix", "covariance", "covariance_row_chunks",
    "config1_matrix", "config2_matrix", "config3_matrix", "config4_batch",
    "config5_arrivals", "request_matrix", "wishart_spd", "CONFIGS", "Workload", "Request",
]

KERNELS = ("exp", "se", "iquad", "matern32", "matern52")


def sorted_points(n: int, dim: int, rng: np.random.Generator) -> np.ndarray:
    """n points uniform in [0,1]^dim (one draw of shape (n, dim)), sorted by coordinate 0."""
    pts = rng.uniform(0.0, 1.0, size=(n, dim)) if dim > 1 else rng.uniform(0.0, 1.0, size=(n, 1))
    order = np.argsort(pts[:, 0], kind="stable")
    return np.ascontiguousarray(pts[order])


def pairwise_distance(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Euclidean distances |x_i - y_j| computed coordinate by coordinate in FP64."""
    d2 = np.zeros((x.shape[0], y.shape[0]), dtype=np.float64)
    for c in range(x.shape[1]):
        diff = x[:, c][:, None] - y[:, c][None, :]
        d2 += diff * diff
    return np.sqrt(d2)


def _kernel_of_distance(r: np.ndarray, kind: str, ell: float, variance: float) -> np.ndarray:
    """Table 1 kernels as functions of the distance r."""
    if kind == "exp":
        return variance * np.exp(-r / ell)
    if kind == "se":
        return variance * np.exp(-(r * r) / (2.0 * ell * ell))
    if kind == "iquad":
        return variance / np.sqrt(1.0 + (r / ell) ** 2)
    if kind == "matern32":
        z = math.sqrt(3.0) * r / ell
        return variance * (1.0 + z) * np.exp(-z)
    if kind == "matern52":
        z = math.sqrt(5.0) * r / ell
        return variance * (1.0 + z + z * z / 3.0) * np.exp(-z)
    raise ValueError(f"unknown kernel {kind!r}; expected one of {KERNELS}")


def kernel_matrix(pts: np.ndarray, kind: str, ell: float, variance: float = 1.0,
                  row_chunk: int = 2048) -> np.ndarray:
    """Dense kernel matrix K(pts, pts) in FP64, built in row chunks to bound memory.

    The result is exactly symmetric without any mirroring: (x_i - x_j)^2 and (x_j - x_i)^2
    are the same IEEE number, the coordinates are summed in the same order, and the kernel
    is an elementwise function of the distance.
    """
    n = pts.shape[0]
    out = np.empty((n, n), dtype=np.float64)
    for r0 in range(0, n, row_chunk):
        r1 = min(n, r0 + row_chunk)
        out[r0:r1] = _kernel_of_distance(pairwise_distance(pts[r0:r1], pts), kind, ell, variance)
    return out


def covariance_row_chunks(pts: np.ndarray, kind: str, ell: float, nugget: float,
                          variance: float = 1.0, row_chunk: int = 2048):
    """The rows of ``covariance(pts, ...)`` in chunks: yields (r0, r1, rows r0..r1-1), the
    same bits as the full matrix, for matrices too large to hold on the host at once."""
    n = pts.shape[0]
    for r0 in range(0, n, row_chunk):
        r1 = min(n, r0 + row_chunk)
        rows = _kernel_of_distance(pairwise_distance(pts[r0:r1], pts), kind, ell, variance)
        rows[np.arange(r1 - r0), np.arange(r0, r1)] += nugget
        yield r0, r1, rows


def covariance(pts: np.ndarray, kind: str, ell: float, nugget: float,
               variance: float = 1.0) -> np.ndarray:
    """Kernel matrix plus ``nugget * I`` (added to the diagonal after the kernel)."""
    a = kernel_matrix(pts, kind, ell, variance)
    a[np.diag_indices_from(a)] += nugget
    return a


# --------------------------------------------------------------------------------------
# The five benchmark workloads.  Seed = workload number unless stated otherwise.
# --------------------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    p: int
    block_rows: int
    overlap: int
    init: str          # "identity" | "blockdiag_inv"
    tol: float
    max_sweeps: int


CONFIGS = {
    1: Workload("exp1d_p256_two_blocks_fp64", 256, 128, 0, "blockdiag_inv", 1e-10, 200),
    2: Workload("matern32_2d_p4096_k8_fp64", 4096, 576, 64, "identity", 1e-10, 500),
    3: Workload("se_2d_p16384_k32", 16384, 576, 64, "identity", 1e-10, 500),
    4: Workload("batched_wishart_256", 0, 128, 16, "identity", 1e-8, 500),
    5: Workload("serving_matern32_2d", 0, 576, 64, "identity", 1e-10, 500),
}


def config1_matrix(seed: int = 1, p: int = 256) -> np.ndarray:
    """Exponential covariance exp(-|x-x'|/0.2) on p sorted uniform points in [0,1], + 1e-2 I."""
    rng = np.random.default_rng(seed)
    x = sorted_points(p, 1, rng)
    return covariance(x, "exp", 0.2, 1e-2)


def config2_matrix(seed: int = 2, p: int = 4096) -> np.ndarray:
    """Matern-3/2 (ell 0.1, variance 1) on p points in the unit square sorted by x, + 1e-2 I."""
    rng = np.random.default_rng(seed)
    pts = sorted_points(p, 2, rng)
    return covariance(pts, "matern32", 0.1, 1e-2)


def config3_matrix(seed: int = 3, p: int = 16384) -> np.ndarray:
    """Squared exponential (ell 0.05) on p points in the unit square sorted by x, + 1e-3 I."""
    rng = np.random.default_rng(seed)
    pts = sorted_points(p, 2, rng)
    return covariance(pts, "se", 0.05, 1e-3)


def _config4_sizes(seed: int, n: int, lo: int, hi: int):
    """Matrix orders p_j = round(exp(U[ln lo, ln hi])), drawn first, before any matrix."""
    rng = np.random.default_rng(seed)
    sizes = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=n))).astype(np.int64)
    return sizes, rng


def config4_batch(seed: int = 4, n: int = 256, lo: int = 128, hi: int = 2048,
                  sizes_only: bool = False):
    """n Wishart-type SPD matrices A = G G^T / p + 0.1 I with G (p x p) i.i.d. N(0,1).

    Orders are log-uniform in [lo, hi]; all orders are drawn first, then the G's in order.
    Returns the list of matrices (or only the orders when ``sizes_only``).
    """
    sizes, rng = _config4_sizes(seed, n, lo, hi)
    if sizes_only:
        return sizes
    mats = []
    for p in sizes:
        g = rng.standard_normal(size=(int(p), int(p)))
        a = (g @ g.T) / float(p)
        a = 0.5 * (a + a.T)
        a[np.diag_indices_from(a)] += 0.1
        mats.append(a)
    return mats


@dataclass(frozen=True)
class Request:
    rid: int
    arrival_s: float
    p: int
    tol: float
    seed: int


def config5_arrivals(seed: int = 5, rate_hz: float = 200.0, duration_s: float = 60.0,
                     lo: int = 512, hi: int = 8192) -> list:
    """Poisson arrivals (exponential gaps, mean 1/rate) of Matern-3/2 inversion requests.

    Per request, in this order: the gap, p = round(exp(U[ln lo, ln hi])), the tolerance
    (1e-6 or 1e-10 with equal probability) and a 32-bit seed for its own point set.
    """
    rng = np.random.default_rng(seed)
    out, t, rid = [], 0.0, 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        p = int(np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi)))))
        tol = 1e-6 if rng.uniform() < 0.5 else 1e-10
        s = int(rng.integers(0, 2**31 - 1))
        out.append(Request(rid, t, p, tol, s))
        rid += 1
    return out


def request_matrix(req: Request) -> np.ndarray:
    """The covariance matrix of one serving request (Matern-3/2, ell 0.1, + 1e-2 I)."""
    rng = np.random.default_rng(req.seed)
    pts = sorted_points(req.p, 2, rng)
    return covariance(pts, "matern32", 0.1, 1e-2)


def wishart_spd(p: int, rng: np.random.Generator, shift: float = 0.1, extra_cols: int = 0):
    """Random SPD test matrix G G^T / n + shift I (G is p x (p + extra_cols)), exactly symmetric."""
    g = rng.standard_normal(size=(p, p + extra_cols))
    a = (g @ g.T) / float(p + extra_cols)
    a = 0.5 * (a + a.T)
    a[np.diag_indices_from(a)] += shift
    return a
