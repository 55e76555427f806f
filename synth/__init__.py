"""Seeded synthetic workloads for randomised primal-dual radio-interferometric imaging.

This module produces *inputs only*: sky images, u-v coverage, the partition of the
visibilities into data blocks, complex noise, the l2-ball radii and the uniform
variates that decide which blocks are active at each iteration.  It applies neither
the measurement operator nor the sparsity operator and implements no step of the
solver; a caller that wants noisy data passes in the noiseless visibilities it
computed with its own measurement operator.

Both the FP64 oracle and the GPU path take their inputs from here, so the two sides
see bit-identical data.  The recipe follows the simulation set-up of Sec. V of
Onose, Carrillo, McEwen & Wiaux (2016): Gaussian u-v sampling with a standard
deviation of a quarter of the maximum frequency, complex Gaussian noise at a given
input SNR, l2-ball radii from the 0.99 quantile of a chi-square law with 2 M_i
degrees of freedom.  The paper's M31 test image is not available; skies are
synthetic Gaussian blobs plus point sources.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 1610088950
SEED_SKY, SEED_UV, SEED_BLOCKS, SEED_NOISE, SEED_MASKS, SEED_POWER = range(6)

# Largest float32 strictly below pi: u-v coordinates are kept in [-pi, pi) rad/px.
_PI32_BELOW = np.nextafter(np.float32(np.pi), np.float32(0.0))


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic imaging problem (sizes, coverage model, block cut, noise, schedule)."""

    name: str
    n: int                   # image is n x n pixels
    n_blobs: int
    n_points: int
    M: int                   # number of visibilities
    d: int                   # number of data blocks requested
    block_scheme: str        # "equal", "annuli" or "lognormal"
    isnr_db: float           # input SNR of the noisy data
    outlier_frac: float      # fraction of u-v points drawn uniformly instead of Gaussian
    iterations: int
    # block-activity schedules used with this workload: (label, kind, params)
    prob_schemes: tuple = ()

    def seed(self, which: int) -> int:
        return BASE_SEED + which


WORKLOADS = {
    w.name: w
    for w in (
        Workload("n64_m8k_d4", 64, 5, 10, 8192, 4, "equal", 30.0, 0.0, 200,
                 (("p1", "uniform", {"p": 1.0}),)),
        Workload("n256_m128k_d16", 256, 5, 10, 131072, 16, "annuli", 20.0, 0.0, 500,
                 (("uniform0.5", "uniform", {"p": 0.5}),
                  ("adaptive8", "adaptive", {"n_nodes": 8.0, "p_min": 0.05, "p_max": 1.0}))),
        Workload("n1024_m4m_d64", 1024, 200, 1000, 1 << 22, 64, "lognormal", 20.0, 0.0, 200,
                 (("p1", "uniform", {"p": 1.0}),
                  ("adaptive16", "adaptive", {"n_nodes": 16.0, "p_min": 0.05, "p_max": 0.5}))),
        # Sec. V's adaptive-probability experiment: 256^2, M = 5N, 16 equal blocks, 20 dB
        Workload("n256_m320k_d16", 256, 5, 10, 5 * 256 * 256, 16, "equal", 20.0, 0.0, 600,
                 (("p1", "uniform", {"p": 1.0}),
                  ("adaptive4", "adaptive", {"n_nodes": 4.0, "p_min": 0.05, "p_max": 0.5}))),
        Workload("n512_m1m_d32", 512, 5, 10, 1 << 20, 32, "equal", 20.0, 0.0, 20,
                 (("p1", "uniform", {"p": 1.0}),)),
        Workload("n2048_m16m_d128", 2048, 200, 1000, 1 << 24, 128, "lognormal", 20.0, 0.1, 1000,
                 (("adaptive32", "adaptive", {"n_nodes": 32.0, "p_min": 0.05, "p_max": 0.5}),)),
    )
}


def sky(n: int, n_blobs: int, n_points: int, rng: np.random.Generator) -> np.ndarray:
    """Nonnegative n x n sky: Gaussian blobs plus single-pixel sources, peak 1 (FP64).

    Blob centres are uniform in [0.1 n, 0.9 n)^2 with widths sigma ~ U[1, 4] px; point
    sources sit on pixels uniform in [0.05 n, 0.95 n)^2; all amplitudes ~ LogNormal(0, 1).
    """
    img = np.zeros((n, n))
    for _ in range(n_blobs):
        cy, cx = rng.uniform(0.1 * n, 0.9 * n, size=2)
        s = rng.uniform(1.0, 4.0)
        a = rng.lognormal(0.0, 1.0)
        r = int(math.ceil(6 * s))
        y0, y1 = max(0, int(cy) - r), min(n, int(cy) + r + 1)
        x0, x1 = max(0, int(cx) - r), min(n, int(cx) + r + 1)
        yy = np.arange(y0, y1)[:, None] - cy
        xx = np.arange(x0, x1)[None, :] - cx
        img[y0:y1, x0:x1] += a * np.exp(-(yy * yy + xx * xx) / (2 * s * s))
    lo, hi = int(0.05 * n), max(int(0.05 * n) + 1, int(0.95 * n))
    py = rng.integers(lo, hi, size=n_points)
    px = rng.integers(lo, hi, size=n_points)
    amp = rng.lognormal(0.0, 1.0, size=n_points)
    np.add.at(img, (py, px), amp)
    np.clip(img, 0.0, None, out=img)
    peak = img.max()
    return img / peak if peak > 0 else img


def uv_coverage(M: int, rng: np.random.Generator, sigma: float = math.pi / 4,
                outlier_frac: float = 0.0) -> np.ndarray:
    """M u-v points (float32, rad/px) in [-pi, pi)^2.

    A fraction ``1 - outlier_frac`` is iid N(0, sigma^2) per coordinate, redrawn when
    outside the band; the rest is uniform over the band.  Rows are (u, v): u pairs
    with the image's column (x) axis and v with its row (y) axis.
    """
    n_out = int(round(outlier_frac * M))
    n_gauss = M - n_out
    pts = np.empty((0, 2), dtype=np.float32)
    while pts.shape[0] < n_gauss:
        need = n_gauss - pts.shape[0]
        cand = (rng.standard_normal((need + need // 8 + 16, 2)) * sigma).astype(np.float32)
        keep = np.all(np.abs(cand) <= _PI32_BELOW, axis=1)
        pts = np.concatenate([pts, cand[keep][:need]])
    if n_out:
        out = rng.uniform(-math.pi, math.pi, size=(n_out, 2)).astype(np.float32)
        out = np.clip(out, -_PI32_BELOW, _PI32_BELOW)
        pts = np.concatenate([pts, out])
        pts = pts[rng.permutation(M)]
    return np.ascontiguousarray(pts, dtype=np.float32)


def partition(uv: np.ndarray, d: int, scheme: str, rng: np.random.Generator | None = None,
              floor: int = 256):
    """Sort visibilities by u-v radius and cut them into d contiguous radial blocks.

    Blocks cover compact u-v regions (Sec. III: each block spans a compact frequency
    range).  Returns (uv_sorted, block_off, order) with block i holding rows
    block_off[i]:block_off[i+1] of uv_sorted = uv[order].

    Schemes: "equal" (equal counts), "annuli" (equal-width radial annuli on
    [0, r_max]; empty annuli are dropped, so fewer than d blocks may result) and
    "lognormal" (sizes proportional to LogNormal(0, 1) draws on top of a floor,
    largest-remainder rounding).
    """
    M = uv.shape[0]
    r = np.hypot(uv[:, 0].astype(np.float64), uv[:, 1].astype(np.float64))
    order = np.argsort(r, kind="stable")
    rs = r[order]
    if scheme == "equal":
        sizes = np.full(d, M // d, dtype=np.int64)
        sizes[: M % d] += 1
    elif scheme == "annuli":
        edges = np.linspace(0.0, rs[-1], d + 1)
        edges[-1] = np.inf
        cuts = np.searchsorted(rs, edges[1:-1], side="left")
        bounds = np.concatenate([[0], cuts, [M]])
        sizes = np.diff(bounds)
        sizes = sizes[sizes > 0]
    elif scheme == "lognormal":
        if rng is None:
            raise ValueError("lognormal partition needs an rng")
        if d * floor > M:
            raise ValueError("floor too large for M")
        w = rng.lognormal(0.0, 1.0, size=d)
        share = (M - d * floor) * w / w.sum()
        base = np.floor(share).astype(np.int64)
        rem = (M - d * floor) - base.sum()
        frac_order = np.argsort(-(share - base), kind="stable")
        base[frac_order[:rem]] += 1
        sizes = base + floor
    else:
        raise ValueError(f"unknown block scheme {scheme!r}")
    block_off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    assert block_off[-1] == M and np.all(sizes > 0)
    return np.ascontiguousarray(uv[order]), block_off, order


def noise_sigma(y0: np.ndarray, isnr_db: float) -> float:
    """Noise standard deviation sigma_n giving input SNR ``isnr_db``:
    sigma_n^2 = (||y0||^2 / M) 10^(-isnr/10)."""
    y0 = np.asarray(y0)
    return float(math.sqrt(np.vdot(y0, y0).real / y0.size * 10.0 ** (-isnr_db / 10.0)))


def complex_noise(M: int, sigma_n: float, rng: np.random.Generator) -> np.ndarray:
    """Circular complex Gaussian noise, E|n_m|^2 = sigma_n^2 (complex128)."""
    g = rng.standard_normal((M, 2))
    return (sigma_n / math.sqrt(2.0)) * (g[:, 0] + 1j * g[:, 1])


def l2_ball_radii(block_off: np.ndarray, sigma_n: float, quantile: float = 0.99) -> np.ndarray:
    """epsilon_i from the chi-square law with 2 M_i degrees of freedom (Sec. V).

    ||n_i||^2 / (sigma_n^2 / 2) follows chi^2_{2 M_i}, so the radius holding the noise
    with probability ``quantile`` is (sigma_n / sqrt 2) sqrt(F^{-1}_{chi^2_{2M_i}}(quantile)).
    """
    from scipy.stats import chi2

    sizes = np.diff(np.asarray(block_off, dtype=np.int64))
    return (sigma_n / math.sqrt(2.0)) * np.sqrt(chi2.ppf(quantile, 2 * sizes))


def activity_uniforms(T: int, d: int, seed: int) -> np.ndarray:
    """U[0, 1) variates u[t, i]; block i is active at iteration t+1 iff u[t, i] < p_i."""
    return np.random.default_rng(seed).random((T, d))


def power_start(n: int, seed: int) -> np.ndarray:
    """Seeded Gaussian start vector (n x n, FP64) for power iterations."""
    return np.random.default_rng(seed).standard_normal((n, n))


@dataclasses.dataclass
class Inputs:
    workload: Workload
    x_true: np.ndarray        # (n, n) float64
    uv: np.ndarray            # (M, 2) float32, sorted into radial blocks
    block_off: np.ndarray     # (d+1,) int64


def make_inputs(w: Workload) -> Inputs:
    """Sky, u-v coverage and block partition of a workload (no data yet)."""
    x = sky(w.n, w.n_blobs, w.n_points, np.random.default_rng(w.seed(SEED_SKY)))
    uv = uv_coverage(w.M, np.random.default_rng(w.seed(SEED_UV)), outlier_frac=w.outlier_frac)
    uv_s, off, _ = partition(uv, w.d, w.block_scheme, np.random.default_rng(w.seed(SEED_BLOCKS)))
    return Inputs(w, x, uv_s, off)


def add_noise(w: Workload, y0: np.ndarray, block_off: np.ndarray):
    """Noisy data y = y0 + n at the workload's input SNR, with sigma_n and the radii."""
    s = noise_sigma(y0, w.isnr_db)
    y = np.asarray(y0, dtype=np.complex128) + complex_noise(y0.size, s, np.random.default_rng(w.seed(SEED_NOISE)))
    return y, s, l2_ball_radii(block_off, s)


def dde_taps(M: int, jd: int, rng: np.random.Generator, strength: float = 0.2) -> np.ndarray:
    """Per-visibility direction-dependent-effect kernels, (M, jd, jd) complex128.

    Entry [m, h + q, h + p] (h = jd // 2, -h <= p, q <= h) is the coefficient d_m[q, p] of a
    smooth, band-limited DDE D_m(l) = sum d_m[q, p] exp(-2 pi i (p l_x + q l_y) / K) on the
    oversampled grid of K cells per axis: a unit central term plus complex Gaussian terms of
    standard deviation `strength` exp(-(p^2 + q^2) / 2), independent per visibility.
    Synthetic stand-in for calibrated DDE kernels (antenna beams, ionosphere)."""
    if jd < 1 or jd % 2 == 0:
        raise ValueError("jd must be odd and positive")
    h = jd // 2
    q, p = np.meshgrid(np.arange(-h, h + 1), np.arange(-h, h + 1), indexing="ij")
    env = strength * np.exp(-(p ** 2 + q ** 2) / 2.0)
    d = (rng.standard_normal((M, jd, jd)) + 1j * rng.standard_normal((M, jd, jd))) * (env / np.sqrt(2.0))
    d[:, h, h] += 1.0
    return d
