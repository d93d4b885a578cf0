"""Seeded synthetic workloads shaped like the paper's ensembles.

The paper's real datasets (E3SM sea-level pressure 240x960, Red Sea 20
members of 500x500; Sec. 5.3) are not available; these generators stand in
for them with smooth random fields plus member noise of the same kind of
structure.  Everything is a pure function of the seed.

Fields are "bumps": a sum of K Gaussian bumps with amplitudes U[-1, 1],
centres uniform over the grid and widths U[3, 10] cells (scaled by
size / 64 for the large grids), min-max rescaled to [0, 1].
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

__all__ = [
    "bumps", "uniform_params_field", "smooth_ensemble", "mixture_ensemble",
    "correlated_ensemble", "upstream", "random_params", "batched_layout",
    "MODEL_UNIFORM", "MODEL_EPANECHNIKOV", "MODEL_HISTOGRAM",
]

MODEL_UNIFORM, MODEL_EPANECHNIKOV, MODEL_HISTOGRAM = 0, 1, 2


def bumps(rng: np.random.Generator, H: int, W: int, K: int, sigma_lo: float, sigma_hi: float) -> np.ndarray:
    """Sum of K separable Gaussian bumps, rescaled to [0, 1] (float64)."""
    field = np.zeros((H, W))
    iy = np.arange(H, dtype=np.float64)
    ix = np.arange(W, dtype=np.float64)
    amp = rng.uniform(-1.0, 1.0, K)
    cy = rng.uniform(0, H, K)
    cx = rng.uniform(0, W, K)
    sig = rng.uniform(sigma_lo, sigma_hi, K)
    for k in range(K):
        gy = np.exp(-((iy - cy[k]) ** 2) / (2 * sig[k] ** 2))
        gx = np.exp(-((ix - cx[k]) ** 2) / (2 * sig[k] ** 2))
        field += amp[k] * np.outer(gy, gx)
    lo, hi = field.min(), field.max()
    if hi > lo:
        field = (field - lo) / (hi - lo)
    return field


def _scale(H: int, W: int) -> float:
    return max(1.0, min(H, W) / 64.0)


def uniform_params_field(seed: int, H: int = 64, W: int = 64) -> np.ndarray:
    """Independent uniform noise per vertex, FP64: mean = 8 bumps (sigma
    U[3,10] cells) on [0, 1], half-width U[0.05, 0.2]; returns (lo, hi)."""
    rng = np.random.default_rng(seed)
    mean = bumps(rng, H, W, 8, 3.0, 10.0)
    hw = rng.uniform(0.05, 0.2, (H, W))
    return np.stack([mean - hw, mean + hw])


def smooth_ensemble(seed: int, H: int, W: int, M: int = 20) -> np.ndarray:
    """[M][H][W] float32: base (64 bumps) + N(0, 0.05^2) noise smoothed by a
    5x5 box filter with reflected edges."""
    rng = np.random.default_rng(seed)
    s = _scale(H, W)
    base = bumps(rng, H, W, 64, 3.0 * s, 10.0 * s).astype(np.float32)
    out = np.empty((M, H, W), dtype=np.float32)
    for k in range(M):
        noise = rng.standard_normal((H, W), dtype=np.float32) * np.float32(0.05)
        out[k] = base + ndimage.uniform_filter(noise, size=5, mode="reflect")
    return out


def mixture_ensemble(seed: int, H: int, W: int, M: int = 20) -> np.ndarray:
    """[M][H][W] float32: base + delta_c + N(0, 0.05^2), c ~ Bernoulli(0.3),
    delta_0 = 0, delta_1 = 0.3, independent per member and vertex (a
    two-component mixture with weights 0.7 / 0.3)."""
    rng = np.random.default_rng(seed)
    s = _scale(H, W)
    base = bumps(rng, H, W, 64, 3.0 * s, 10.0 * s).astype(np.float32)
    out = np.empty((M, H, W), dtype=np.float32)
    for k in range(M):
        comp = (rng.random((H, W), dtype=np.float32) < 0.3).astype(np.float32)
        noise = rng.standard_normal((H, W), dtype=np.float32) * np.float32(0.05)
        out[k] = base + np.float32(0.3) * comp + noise
    return out


def correlated_ensemble(seed: int, H: int, W: int, M: int = 20, corr_len: float = 4.0) -> np.ndarray:
    """[M][H][W] float32: base + Gaussian-smoothed white noise (sigma =
    corr_len cells), rescaled to a standard deviation of 0.05."""
    rng = np.random.default_rng(seed)
    s = _scale(H, W)
    base = bumps(rng, H, W, 64, 3.0 * s, 10.0 * s)
    noise = np.empty((M, H, W))
    for k in range(M):
        noise[k] = ndimage.gaussian_filter(rng.standard_normal((H, W)), sigma=corr_len, mode="reflect")
    noise *= 0.05 / noise.std()
    return (base[None] + noise).astype(np.float32)


def upstream(seed: int, H: int, W: int, dtype=np.float32) -> tuple[np.ndarray, np.ndarray]:
    """Upstream gradients g_min, g_max ~ N(0, 1)."""
    rng = np.random.default_rng(seed + 7919)
    return (rng.standard_normal((H, W)).astype(dtype), rng.standard_normal((H, W)).astype(dtype))


def random_params(model: int, seed: int, H: int, W: int, nbins: int = 10, dtype=np.float64,
                  width: float = 0.02) -> np.ndarray:
    """A parameter field directly (no fit): smooth centre (8 bumps) with
    per-vertex widths.  uniform (lo, hi), Epanechnikov (m, w), histogram
    (lo, hi, Dirichlet masses)."""
    rng = np.random.default_rng(seed)
    base = bumps(rng, H, W, 8, 2.0, 6.0)
    wd = rng.uniform(0.25 * width, width, (H, W))
    if model == MODEL_UNIFORM:
        p = np.stack([base - wd, base + wd])
    elif model == MODEL_EPANECHNIKOV:
        p = np.stack([base, wd])
    else:
        masses = rng.dirichlet(np.ones(nbins), size=(H, W)).transpose(2, 0, 1)
        p = np.concatenate([np.stack([base - wd, base + wd]), masses])
    return p.astype(dtype)


def batched_layout(seed: int, n_fields: int = 64, log2_lo: float = 7.0, log2_hi: float = 11.0):
    """Field sides drawn log-uniformly between 2^log2_lo and 2^log2_hi, square
    grids; models cycle uniform / Epanechnikov / histogram.  Returns a list of
    (side, model, member_seed)."""
    rng = np.random.default_rng(seed)
    sides = np.round(2.0 ** rng.uniform(log2_lo, log2_hi, n_fields)).astype(int)
    return [(int(sides[i]), i % 3, int(seed * 1000 + i)) for i in range(n_fields)]

