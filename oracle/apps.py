"""Oracle: applications of the transform, FP64 (test infrastructure only).

  * hard thresholding and per-filter thresholds (Section 4.2),
  * denoising  f_denoised = SH^-1 T_delta SH f_noisy  (Section 4.2),
  * PSNR (Section 4.2),
  * inpainting by iterative hard thresholding (Section 4.3, Algorithm 3).

SH is ``transform.forward_plain`` and SH^-1 ``transform.inverse_plain``: the
coefficients are real planes c[k], and every plane k has its own threshold.

Readings (paper silent or garbled):
  * Threshold comparison: a coefficient is kept when |c| >= delta (the
    operator's definition in Section 4.2); the listing zeroes |c|/delta < 1,
    the same set.
  * Per-filter thresholds: delta_k = K_j * sigma * RMS_k for a filter k of
    scale j. The text gives delta_j = K_j sigma; its listing multiplies by the
    RMS of each filter. K = [2.5, 2.5, 2.5, 3.8] for four scales (coarse to
    fine); for J scales the finest gets 3.8 and the others 2.5. The listing
    thresholds every plane (its weights loop over all RMS entries), the
    low-pass included; the low-pass belongs to no scale j of the text, so it
    takes the factor of the coarsest scale, K_1. Algorithm 3 thresholds every
    plane in the same way.
  * The denoising listing thresholds one array and reconstructs another
    (a garble); the thresholded coefficients are reconstructed.
  * Algorithm 3's decay: as printed lambda = delta_min^(1/(iterations-1)),
    which reaches delta_min only if delta_init = 1; taken as
    lambda = (delta_min / delta_init)^(1/(iterations-1)), so delta goes
    geometrically from delta_init (first iteration) to delta_min (last).
  * Algorithm 3's threshold is weighted per filter like the denoising
    listing: delta_k = delta * RMS_k for every filter, low-pass included.
"""
from __future__ import annotations

import numpy as np

from . import transform as T

__all__ = [
    "scale_factors",
    "thresholds",
    "hard_threshold",
    "kept_counts",
    "denoise",
    "psnr",
    "delta_schedule",
    "delta_schedule_linear",
    "inpaint",
]


def scale_factors(n_scales: int) -> np.ndarray:
    """K_j for j = 1..J (coarse to fine): 2.5 for every scale but the finest, 3.8 there (Section 4.2)."""
    if n_scales < 1:
        raise ValueError("n_scales must be positive")
    f = np.full(n_scales, 2.5)
    f[-1] = 3.8
    return f


def thresholds(idx: np.ndarray, rms: np.ndarray, sigma: float, factors=None) -> np.ndarray:
    """delta_k = K_j sigma RMS_k for filter k of scale j = idx[k, 1] (Section 4.2 and its listing);
    the low-pass (scale 0) takes K_1, the factor of the coarsest scale."""
    idx = np.asarray(idx)
    scale = idx[:, 1]
    J = int(scale.max())
    f = scale_factors(J) if factors is None else np.asarray(factors, dtype=np.float64)
    if f.shape != (J,):
        raise ValueError(f"need {J} factors, got {f.shape}")
    out = np.zeros(len(scale), dtype=np.float64)
    for k, j in enumerate(scale):
        out[k] = f[max(int(j), 1) - 1] * sigma * float(rms[k])
    return out


def hard_threshold(c: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """(T_delta c)[k](n) = c[k](n) if |c[k](n)| >= delta[k], else 0 (Section 4.2); c is (K, N, M)."""
    d = np.asarray(delta, dtype=np.float64).reshape(-1, 1, 1)
    return np.where(np.abs(c) >= d, c, 0.0)


def kept_counts(c: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """Number of coefficients of each plane that T_delta keeps."""
    d = np.asarray(delta, dtype=np.float64).reshape(-1, 1, 1)
    return (np.abs(c) >= d).sum(axis=(1, 2)).astype(np.int64)


def denoise(x_noisy: np.ndarray, spectra: np.ndarray, W: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """f_denoised = SH^-1 T_delta SH f_noisy (Section 4.2)."""
    c = T.forward_plain(x_noisy, spectra)
    return T.inverse_plain(hard_threshold(c, delta), spectra, W)


def psnr(f: np.ndarray, g: np.ndarray) -> float:
    """PSNR = 20 log10(255 sqrt(N) / ||f - g||_F), N the number of pixels (Section 4.2)."""
    f = np.asarray(f, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    return float(20.0 * np.log10(255.0 * np.sqrt(f.size) / np.linalg.norm(f - g)))


def delta_schedule(delta_init: float, delta_min: float, iterations: int) -> np.ndarray:
    """The thresholds of Algorithm 3's iterations: delta_init * lambda^i, i < iterations."""
    if iterations < 1:
        raise ValueError("iterations must be positive")
    lam = (delta_min / delta_init) ** (1.0 / (iterations - 1)) if iterations > 1 else 1.0
    out = np.empty(iterations)
    delta = float(delta_init)
    for i in range(iterations):
        out[i] = delta
        delta *= lam
    return out


def delta_schedule_linear(delta_init: float, iterations: int) -> np.ndarray:
    """A linear decay to zero over the iterations: delta_init (1 - i / (iterations - 1)), i < iterations."""
    if iterations < 1:
        raise ValueError("iterations must be positive")
    if iterations == 1:
        return np.array([float(delta_init)])
    return np.array([delta_init * (1.0 - i / (iterations - 1)) for i in range(iterations)])


def inpaint(f_masked: np.ndarray, mask: np.ndarray, spectra: np.ndarray, W: np.ndarray, rms: np.ndarray,
            deltas) -> np.ndarray:
    """Shearlet inpainting by iterative hard thresholding (Section 4.3, Algorithm 3).

    f_inpainted = 0; for each delta of the schedule (``delta_schedule``: the paper's geometric decay)
      f_res = M (f_masked - f_inpainted)
      f_inpainted = SH^-1 T_{delta RMS} SH (f_res + f_inpainted).
    ``deltas`` is (iterations,) scalars, or (iterations, K) per-filter thresholds used as given.
    """
    M = np.asarray(mask, dtype=np.float64)
    fm = np.asarray(f_masked, dtype=np.float64)
    f = np.zeros_like(fm)
    r = np.asarray(rms, dtype=np.float64)
    for delta in np.asarray(deltas, dtype=np.float64):
        f_res = M * (fm - f)
        # a scalar delta is weighted by the filters' RMS; a row of K values is used as the thresholds
        f = denoise(f_res + f, spectra, W, delta * r if np.ndim(delta) == 0 else delta)
    return f
