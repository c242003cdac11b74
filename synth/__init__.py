"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module holds no arithmetic of the shearlet method itself: it only draws
images, noise and masks. Both the FP64 oracle and the GPU path consume what it
returns, so neither side depends on the other.

The paper measures on photographs (a flower image in Section 4.1, 512x512
images in Sections 4.2-4.3) that are not available; its own learned
reconstruction experiment trains on randomly generated ellipses (Section 4.4).
The stand-in is therefore a piecewise-constant "cartoon" of random ellipses,
the image class shearlets are designed for.

Recipe (``numpy.random.default_rng(seed)``, PCG64, FP64):
  * number of ellipses n ~ integers(5, 11)
  * per ellipse: centre ~ U[0,N) x U[0,M); semi-axes ~ U[0.05, 0.35]*min(N, M);
    angle ~ U[0, pi); intensity ~ U[0, 255]
  * painted in order on a background of 0, later ellipses overwrite earlier ones;
    a pixel centre (i, j) is inside when its rotated normalised radius is <= 1.
Noise is N(0, sigma^2) from a separate generator. Everything is rounded to
float32 once; FP64 consumers use float64(float32(.)).
"""
from __future__ import annotations

import numpy as np

__all__ = ["cartoon", "cartoon_batch", "gaussian_noise", "random_mask", "seed_image", "seed_noise"]


def seed_image(config: int, i: int) -> int:
    """Seed of image ``i`` of workload ``config``."""
    return 1000 * config + i


def seed_noise(config: int, i: int) -> int:
    """Seed of the noise field added to image ``i`` of workload ``config``."""
    return 1000 * config + 500 + i


def cartoon(rows: int, cols: int, seed: int) -> np.ndarray:
    """One cartoon image of random ellipses, float32, values in [0, 255]."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 11))
    img = np.zeros((rows, cols), dtype=np.float64)
    ii, jj = np.meshgrid(np.arange(rows, dtype=np.float64), np.arange(cols, dtype=np.float64), indexing="ij")
    m = min(rows, cols)
    for _ in range(n):
        ci = rng.uniform(0, rows)
        cj = rng.uniform(0, cols)
        a = rng.uniform(0.05, 0.35) * m
        b = rng.uniform(0.05, 0.35) * m
        th = rng.uniform(0, np.pi)
        val = rng.uniform(0, 255)
        di, dj = ii - ci, jj - cj
        u = (di * np.cos(th) + dj * np.sin(th)) / a
        v = (-di * np.sin(th) + dj * np.cos(th)) / b
        img[u * u + v * v <= 1.0] = val
    return img.astype(np.float32)


def gaussian_noise(rows: int, cols: int, sigma: float, seed: int) -> np.ndarray:
    """White Gaussian noise N(0, sigma^2), float32."""
    rng = np.random.default_rng(seed)
    return (sigma * rng.standard_normal((rows, cols))).astype(np.float32)


def cartoon_batch(batch: int, rows: int, cols: int, config: int, sigma: float = 0.0) -> np.ndarray:
    """``batch`` cartoons of workload ``config`` (seeds 1000*config+i), plus
    N(0, sigma^2) noise (seeds 1000*config+500+i) when sigma > 0. float32, (B, rows, cols)."""
    out = np.empty((batch, rows, cols), dtype=np.float32)
    for i in range(batch):
        img = cartoon(rows, cols, seed_image(config, i))
        if sigma > 0:
            img = (img.astype(np.float64) + gaussian_noise(rows, cols, sigma, seed_noise(config, i))).astype(np.float32)
        out[i] = img
    return out


def random_mask(rows: int, cols: int, keep: float, seed: int) -> np.ndarray:
    """Binary mask with a fraction ``keep`` of ones at random pixels, float32."""
    rng = np.random.default_rng(seed)
    return (rng.random((rows, cols)) < keep).astype(np.float32)
