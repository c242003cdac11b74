"""Pins of the oracle's applications (Section 4.2 denoising, Section 4.3
inpainting): hand-worked thresholding cases, the printed threshold factors,
closed forms of PSNR, and invariants of denoising and inpainting."""
import os

import numpy as np
import pytest

import synth
from oracle import apps as A
from oracle import filters as OF
from oracle import transform as OT

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def sys128():
    return OF.build_system(128, 128, 2)


def test_hard_threshold_hand_case():
    # |c| >= delta is kept (ties included), per plane
    c = np.array([[[-3.0, -2.0, 2.0], [1.999, 0.0, 5.0]],
                  [[0.5, -0.6, 0.7], [-0.7, 0.69, 10.0]]])
    delta = np.array([2.0, 0.7])
    want = np.array([[[-3.0, -2.0, 2.0], [0.0, 0.0, 5.0]],
                     [[0.0, 0.0, 0.7], [-0.7, 0.0, 10.0]]])
    assert np.array_equal(A.hard_threshold(c, delta), want)
    assert list(A.kept_counts(c, delta)) == [4, 3]
    # zero threshold keeps everything, infinite drops everything
    assert np.array_equal(A.hard_threshold(c, [0.0, 0.0]), c)
    assert not A.hard_threshold(c, [np.inf, np.inf]).any()


def test_scale_factors_printed():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "denoise_factors.txt")) if not l.startswith("#")]
    for r in rows:
        J = int(r[0])
        assert np.array_equal(A.scale_factors(J), np.array([float(v) for v in r[1:]]))
    assert list(A.scale_factors(2)) == [2.5, 3.8]


def test_thresholds_per_filter(sys128):
    s = sys128
    sigma = 30.0
    t = A.thresholds(s.idx, s.rms, sigma)
    assert t.shape == (s.K,)
    for k, (cone, j, shear) in enumerate(s.idx):
        if j == 0:
            # the low-pass: thresholded like every plane of the listing, with the coarsest scale's factor
            assert (cone, shear) == (0, 0) and t[k] == pytest.approx(2.5 * sigma * s.rms[k], rel=1e-15)
        else:
            assert t[k] == pytest.approx({1: 2.5, 2: 3.8}[int(j)] * sigma * s.rms[k], rel=1e-15)
    assert np.all(t > 0) and s.idx[-1, 1] == 0
    with pytest.raises(ValueError):
        A.thresholds(s.idx, s.rms, sigma, factors=[1.0])


def test_psnr_closed_forms():
    rng = np.random.default_rng(0)
    f = rng.uniform(0, 255, (32, 48))
    # a constant offset d gives ||f-g|| = |d| sqrt(N): PSNR = 20 log10(255/|d|)
    assert A.psnr(f, f + 2.55) == pytest.approx(40.0, abs=1e-12)
    assert A.psnr(f, f - 25.5) == pytest.approx(20.0, abs=1e-12)
    # a single pixel off by e: PSNR = 20 log10(255 sqrt(N) / e)
    g = f.copy()
    g[3, 7] += 5.0
    assert A.psnr(f, g) == pytest.approx(20 * np.log10(255 * np.sqrt(f.size) / 5.0), abs=1e-12)


def test_denoise_zero_threshold_is_perfect_reconstruction(sys128):
    s = sys128
    x = synth.cartoon(128, 128, seed=11) + synth.gaussian_noise(128, 128, 30.0, seed=12)
    y = A.denoise(x, s.spectra, s.W, np.zeros(s.K))
    assert np.linalg.norm(y - x) <= 1e-12 * np.linalg.norm(x)


def test_denoise_constant_image_is_fixed_point(sys128):
    # band-passes vanish on a constant image, so any band thresholds leave it unchanged
    s = sys128
    x = np.full((128, 128), 77.0)
    t = A.thresholds(s.idx, s.rms, 1e3)
    t[-1] = 0.0  # keep the low-pass plane, which carries the constant
    y = A.denoise(x, s.spectra, s.W, t)
    assert np.max(np.abs(y - x)) <= 1e-10
    # with the low-pass thresholded above the constant every plane is zeroed
    assert np.max(np.abs(A.denoise(x, s.spectra, s.W, A.thresholds(s.idx, s.rms, 1e3)))) <= 1e-10


def test_denoise_improves_psnr(sys128):
    s = sys128
    clean = synth.cartoon(128, 128, seed=21)
    noisy = clean + synth.gaussian_noise(128, 128, 30.0, seed=22)
    y = A.denoise(noisy, s.spectra, s.W, A.thresholds(s.idx, s.rms, 30.0))
    p0, p1 = A.psnr(clean, noisy), A.psnr(clean, y)
    assert p0 == pytest.approx(20 * np.log10(255 / 30.0), abs=0.3)
    assert p1 > p0 + 3.0


def test_kept_counts_monotone(sys128):
    s = sys128
    x = synth.cartoon(128, 128, seed=31) + synth.gaussian_noise(128, 128, 20.0, seed=32)
    c = OT.forward_plain(x, s.spectra)
    base = A.thresholds(s.idx, s.rms, 20.0)
    prev = None
    for f in (0.5, 1.0, 2.0, 4.0):
        n = A.kept_counts(c, f * base)
        if prev is not None:
            assert np.all(n <= prev)
        prev = n
    # the counts are the plain number of |c| >= delta per plane
    d = 4.0 * base
    assert np.array_equal(prev, [int(np.sum(np.abs(c[k]) >= d[k])) for k in range(s.K)])


def test_delta_schedule():
    d = A.delta_schedule(8.0, 0.5, 5)
    assert d[0] == 8.0 and d[-1] == pytest.approx(0.5, rel=1e-14)
    assert np.allclose(d[1:] / d[:-1], (0.5 / 8.0) ** 0.25, rtol=1e-14)
    assert list(A.delta_schedule(3.0, 1.0, 1)) == [3.0]
    with pytest.raises(ValueError):
        A.delta_schedule(1.0, 0.1, 0)


def test_delta_schedule_linear():
    d = A.delta_schedule_linear(9.0, 4)
    assert np.allclose(d, [9.0, 6.0, 3.0, 0.0], rtol=0, atol=1e-15)
    assert list(A.delta_schedule_linear(2.0, 1)) == [2.0]


def test_inpaint_one_step_is_denoising(sys128):
    # with f_inpainted = 0 the first iteration thresholds the masked image itself
    s = sys128
    f = synth.cartoon(128, 128, seed=61)
    mask = synth.random_mask(128, 128, 0.5, seed=62)
    fm = (f * mask).astype(np.float64)
    y = A.inpaint(fm, mask, s.spectra, s.W, s.rms, [40.0])
    want = A.denoise(fm, s.spectra, s.W, 40.0 * s.rms)
    assert np.array_equal(y, want)


def test_inpaint_per_filter_rows_equal_scalar_schedule(sys128):
    s = sys128
    f = synth.cartoon(128, 128, seed=71)
    mask = synth.random_mask(128, 128, 0.5, seed=72)
    d = A.delta_schedule(300.0, 2.0, 4)
    y1 = A.inpaint(f * mask, mask, s.spectra, s.W, s.rms, d)
    y2 = A.inpaint(f * mask, mask, s.spectra, s.W, s.rms, d[:, None] * s.rms[None, :])
    assert np.array_equal(y1, y2)


def test_inpaint_full_mask_returns_image(sys128):
    s = sys128
    f = synth.cartoon(128, 128, seed=41)
    y = A.inpaint(f, np.ones_like(f), s.spectra, s.W, s.rms, A.delta_schedule(1e-9, 1e-12, 3))
    assert np.linalg.norm(y - f) <= 1e-10 * np.linalg.norm(f)


def test_inpaint_recovers_missing_pixels(sys128):
    s = sys128
    f = synth.cartoon(128, 128, seed=51)
    mask = synth.random_mask(128, 128, 0.5, seed=52)
    fm = f * mask
    # delta_init near the largest RMS-normalised coefficient, so that the first
    # iterations remove the mask's pixel-scale pattern
    d0 = float(np.max(np.abs(OT.forward_plain(fm.astype(np.float64), s.spectra)) / s.rms[:, None, None]))
    assert 200.0 < d0 < 1000.0
    y = A.inpaint(fm, mask, s.spectra, s.W, s.rms, A.delta_schedule(d0, 1.0, 25))
    # the known pixels are matched closely and the masked ones far better than by zeros
    assert A.psnr(f, y) > A.psnr(f, fm) + 15.0
    assert A.psnr(f * mask, y * mask) > 40.0
    # a linear decay to zero ends with an unthresholded step: the known pixels are reproduced
    y2 = A.inpaint(fm, mask, s.spectra, s.W, s.rms, A.delta_schedule_linear(d0, 25))
    assert A.psnr(f, y2) > A.psnr(f, fm) + 15.0
    assert np.max(np.abs((y2 - f) * mask)) <= 1e-9 * np.max(np.abs(f))
