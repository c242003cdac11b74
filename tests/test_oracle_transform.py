"""Pins of the oracle's transforms (CPU, FP64).

Each check compares the oracle with something other than itself: numpy's
fftshift/ifftshift, brute-force circular correlation, scipy's wrap-mode
correlation, closed-form special cases, or identities that the mathematics
fixes (perfect reconstruction, the adjoint identity, the frame-energy
identity). A plausible slip (a dropped conjugate, a transposed operand, a
missing 1/W, a wrong shift) fails at least one of them.
"""
import numpy as np
import pytest
import scipy.ndimage

import synth
from oracle import filters as F
from oracle import transform as T


def _random_bank(rng, K, N, M):
    """K Hermitian spectra (DFTs of random real kernels), natural order, plus the kernels."""
    ker = rng.standard_normal((K, N, M))
    return np.fft.fft2(ker), ker


# ---------------------------------------------------------------- Section 3.3 shifts


@pytest.mark.parametrize("n", list(range(1, 12)))
def test_centring_matches_numpy(n):
    """The centred layout of Section 3.3 is numpy's fftshift (ifftshift undoes it), even and odd n."""
    x = np.arange(n * (n + 3)).reshape(n, n + 3).astype(float)
    assert np.array_equal(T.to_centred(x), np.fft.fftshift(x))
    assert np.array_equal(T.from_centred(x), np.fft.ifftshift(x))
    assert np.array_equal(T.from_centred(T.to_centred(x)), x)
    # zero frequency (natural index 0) sits at index floor(n/2) of each centred axis
    d = np.zeros((n, n + 3))
    d[0, 0] = 1.0
    assert T.to_centred(d)[n // 2, (n + 3) // 2] == 1.0


@pytest.mark.parametrize("N,M", [(16, 16), (15, 17), (8, 13)])
def test_literal_algorithm1_equals_shift_free(N, M):
    rng = np.random.default_rng(1)
    S, _ = _random_bank(rng, 3, N, M)
    x = rng.standard_normal((N, M))
    lit = T.decompose(x, np.fft.fftshift(S, axes=(1, 2)))
    assert np.max(np.abs(lit - T.forward_plain(x, S))) < 1e-13 * np.max(np.abs(lit))
    c = rng.standard_normal((3, N, M))
    W = np.sum(np.abs(S) ** 2, 0)
    Wc = np.fft.fftshift(W)
    Sc = np.fft.fftshift(S, axes=(1, 2))
    assert np.allclose(T.reconstruct(c, Sc, Wc), T.inverse_plain(c, S, W), atol=1e-13)
    assert np.allclose(T.adjoint(c, Sc), T.adjoint_plain(c, S), atol=1e-12)


# ---------------------------------------------------------------- forward = circular correlation


@pytest.mark.parametrize("N,M", [(16, 16), (15, 17)])
def test_forward_is_brute_force_correlation(N, M):
    rng = np.random.default_rng(2)
    S, ker = _random_bank(rng, 2, N, M)
    x = rng.standard_normal((N, M))
    c = T.decompose(x, np.fft.fftshift(S, axes=(1, 2)))
    for k in range(2):
        ref = T.correlate_direct(x, ker[k])
        assert np.max(np.abs(c[k] - ref)) < 1e-12 * np.max(np.abs(ref))


def test_forward_matches_scipy_wrap_correlation():
    # a small odd kernel centred at the origin: c[n] = sum_m x[m] k[m - n] = scipy correlate (wrap)
    rng = np.random.default_rng(3)
    N, M = 20, 24
    small = rng.standard_normal((5, 7))
    h = np.zeros((N, M))
    for a in range(-2, 3):
        for b in range(-3, 4):
            h[a % N, b % M] = small[a + 2, b + 3]
    x = rng.standard_normal((N, M))
    c = T.forward_plain(x, np.fft.fft2(h)[None])[0]
    ref = scipy.ndimage.correlate(x, small, mode="wrap")
    assert np.max(np.abs(c - ref)) < 1e-12


def test_algorithm1_as_printed_is_point_reflection():
    rng = np.random.default_rng(4)
    N, M = 16, 16
    S, _ = _random_bank(rng, 2, N, M)
    x = rng.standard_normal((N, M))
    Sc = np.fft.fftshift(S, axes=(1, 2))
    a = T.decompose(x, Sc)
    b = T.decompose_alg1_as_printed(x, Sc)
    refl = a[:, (-np.arange(N)) % N][:, :, (-np.arange(M)) % M]
    assert np.max(np.abs(b - refl)) < 1e-12


# ---------------------------------------------------------------- special cases


def test_impulse_gives_reflected_kernels():
    rng = np.random.default_rng(5)
    N, M = 16, 12
    S, ker = _random_bank(rng, 3, N, M)
    x = np.zeros((N, M))
    x[0, 0] = 1.0
    c = T.forward_plain(x, S)
    refl = ker[:, (-np.arange(N)) % N][:, :, (-np.arange(M)) % M]
    assert np.max(np.abs(c - refl)) < 1e-12


def test_constant_image_bandpass_vanish():
    s = F.build_system(128, 128, 2)
    x = np.full((128, 128), 7.5)
    c = T.decompose(x, s.centred)
    assert np.max(np.abs(c[:-1])) < 1e-11
    assert np.max(np.abs(c[-1] - 7.5)) < 1e-11  # low-pass has unit DC gain


def test_identity_filter_is_identity():
    rng = np.random.default_rng(6)
    x = rng.standard_normal((16, 16))
    one = np.ones((1, 16, 16), complex)
    assert np.max(np.abs(T.decompose(x, one)[0] - x)) < 1e-13
    assert np.max(np.abs(T.reconstruct(x[None], one, np.ones((16, 16))) - x)) < 1e-13


# ---------------------------------------------------------------- frame identities


@pytest.fixture(scope="module")
def cfg1():
    s = F.build_system(128, 128, 2, [1, 1])
    x = synth.cartoon(128, 128, synth.seed_image(1, 0)).astype(np.float64)
    return s, x


def test_perfect_reconstruction_config1(cfg1):
    s, x = cfg1
    c = T.decompose(x, s.centred)
    y = T.reconstruct(c, s.centred, np.fft.fftshift(s.W))
    assert np.linalg.norm(y - x) / np.linalg.norm(x) < 1e-12


def test_perfect_reconstruction_random_bank():
    rng = np.random.default_rng(7)
    S, _ = _random_bank(rng, 5, 16, 16)
    W = np.sum(np.abs(S) ** 2, 0)
    x = rng.standard_normal((16, 16))
    y = T.inverse_plain(T.forward_plain(x, S), S, W)
    assert np.linalg.norm(y - x) / np.linalg.norm(x) < 1e-12


def test_weight_is_unique_pr_weight():
    # Algorithm 2 o Algorithm 1 multiplies fft2(x) by sum|Psi|^2 / W: any other W breaks PR
    rng = np.random.default_rng(8)
    S, _ = _random_bank(rng, 4, 12, 12)
    W = np.sum(np.abs(S) ** 2, 0)
    x = rng.standard_normal((12, 12))
    c = T.forward_plain(x, S)
    assert np.allclose(T.inverse_plain(c, S, W), x, atol=1e-12)
    assert not np.allclose(T.inverse_plain(c, S, W * 1.01), x, atol=1e-6)


def test_adjoint_identity_config1(cfg1):
    s, x = cfg1
    rng = np.random.default_rng(9)
    c = rng.standard_normal((s.K, 128, 128))
    SHx = T.decompose(x, s.centred)
    lhs = np.sum(SHx * c)
    rhs = np.sum(x * T.adjoint(c, s.centred))
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(SHx) * np.linalg.norm(c)


def test_adjoint_matrix_and_gram_8x8():
    s = F.build_system(8, 8, 1, [1], p=np.array([[1.0]]))  # tiny size needs a trivial fan; identities still hold
    N = 8
    K = s.K
    A = np.zeros((K * N * N, N * N))
    for i in range(N * N):
        e = np.zeros(N * N)
        e[i] = 1
        A[:, i] = T.forward_plain(e.reshape(N, N), s.spectra).ravel()
    B = np.zeros((N * N, K * N * N))
    for i in range(K * N * N):
        e = np.zeros(K * N * N)
        e[i] = 1
        B[:, i] = T.adjoint_plain(e.reshape(K, N, N), s.spectra).ravel()
    assert np.max(np.abs(B - A.T)) < 1e-13
    # SH* SH = F^-1 W F: a circulant with eigenvalues W
    G = A.T @ A
    Fm = np.kron(np.fft.fft(np.eye(N)), np.fft.fft(np.eye(N)))
    ref = np.real(np.linalg.inv(Fm) @ np.diag(s.W.ravel()) @ Fm)
    assert np.max(np.abs(G - ref)) < 1e-12


def test_frame_energy_identity_and_bounds(cfg1):
    s, x = cfg1
    c = T.decompose(x, s.centred)
    X = np.fft.fft2(x)
    e = np.sum(c ** 2)
    assert abs(e - np.sum(s.W * np.abs(X) ** 2) / x.size) < 1e-10 * e
    nx = np.sum(x ** 2)
    assert s.W.min() * nx <= e * (1 + 1e-12) and e <= s.W.max() * nx * (1 + 1e-12)


def test_coefficients_real_for_hermitian_bank(cfg1):
    s, x = cfg1
    X = T.fourier(x)
    z = T.inverse_fourier(X[None] * np.conj(s.centred))
    assert np.max(np.abs(z.imag)) <= 1e-13 * np.max(np.abs(z.real))


def test_threaded_forms_match_plain(cfg1):
    """The multi-threaded scipy.fft forms (the all-cores host baseline) compute the plain forms."""
    s, x = cfg1
    c = T.forward_plain(x, s.spectra)
    ct = T.forward_plain_threaded(x, s.spectra, workers=4)
    assert np.linalg.norm(ct - c) <= 1e-12 * np.linalg.norm(c)
    y = T.inverse_plain(c, s.spectra, s.W)
    yt = T.inverse_plain_threaded(c, s.spectra, s.W, workers=4)
    assert np.linalg.norm(yt - y) <= 1e-12 * np.linalg.norm(y)
    assert np.linalg.norm(yt - x) <= 1e-10 * np.linalg.norm(x)
