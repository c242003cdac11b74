"""Oracle: shearlet decomposition, reconstruction and adjoint, FP64 (test infrastructure only).

Conventions (Section 3.2-3.4): the 2-D FFT is unnormalised and its inverse
carries 1/(N M), as TensorFlow's fft2d / ifft2d do. Fourier transforms of
images and filters use the centred layout of Section 3.3 (zero frequency at
index floor(n/2) along each axis): Fourier(f) = centre(fft2(uncentre(f))).

Readings (paper inconsistent or silent):
  * Conjugation: Algorithm 1 conjugates the image spectrum while its listing
    conjugates the filters; the listing's form (filters conjugated, matching
    the conj(psi) of Definition 2.3) is taken. ``decompose_alg1_as_printed``
    keeps the other form so the difference (a point reflection) stays tested.
  * Coefficients are real planes: the imaginary part is dropped, which is
    exact when every filter spectrum is Hermitian (real kernels).
  * The dual-frame weight W is sum_k |Psi_k|^2 (see oracle.filters).
  * The adjoint is Algorithm 2 without the division by W.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "to_centred",
    "from_centred",
    "fourier",
    "inverse_fourier",
    "decompose",
    "decompose_alg1_as_printed",
    "reconstruct",
    "adjoint",
    "forward_plain",
    "inverse_plain",
    "adjoint_plain",
    "forward_plain_threaded",
    "inverse_plain_threaded",
    "correlate_direct",
]


def _axes(x: np.ndarray, axes):
    return list(range(x.ndim - 2, x.ndim)) if axes is None else list(axes)


def to_centred(x: np.ndarray, axes=None) -> np.ndarray:
    """Natural DFT order -> the centred layout of Section 3.3: along each axis of length n the
    element at index 0 moves to index floor(n/2) (a circular shift by floor(n/2))."""
    ax = _axes(x, axes)
    return np.roll(x, [x.shape[a] // 2 for a in ax], axis=ax)


def from_centred(x: np.ndarray, axes=None) -> np.ndarray:
    """Centred layout -> natural DFT order: the circular shift by -floor(n/2) that undoes to_centred."""
    ax = _axes(x, axes)
    return np.roll(x, [-(x.shape[a] // 2) for a in ax], axis=ax)


def fourier(f: np.ndarray) -> np.ndarray:
    """Fourier(f) = fftshift(fft2(ifftshift(f))) over the last two axes (Section 3.3)."""
    return to_centred(np.fft.fft2(from_centred(f)))


def inverse_fourier(F: np.ndarray) -> np.ndarray:
    """InverseFourier(F) = fftshift(ifft2(ifftshift(F))) over the last two axes (Section 3.3)."""
    return to_centred(np.fft.ifft2(from_centred(F)))


def decompose(x: np.ndarray, filters_centred: np.ndarray) -> np.ndarray:
    """Algorithm 1 / its TensorFlow listing (Section 3.4.2), one image (N, M) -> (K, N, M).

    coeffs_i = InverseFourier(Fourier(x) * conj(shearletFilters_i)), real part.
    """
    X = fourier(np.asarray(x, dtype=np.float64))
    return np.real(inverse_fourier(X[None, :, :] * np.conj(filters_centred)))


def decompose_alg1_as_printed(x: np.ndarray, filters_centred: np.ndarray) -> np.ndarray:
    """Algorithm 1 exactly as printed: the conjugate is taken of the image spectrum."""
    X = fourier(np.asarray(x, dtype=np.float64))
    return np.real(inverse_fourier(filters_centred * np.conj(X)[None, :, :]))


def reconstruct(coeffs: np.ndarray, filters_centred: np.ndarray, W_centred: np.ndarray) -> np.ndarray:
    """Algorithm 2 / its listing: f = InverseFourier( sum_i Fourier(c_i) * Psi_i / W ), real part."""
    S = np.sum(fourier(np.asarray(coeffs, dtype=np.float64)) * filters_centred, axis=0)
    return np.real(inverse_fourier(S / W_centred))


def adjoint(coeffs: np.ndarray, filters_centred: np.ndarray) -> np.ndarray:
    """Adjoint SH*: Algorithm 2 without the division by W."""
    S = np.sum(fourier(np.asarray(coeffs, dtype=np.float64)) * filters_centred, axis=0)
    return np.real(inverse_fourier(S))


def forward_plain(x: np.ndarray, spectra: np.ndarray) -> np.ndarray:
    """Shift-free form: c_k = Re ifft2(fft2(x) * conj(Psi_k)), filters in natural order."""
    return np.real(np.fft.ifft2(np.fft.fft2(np.asarray(x, dtype=np.float64))[None] * np.conj(spectra)))


def inverse_plain(coeffs: np.ndarray, spectra: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Shift-free form: y = Re ifft2( sum_k fft2(c_k) Psi_k / W )."""
    return np.real(np.fft.ifft2(np.sum(np.fft.fft2(np.asarray(coeffs, dtype=np.float64)) * spectra, axis=0) / W))


def adjoint_plain(coeffs: np.ndarray, spectra: np.ndarray) -> np.ndarray:
    """Shift-free adjoint: y = Re ifft2( sum_k fft2(c_k) Psi_k )."""
    return np.real(np.fft.ifft2(np.sum(np.fft.fft2(np.asarray(coeffs, dtype=np.float64)) * spectra, axis=0)))


def forward_plain_threaded(x: np.ndarray, spectra: np.ndarray, workers: int) -> np.ndarray:
    """forward_plain with scipy.fft's multi-threaded FFTs (the K planes' transforms split over
    `workers` threads); same definition, different FFT library and summation order."""
    import scipy.fft as sf

    X = sf.fft2(np.asarray(x, dtype=np.float64), workers=workers)
    return np.real(sf.ifft2(X[None] * np.conj(spectra), workers=workers))


def inverse_plain_threaded(coeffs: np.ndarray, spectra: np.ndarray, W: np.ndarray, workers: int) -> np.ndarray:
    """inverse_plain with scipy.fft's multi-threaded FFTs over `workers` threads."""
    import scipy.fft as sf

    S = np.sum(sf.fft2(np.asarray(coeffs, dtype=np.float64), workers=workers) * spectra, axis=0)
    return np.real(sf.ifft2(S / W, workers=workers))


def correlate_direct(x: np.ndarray, kernel: np.ndarray) -> np.ndarray:
    """Brute-force circular correlation c[n] = sum_m x[m] h[(m - n) mod (N, M)], h indexed from 0.

    For small inputs only (O(N^2 M^2)); the plain definition of what the
    forward transform computes for the filter whose inverse DFT is h.
    """
    N, M = x.shape
    out = np.zeros((N, M))
    for n0 in range(N):
        for n1 in range(M):
            acc = 0.0
            for m0 in range(N):
                for m1 in range(M):
                    acc += x[m0, m1] * kernel[(m0 - n0) % N, (m1 - n1) % M]
            out[n0, n1] = acc
    return out
