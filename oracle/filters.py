"""Oracle: the shearlet system in the Fourier domain, FP64 (test infrastructure only).

Follows the digital construction of Section 2.1 (two-scale filters h, g,
eqs. (2.1)-(2.2); iterated filters; generator = fan filter times separable
wavelet; digital shear operator, eqs. (2.4)-(2.5); digital shearlets,
Definition 2.3 / eq. (2.6)) with the default filters of Section 3.4.1, and the
filter count of Section 3.4.1 (nShearlets).

Readings taken where the paper is silent, garbled or inconsistent:
  * Scales j = 1..J, scale 1 coarsest; shear level s_j = ceil(j/2); shears
    |k| <= 2^{s_j} (the range of the reconstruction formula after eq. (2.7)).
    Cone 1 keeps all 2^{s+1}+1 shears, cone 2 the 2^{s+1}-1 with |k| < 2^s,
    plus one low-pass: K = 1 + sum_j 2^{s_j+2} (17 / 33 / 49 for J = 2 / 3 / 4),
    which is the nShearlets formula with |K_j| = 2*2^{s_j}+1.
  * Default low-pass h: the 9-tap symmetric filter fixed by the design spec of
    Section 3.4.1 (order 8, maximally flat, half-power at half band):
    hhat(0) = 1, hhat''(0) = hhat''''(0) = 0, hhat(pi) = 0, hhat(pi/2) = 1/sqrt 2.
    The mirror high-pass is g[n] = (-1)^n h[n].
  * Default fan filter: the maximally flat diamond half-band filter obtained
    by a McClellan mapping cos w -> (cos w1 + cos w2)/2 of the 1-D maxflat
    half-band polynomial of order L = 4, modulated by (-1)^{n1} into a fan
    whose pass band is |w2| < |w1|, with unit peak gain.
  * Axis 0 of the array plays x1 (the axis of the wavelet); cone 2 is cone 1
    with the axes exchanged.
  * Shearlet (cone 1, scale j, shear k) = band(j) * wedge(s_j, k), with
    band(j) = ghat_{J-j+1}(w1) (a-trous high-pass) and the wedge the spectrum
    of the digitally sheared directional filter:
      1. narrow the fan by 2^s along x2: upsample along x2 by U = 2^s and
         convolve along x2 with the a-trous low-pass h_(s);
      2. eqs. (2.5), (2.4): upsample along x1 by U, convolve along x1 with
         h_(s), shear n -> (n1 + k n2, n2), convolve along x1 with the
         reversed h_(s), keep every U-th sample along x1 and scale by U.
    In the Fourier domain these steps give the closed form implemented in
    ``wedge_response``.
  * Low-pass = hhat_J(w1) hhat_J(w2).
  * RMS_k = ||Psi_k||_F / sqrt(N M) (Section 3.4.1, used by the denoising
    listing of Section 4.2).
  * Dual-frame weight (used in Algorithm 2, never defined): W = sum_k |Psi_k|^2,
    the unique pointwise weight that makes Algorithm 2 invert Algorithm 1.
"""
from __future__ import annotations

from dataclasses import dataclass
from math import comb, gcd

import numpy as np

__all__ = [
    "default_scaling_filter",
    "mirror_filter",
    "default_fan_filter",
    "shear_levels_default",
    "n_shearlets",
    "dtft_on_grid",
    "atrous_lowpass",
    "atrous_highpass",
    "wedge_response",
    "ShearletSystem",
    "build_system",
    "kernel_radii",
    "system_fits",
]


def default_scaling_filter() -> np.ndarray:
    """9-tap symmetric low-pass h[-4..4] of Section 3.4.1 (see module readings).

    With hhat(w) = a0 + 2 sum_{n=1..4} a_n cos(n w) the five design conditions
    are linear in (a0..a4) and are solved directly.
    """
    rows = np.array(
        [
            [1, 2, 2, 2, 2],  # hhat(0) = 1
            [0, 1, 4, 9, 16],  # second derivative at 0 vanishes: sum n^2 a_n = 0
            [0, 1, 16, 81, 256],  # fourth derivative at 0 vanishes: sum n^4 a_n = 0
            [1, -2, 2, -2, 2],  # hhat(pi) = 0
            [1, 0, -2, 0, 2],  # hhat(pi/2) = 1/sqrt(2)
        ],
        dtype=np.float64,
    )
    rhs = np.array([1.0, 0.0, 0.0, 0.0, 2.0 ** -0.5])
    a = np.linalg.solve(rows, rhs)
    return np.concatenate([a[:0:-1], a])


def mirror_filter(h: np.ndarray) -> np.ndarray:
    """Mirror high-pass g[n] = (-1)^n h[n], n counted from the centre tap (Section 3.4.1)."""
    r = len(h) // 2
    n = np.arange(-r, r + 1)
    return np.where(n % 2 == 0, 1.0, -1.0) * h


def default_fan_filter(order: int = 4) -> np.ndarray:
    """Fan filter kernel p[n1, n2] (Section 3.4.1 reading; odd x odd, centred).

    Frequency response P(w1, w2) = H(y), y = (1 - t)/2,
    t = (cos w2 - cos w1)/2, H(y) = (1-y)^L sum_{i<L} C(L-1+i, i) y^i.
    P is a trigonometric polynomial of degree d = 2L-1 in each variable, so its
    Fourier coefficients are obtained exactly from samples on a grid of
    size >= 2d+1.
    """
    L = order
    d = 2 * L - 1
    g = 4 * (d + 1)
    w = 2 * np.pi * np.arange(g) / g
    w1, w2 = np.meshgrid(w, w, indexing="ij")
    t = (np.cos(w2) - np.cos(w1)) / 2
    y = (1 - t) / 2
    H = (1 - y) ** L * sum(comb(L - 1 + i, i) * y ** i for i in range(L))
    coef = np.fft.fftshift(np.real(np.fft.ifft2(H)))
    c = g // 2
    return coef[c - d : c + d + 1, c - d : c + d + 1].copy()


def shear_levels_default(n_scales: int) -> list[int]:
    """s_j = ceil(j/2) for j = 1..J."""
    return [(j + 1) // 2 for j in range(1, n_scales + 1)]


def n_shearlets(levels) -> int:
    """K = 2 sum_j (|K_j| - 1) + 1 with |K_j| = 2*2^{s_j} + 1 (Section 3.4.1)."""
    return 2 * sum(2 * 2 ** s for s in levels) + 1


def dtft_on_grid(taps: np.ndarray, Q: int) -> np.ndarray:
    """1-D DTFT of centred real taps at w = 2 pi q / Q, q = 0..Q-1."""
    r = len(taps) // 2
    n = np.arange(-r, r + 1)
    q = np.arange(Q)
    ph = (np.outer(q, n) % Q).astype(np.float64)
    return np.exp(-2j * np.pi * ph / Q) @ taps.astype(np.complex128)


def _dtft2_on_grid(taps: np.ndarray, Q0: int, Q1: int) -> np.ndarray:
    """2-D DTFT of a centred kernel at (2 pi q0/Q0, 2 pi q1/Q1)."""
    r0, r1 = taps.shape[0] // 2, taps.shape[1] // 2
    n0 = np.arange(-r0, r0 + 1)
    n1 = np.arange(-r1, r1 + 1)
    E0 = np.exp(-2j * np.pi * (np.outer(np.arange(Q0), n0) % Q0) / Q0)
    E1 = np.exp(-2j * np.pi * (np.outer(np.arange(Q1), n1) % Q1) / Q1)
    return E0 @ taps.astype(np.complex128) @ E1.T


def atrous_lowpass(Hq: np.ndarray, level: int, idx: np.ndarray) -> np.ndarray:
    """hhat_l(w) = prod_{i<l} hhat(2^i w) (Section 2.1), at w = 2 pi idx / Q, Hq = hhat on the Q-grid."""
    Q = len(Hq)
    out = np.ones(np.shape(idx), dtype=np.complex128)
    for i in range(level):
        out = out * Hq[(idx * 2 ** i) % Q]
    return out


def atrous_highpass(Hq: np.ndarray, Gq: np.ndarray, level: int, idx: np.ndarray) -> np.ndarray:
    """ghat_l(w) = ghat(2^{l-1} w) hhat_{l-1}(w) (Section 2.1), level >= 1."""
    Q = len(Hq)
    return Gq[(idx * 2 ** (level - 1)) % Q] * atrous_lowpass(Hq, level - 1, idx)


def _lcm(a: int, b: int) -> int:
    return a * b // gcd(a, b)


def wedge_response(R: int, C: int, h: np.ndarray, p: np.ndarray, s: int, k: int) -> np.ndarray:
    """Spectrum D_{s,k} of the digitally sheared directional filter on an R x C DFT grid.

    With a = 2 pi m1/R (axis 0 = x1), b = 2 pi m2/C, U = 2^s and Hs = hhat_(s):
        D(a, b) = P(a, U b - k a) * sum_{m=0}^{U-1} |Hs(alpha_m)|^2 Hs(b - k alpha_m),
        alpha_m = (a + 2 pi m)/U,
    which is the Fourier image of the spatial steps listed in the module
    docstring (narrowing, then eqs. (2.5) and (2.4)). Every argument is a rational
    multiple of 2 pi, so each factor is read off an exact DFT grid.
    """
    U = 2 ** s
    m1 = np.arange(R)[:, None]
    m2 = np.arange(C)[None, :]
    # fan factor P(a, U b - k a): second argument = 2 pi (U m2/C - k m1/R) on the lcm(R, C) grid
    Q = _lcm(R, C)
    Pg = _dtft2_on_grid(p, R, Q)
    col = (U * m2 * (Q // C) - k * m1 * (Q // R)) % Q
    fan = Pg[np.broadcast_to(m1, (R, C)), col]
    # interpolation sum over the U aliases of the x1 down-sampling
    QA = R * U
    HA = dtft_on_grid(h, QA)
    QB = _lcm(C, R * U)
    HB = dtft_on_grid(h, QB)
    acc = np.zeros((R, C), dtype=np.complex128)
    for m in range(U):
        ia = m1 + m * R  # alpha_m = 2 pi ia / (R U)
        Ha = atrous_lowpass(HA, s, ia)
        ib = (m2 * (QB // C) - k * ia * (QB // (R * U))) % QB
        Hb = atrous_lowpass(HB, s, ib)
        acc = acc + np.abs(Ha) ** 2 * Hb
    return fan * acc


def _cone1_spectrum(R: int, C: int, h: np.ndarray, g: np.ndarray, p: np.ndarray, J: int, j: int, s: int, k: int) -> np.ndarray:
    """Cone-1 shearlet (scale j, shear k) on an R x C grid: band(j) * wedge(s, k)."""
    level = J - j + 1
    idx = np.arange(R)[:, None]
    band = atrous_highpass(dtft_on_grid(h, R), dtft_on_grid(g, R), level, idx)
    return band * wedge_response(R, C, h, p, s, k)


def kernel_radii(J: int, levels, h_len: int, p_shape) -> list[tuple[int, int, int, int, int]]:
    """Spatial half-widths (cone, scale, shear, r0, r1) of every constructed kernel.

    r0 / r1 are the half-widths along axis 0 / axis 1 that the construction
    steps produce (upsampling multiplies a half-width by U, a convolution adds
    the filter's half-width, the shear adds |k| times the x2 half-width, the
    down-sampling divides by U rounding down).
    """
    rh = h_len // 2
    p0, p1 = p_shape[0] // 2, p_shape[1] // 2
    out = []
    for j in range(1, J + 1):
        s = levels[j - 1]
        U = 2 ** s
        level = J - j + 1
        band = rh * 2 ** (level - 1) + rh * (2 ** (level - 1) - 1)
        rhs_ = rh * (U - 1)  # half-width of h_(s)
        q1 = p1 * U + rhs_
        q0 = p0 * U + rhs_
        for cone, ks in ((1, range(-U, U + 1)), (2, range(-U + 1, U))):
            for k in ks:
                d0 = (q0 + abs(k) * q1 + rhs_) // U
                r0, r1 = d0 + band, q1
                if cone == 2:
                    r0, r1 = r1, r0
                out.append((cone, j, k, r0, r1))
    rl = rh * (2 ** J - 1)
    out.append((0, 0, 0, rl, rl))
    return out


def system_fits(rows: int, cols: int, J: int, levels, h_len: int = 9, p_shape=(15, 15)) -> bool:
    """True when every kernel of the system fits in rows x cols (2r+1 <= size per axis)."""
    return all(2 * r0 + 1 <= rows and 2 * r1 + 1 <= cols for (_, _, _, r0, r1) in kernel_radii(J, levels, h_len, p_shape))


@dataclass
class ShearletSystem:
    """A built system. Spectra are complex128 (K, rows, cols)."""

    rows: int
    cols: int
    levels: list
    spectra: np.ndarray  # natural DFT order (index 0 = zero frequency)
    idx: np.ndarray  # (K, 3) int: cone (0 = low-pass), scale, shear

    @property
    def K(self) -> int:
        return self.spectra.shape[0]

    @property
    def centred(self) -> np.ndarray:
        """Spectra in the paper's centred layout (fftshift of the natural order)."""
        return np.fft.fftshift(self.spectra, axes=(1, 2))

    @property
    def W(self) -> np.ndarray:
        """Dual-frame weight sum_k |Psi_k|^2, natural order."""
        return np.sum(np.abs(self.spectra) ** 2, axis=0)

    @property
    def rms(self) -> np.ndarray:
        """RMS_k = ||Psi_k||_F / sqrt(rows cols)."""
        return np.sqrt(np.sum(np.abs(self.spectra) ** 2, axis=(1, 2)) / (self.rows * self.cols))


def build_system(rows: int, cols: int, n_scales: int, levels=None, h: np.ndarray | None = None, p: np.ndarray | None = None) -> ShearletSystem:
    """getshearletsystem2D(rows, cols, nScales, directionalFilter, scalingFilter) (Section 3.4.1).

    Filter order: for each scale j = 1..J, cone 1 shears -2^s..2^s, then cone 2
    shears -(2^s-1)..(2^s-1); the low-pass comes last with index (0, 0, 0).
    """
    J = n_scales
    levels = list(shear_levels_default(J) if levels is None else levels)
    if len(levels) != J:
        raise ValueError("need one shear level per scale")
    h = default_scaling_filter() if h is None else np.asarray(h, dtype=np.float64)
    p = default_fan_filter() if p is None else np.asarray(p, dtype=np.float64)
    g = mirror_filter(h)
    specs, idx = [], []
    for j in range(1, J + 1):
        s = levels[j - 1]
        U = 2 ** s
        for k in range(-U, U + 1):
            specs.append(_cone1_spectrum(rows, cols, h, g, p, J, j, s, k))
            idx.append((1, j, k))
        for k in range(-U + 1, U):
            specs.append(_cone1_spectrum(cols, rows, h, g, p, J, j, s, k).T)
            idx.append((2, j, k))
    HR = dtft_on_grid(h, rows)
    HC = dtft_on_grid(h, cols)
    low = atrous_lowpass(HR, J, np.arange(rows))[:, None] * atrous_lowpass(HC, J, np.arange(cols))[None, :]
    specs.append(low)
    idx.append((0, 0, 0))
    return ShearletSystem(rows, cols, levels, np.array(specs), np.array(idx, dtype=np.int64))
