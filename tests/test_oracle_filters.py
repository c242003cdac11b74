"""Pins of the oracle's shearlet system (CPU, FP64).

The filter values the paper used are MATLAB outputs that it does not print,
so the system is pinned by what the paper fixes (filter count, index triples,
design conditions of the low-pass and the fan filter) and by an independent
spatial re-construction of the digital shear (eqs. (2.4)-(2.5)) written out
below with plain convolutions.
"""
import os

import numpy as np
import pytest

from oracle import filters as F

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line)
    return rows


# ---------------------------------------------------------------- low-pass design


def _dtft_fft(taps, n=4096):
    """DTFT of centred taps sampled by a zero-padded library FFT (independent of the oracle's evaluator)."""
    r = len(taps) // 2
    buf = np.zeros(n)
    buf[: r + 1] = taps[r:]
    buf[n - r :] = taps[:r]
    return np.fft.fft(buf)


def test_scaling_filter_design_conditions():
    h = F.default_scaling_filter()
    assert h.shape == (9,)
    assert np.allclose(h, h[::-1], atol=0)  # linear phase
    H = _dtft_fft(h, 4096)
    assert abs(H[0] - 1) < 1e-14  # unit DC gain
    assert abs(H[2048]) < 1e-14  # zero at pi
    assert abs(abs(H[1024]) - 2 ** -0.5) < 1e-14  # half power at half band
    assert np.max(np.abs(H.imag)) < 1e-14
    # maximal flatness: 1 - H(w) = O(w^6) near 0
    w = 2 * np.pi * np.arange(1, 6) / 4096
    dev = np.abs(1 - H[1:6].real)
    assert np.all(dev < 5.0 * w ** 6)
    # monotone low-pass on [0, pi]
    assert np.all(np.diff(H[:2049].real) <= 1e-15)


def test_mirror_filter_is_highpass():
    h = F.default_scaling_filter()
    g = F.mirror_filter(h)
    G = _dtft_fft(g, 4096)
    H = _dtft_fft(h, 4096)
    assert abs(G[0]) < 1e-14 and abs(G[2048] - 1) < 1e-14
    assert np.allclose(G, np.roll(H, 2048), atol=1e-14)  # ghat(w) = hhat(w + pi)


def test_fan_filter_properties():
    p = F.default_fan_filter()
    assert p.shape == (15, 15)
    n = 64
    buf = np.zeros((n, n))
    r = 7
    buf[np.ix_(np.arange(-r, r + 1) % n, np.arange(-r, r + 1) % n)] = p
    P = np.fft.fft2(buf)
    assert np.max(np.abs(P.imag)) < 1e-14
    P = P.real
    assert abs(P[n // 2, 0] - 1) < 1e-14  # pass band at (pi, 0)
    assert abs(P[0, n // 2]) < 1e-14  # stop band at (0, pi)
    # half-band: P(w) + P(w + (pi, pi)) = 1
    assert np.allclose(P + np.roll(P, (n // 2, n // 2), axis=(0, 1)), 1.0, atol=1e-13)
    # fan geometry: > 1/2 inside |w2| < |w1|, < 1/2 inside |w2| > |w1| (centred frequencies)
    f = np.fft.fftfreq(n) * n
    a, b = np.meshgrid(np.abs(f), np.abs(f), indexing="ij")
    assert np.all(P[(b < a)] >= 0.5 - 1e-13)
    assert np.all(P[(b > a)] <= 0.5 + 1e-13)


def test_fan_filter_flatness_order():
    """Maximal flatness of order L = 4 (Section 3.4.1's maxflat design): 1 - P vanishes to order 2L = 8
    at the pass-band centre (pi, 0) and P to order 8 at the stop-band centre (0, pi). Evaluated by the
    plain trigonometric sum of the taps: halving the distance divides the deviation by 2^8 (an order-6
    or order-10 design would give 2^6 or 2^10)."""
    p = F.default_fan_filter()
    r = p.shape[0] // 2
    n = np.arange(-r, r + 1)

    def P(w1, w2):
        return float(np.real(np.sum(p * np.exp(-1j * (w1 * n[:, None] + w2 * n[None, :])))))

    for a, b in ((1.0, 0.0), (0.6, 0.8), (0.0, 1.0), (0.8, -0.6)):
        for eps in (0.1, 0.05):
            dev = [1.0 - P(np.pi + a * e, b * e) for e in (eps, eps / 2)]
            assert 0.8 * 256 < dev[0] / dev[1] < 1.2 * 256, (a, b, eps, dev)
            stop = [P(a * e, np.pi + b * e) for e in (eps, eps / 2)]
            assert 0.8 * 256 < stop[0] / stop[1] < 1.2 * 256, (a, b, eps, stop)


# ---------------------------------------------------------------- counts and indices


@pytest.mark.parametrize("row", _read_golden("filter_counts.txt"))
def test_filter_count_formula(row):
    lv, k = row.split(";")
    levels = [int(v) for v in lv.split(",")]
    K = int(k)
    assert F.n_shearlets(levels) == K
    sys_ = F.build_system(64 if max(levels) < 2 else 128, 64 if max(levels) < 2 else 128, len(levels), levels)
    assert sys_.K == K
    assert sys_.idx.shape == (K, 3)


def test_default_shear_levels():
    assert F.shear_levels_default(2) == [1, 1]
    assert F.shear_levels_default(3) == [1, 1, 2]
    assert F.shear_levels_default(4) == [1, 1, 2, 2]


def test_figure_index_triples_exist():
    s = F.build_system(128, 128, 4)  # index triples only; size is irrelevant here
    have = {tuple(int(v) for v in t) for t in s.idx}
    for row in _read_golden("figure_indices.txt"):
        assert tuple(int(v) for v in row.split(",")) in have
    assert tuple(s.idx[-1]) == (0, 0, 0)


# ---------------------------------------------------------------- structural identities


@pytest.fixture(scope="module")
def sys128():
    return F.build_system(128, 128, 2)


def test_spectra_real_even_hermitian(sys128):
    S = sys128.spectra
    assert np.max(np.abs(S.imag)) < 1e-14
    mirror = S[:, (-np.arange(128)) % 128][:, :, (-np.arange(128)) % 128]
    assert np.max(np.abs(mirror - np.conj(S))) < 1e-14


def test_bandpass_zero_dc_lowpass_unit_dc(sys128):
    S = sys128.spectra
    assert np.max(np.abs(S[:-1, 0, 0])) < 1e-15
    assert abs(S[-1, 0, 0] - 1) < 1e-15


def test_cone2_is_transpose_of_cone1(sys128):
    S, idx = sys128.spectra, sys128.idx
    pos = {tuple(t): i for i, t in enumerate(map(tuple, idx))}
    for (c, j, k), i in pos.items():
        if c == 2:
            assert np.allclose(S[i], S[pos[(1, j, k)]].T, atol=1e-15)


def test_shear_mirror_symmetry(sys128):
    # Psi_{1,j,-k}(w1, w2) = Psi_{1,j,k}(w1, -w2): the design is symmetric in x2
    S, idx = sys128.spectra, sys128.idx
    pos = {tuple(t): i for i, t in enumerate(map(tuple, idx))}
    neg = (-np.arange(128)) % 128
    for (c, j, k), i in pos.items():
        if c == 1:
            assert np.allclose(S[pos[(1, j, -k)]], S[i][:, neg], atol=1e-14)


def test_frame_weight_positive_and_bounded(sys128):
    W = sys128.W
    assert W.min() > 0.5 and W.max() < 3.0


def test_rms_is_kernel_l2_norm(sys128):
    kern = np.fft.ifft2(sys128.spectra)
    assert np.allclose(sys128.rms, np.sqrt(np.sum(np.abs(kern) ** 2, axis=(1, 2))), rtol=1e-13)


def test_system_fits_policy():
    assert F.system_fits(128, 128, 2, [1, 1])
    assert F.system_fits(256, 256, 3, [1, 1, 2])
    assert F.system_fits(512, 512, 4, [1, 1, 2, 2])
    assert not F.system_fits(64, 64, 4, [1, 1, 2, 2])
    assert not F.system_fits(32, 32, 2, [1, 1])


# ---------------------------------------------------------------- spatial re-construction pin


def _up(x, U, axis):
    shp = list(x.shape)
    shp[axis] = (shp[axis] - 1) * U + 1
    out = np.zeros(shp)
    sl = [slice(None)] * x.ndim
    sl[axis] = slice(None, None, U)
    out[tuple(sl)] = x
    return out


def _conv(x, taps, axis):
    return np.apply_along_axis(lambda v: np.convolve(v, taps), axis, x)


def _atrous_low_taps(h, level):
    out = np.array([1.0])
    for i in range(level):
        out = np.convolve(out, _up(h, 2 ** i, 0))
    return out


def _spatial_wedge(h, p, s, k):
    """Directional filter narrowed by 2^s along x2, then digitally sheared per eqs. (2.5), (2.4)."""
    U = 2 ** s
    hs = _atrous_low_taps(h, s)
    ps = _conv(_up(p, U, 1), hs, 1)
    q = _conv(_up(ps, U, 0), hs, 0)
    r0, r1 = q.shape[0] // 2, q.shape[1] // 2
    R0 = r0 + abs(k) * r1
    qk = np.zeros((2 * R0 + 1, q.shape[1]))
    for n1 in range(-R0, R0 + 1):
        for n2 in range(-r1, r1 + 1):
            src = n1 + k * n2
            if -r0 <= src <= r0:
                qk[n1 + R0, n2 + r1] = q[src + r0, n2 + r1]
    rk = _conv(qk, hs[::-1], 0)
    c = rk.shape[0] // 2
    keep = np.arange(c % U, rk.shape[0], U)
    assert c in keep
    return U * rk[keep]


def _embed(kern, N, M):
    out = np.zeros((N, M))
    r0, r1 = kern.shape[0] // 2, kern.shape[1] // 2
    ii, jj = np.meshgrid(np.arange(-r0, r0 + 1) % N, np.arange(-r1, r1 + 1) % M, indexing="ij")
    np.add.at(out, (ii, jj), kern)  # wraps circularly when the kernel is larger than the grid
    return out


def _spatial_kernels(levels):
    """Every kernel of a system built spatially, in the filter order: ((cone, j, k), kernel)."""
    J = len(levels)
    h = F.default_scaling_filter()
    g = F.mirror_filter(h)
    p = F.default_fan_filter()
    out = []
    for j in range(1, J + 1):
        s = levels[j - 1]
        U = 2 ** s
        lvl = J - j + 1
        band = np.convolve(_up(g, 2 ** (lvl - 1), 0), _atrous_low_taps(h, lvl - 1))
        for cone, ks in ((1, range(-U, U + 1)), (2, range(-U + 1, U))):
            for k in ks:
                ker = _conv(_spatial_wedge(h, p, s, k), band, 0)
                out.append(((cone, j, k), ker.T if cone == 2 else ker))
    low = _atrous_low_taps(h, J)
    out.append(((0, 0, 0), np.outer(low, low)))
    return out


@pytest.mark.parametrize("N,M,levels", [(128, 128, [1, 1]), (96, 128, [1, 2]), (256, 256, [1, 1, 2]),
                                        (512, 512, [1, 1, 2, 2])])
def test_spectra_equal_dft_of_spatial_construction(N, M, levels):
    """All K filters of the system, the 4-scale [1, 1, 2, 2] system of the 512 x 512 workload included
    (band-pass levels 3-4 and the level-4 low-pass), against the DFT of the spatial construction."""
    sysx = F.build_system(N, M, len(levels), levels)
    kers = _spatial_kernels(levels)
    assert len(kers) == sysx.K
    for i, (trip, ker) in enumerate(kers):
        ref = np.fft.fft2(_embed(ker, N, M))
        assert tuple(sysx.idx[i]) == trip
        assert np.max(np.abs(ref - sysx.spectra[i])) < 1e-12 * max(1.0, np.max(np.abs(ref))), trip


@pytest.mark.parametrize("levels", [[1, 1], [1, 2], [1, 1, 2], [1, 1, 2, 2], [0, 1, 2], [2, 2, 2, 2, 3]])
def test_kernel_radii_match_spatial_supports(levels):
    """kernel_radii (and so system_fits) against the supports of the spatially built kernels: each
    kernel's array is (2 r0 + 1) x (2 r1 + 1) and its outermost non-zero taps reach both half-widths."""
    rad = F.kernel_radii(len(levels), levels, 9, (15, 15))
    kers = _spatial_kernels(levels)
    assert len(rad) == len(kers)
    for (cone, j, k, r0, r1), (trip, ker) in zip(rad, kers):
        assert (cone, j, k) == trip
        assert ker.shape == (2 * r0 + 1, 2 * r1 + 1), trip
        nz0, nz1 = np.nonzero(ker)
        assert np.max(np.abs(nz0 - r0)) == r0 and np.max(np.abs(nz1 - r1)) == r1, trip
    # a system fits exactly when its widest kernel does
    w0 = max(2 * r[3] + 1 for r in rad)
    w1 = max(2 * r[4] + 1 for r in rad)
    assert F.system_fits(w0, w1, len(levels), levels)
    assert not F.system_fits(w0 - 1, w1, len(levels), levels) and not F.system_fits(w0, w1 - 1, len(levels), levels)
