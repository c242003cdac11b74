"""Pins of the learned-shrinkage oracle: bfloat16 rounding against the format's
definition, the circular 3x3 correlation against scipy, identity and shift
kernels, and the untrained network's reduction to plain hard thresholding."""
import numpy as np
import pytest
from scipy import signal

from oracle import apps as A
from oracle import shrink as S


def test_bf16_known_values():
    v = S.to_bf16(np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1.5, 3.14159, 0.0, 2 ** -130, 65280.0]))
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties go to the even significand (1);
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: to 1 + 2^-6
    assert list(v[:6]) == [1.0, 1.0, 1 + 2 ** -6, -1.5, 3.140625, 0.0]
    assert v[6] == np.float32(2 ** -130)  # subnormal, representable with 7 significand bits
    assert v[7] == 65280.0


def test_bf16_error_bound_and_idempotence():
    rng = np.random.default_rng(0)
    x = rng.standard_normal(10000) * 10.0 ** rng.uniform(-5, 5, 10000)
    r = S.to_bf16(x)
    assert np.all(np.abs(r - x) <= 2.0 ** -8 * np.abs(x) * (1 + 1e-6))
    assert np.array_equal(S.to_bf16(r), r)
    # representable numbers: 8 significant bits
    m, _ = np.frexp(r[r != 0])
    assert np.all(np.mod(m * 2 ** 8, 1.0) == 0.0)


def test_softplus():
    assert S.softplus(0.0) == pytest.approx(np.log(2.0), rel=1e-15)
    assert S.softplus(50.0) == pytest.approx(50.0, rel=1e-15)
    assert S.softplus(-40.0) == pytest.approx(np.exp(-40.0), rel=1e-12)
    x = np.linspace(-5, 5, 11)
    assert np.allclose(S.softplus(x), np.log1p(np.exp(x)), rtol=1e-14)


def test_conv_matches_scipy_wrap():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((3, 9, 12))
    W = rng.standard_normal((2, 3, 3, 3))
    b = rng.standard_normal(2)
    got = S.conv3x3_circular(x, W, b)
    for co in range(2):
        want = b[co] + sum(signal.correlate2d(x[ci], W[co, ci], mode="same", boundary="wrap") for ci in range(3))
        assert np.allclose(got[co], want, rtol=1e-13, atol=1e-13)


def test_conv_identity_and_shift():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((4, 8, 8))
    W = np.zeros((4, 4, 3, 3))
    for c in range(4):
        W[c, c, 1, 1] = 1.0
    assert np.array_equal(S.conv3x3_circular(x, W), x)
    Ws = np.zeros((1, 4, 3, 3))
    Ws[0, 2, 0, 1] = 1.0  # tap (dy, dx) = (0, 1): reads in(y - 1, x)
    got = S.conv3x3_circular(x, Ws)[0]
    assert np.array_equal(got, np.roll(x[2], 1, axis=0))
    assert got[0, 3] == x[2, 7, 3]


def test_untrained_network_is_hard_thresholding():
    rng = np.random.default_rng(3)
    K, N = 5, 16
    c = rng.standard_normal((K, N, N)) * 20.0
    rms = rng.uniform(0.1, 0.5, K)
    sigma = 7.0
    p = S.init_params(K, hidden=8, seed=4, tau0=3.0)
    p.W3[:] = 0.0
    out, tau = S.shrink(c, sigma, rms, p)
    assert np.allclose(tau[:-1], 3.0, rtol=1e-6) and np.all(tau[-1] == 0.0)
    delta = 3.0 * sigma * rms
    delta[-1] = 0.0
    want = A.hard_threshold(c, delta * (1 + 1e-7))  # tau is softplus(log(e^3 - 1)) = 3 to rounding
    assert np.array_equal(out, want) or np.array_equal(out, A.hard_threshold(c, delta * (1 - 1e-7)))


def test_init_params_output_bias():
    p = S.init_params(7, seed=0, tau0=2.5)
    assert np.allclose(S.softplus(p.b3), 2.5, rtol=1e-6)
    assert p.W1.shape == (32, 7, 3, 3) and p.W3.shape == (7, 32, 3, 3)
    assert np.array_equal(S.to_bf16(p.W2), p.W2)


def test_conv_adjoint_identity():
    rng = np.random.default_rng(21)
    x = rng.standard_normal((3, 8, 16))
    d = rng.standard_normal((4, 8, 16))
    W = rng.standard_normal((4, 3, 3, 3))
    lhs = np.vdot(S.conv3x3_circular(x, W), d)
    rhs = np.vdot(x, S.conv3x3_adjoint(d, W))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_train_loss_gradients_match_finite_differences():
    """Unrounded network in FP64: every analytic gradient equals central differences of the loss."""
    rng = np.random.default_rng(22)
    K, N, M = 3, 8, 16
    rms = rng.uniform(0.2, 0.6, K)
    sigma = 5.0
    cc = rng.standard_normal((K, N, M)) * 20.0 * rms[:, None, None]
    cn = cc + rng.standard_normal((K, N, M)) * sigma * rms[:, None, None]
    p = S.init_params(K, seed=23, tau0=2.0)
    p.W3 *= 20.0
    p.b1 += rng.standard_normal(32) * 0.1
    p.b2 += rng.standard_normal(32) * 0.1
    T, scale = 0.5, 1.0 / cn.size
    L0, g = S.train_loss(cn, cc, sigma, rms, p, T, scale, rounded=False)
    assert L0 > 0
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        arr = getattr(p, name)
        flat = arr.reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            h = 1e-4 * max(1.0, abs(old))
            flat[idx] = old + h
            Lp, _ = S.train_loss(cn, cc, sigma, rms, p, T, scale, rounded=False)
            flat[idx] = old - h
            Lm, _ = S.train_loss(cn, cc, sigma, rms, p, T, scale, rounded=False)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            an = g[name].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g[name]).max()), (name, idx, fd, an)
