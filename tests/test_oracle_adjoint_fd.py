"""FP64 finite-difference pins of the oracle's adjoint (the gradient the
autograd layer's backward must reproduce): for the linear forward map SH,
<g, (SH(x + e v) - SH(x - e v)) / (2 e)> = <SH* g, v> for every x, v, g."""
import numpy as np
import pytest

from oracle import filters as OF
from oracle import transform as OT


def _bank(rng, K, N, M):
    ker = rng.standard_normal((K, N, M))  # real kernels: Hermitian spectra
    return np.fft.fft2(ker)


@pytest.mark.parametrize("eps", [1e-3, 1.0])
def test_fd_gradient_32x32(eps):
    rng = np.random.default_rng(2006)
    K, N, M = 5, 32, 32
    S = _bank(rng, K, N, M)
    x = rng.standard_normal((N, M))
    g = rng.standard_normal((K, N, M))
    grad = OT.adjoint_plain(g, S)
    worst = 0.0
    for _ in range(6):
        v = rng.standard_normal((N, M))
        fd = (np.vdot(g, OT.forward_plain(x + eps * v, S)) - np.vdot(g, OT.forward_plain(x - eps * v, S))) / (2 * eps)
        worst = max(worst, abs(fd - np.vdot(grad, v)) / abs(np.vdot(grad, v)))
    assert worst <= 1e-9


def test_fd_gradient_coordinates_16x16():
    # full gradient by central differences along every pixel direction
    rng = np.random.default_rng(7)
    K, N, M = 3, 16, 16
    S = _bank(rng, K, N, M)
    x = rng.standard_normal((N, M))
    g = rng.standard_normal((K, N, M))
    fd = np.empty((N, M))
    for i in range(N):
        for j in range(M):
            e = np.zeros((N, M))
            e[i, j] = 0.5
            fd[i, j] = (np.vdot(g, OT.forward_plain(x + e, S)) - np.vdot(g, OT.forward_plain(x - e, S))) / 1.0
    assert np.max(np.abs(fd - OT.adjoint_plain(g, S))) <= 1e-10 * np.max(np.abs(fd))


def test_fd_gradient_default_system_128():
    ref = OF.build_system(128, 128, 2)
    rng = np.random.default_rng(11)
    x = rng.standard_normal((128, 128))
    v = rng.standard_normal((128, 128))
    g = rng.standard_normal((ref.K, 128, 128))
    fd = (np.vdot(g, OT.forward_plain(x + v, ref.spectra)) - np.vdot(g, OT.forward_plain(x - v, ref.spectra))) / 2
    want = np.vdot(OT.adjoint_plain(g, ref.spectra), v)
    assert abs(fd - want) <= 1e-10 * abs(want)
