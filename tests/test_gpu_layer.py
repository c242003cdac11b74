"""GPU parity of the differentiable layer: forward = shear_forward, backward =
shear_adjoint, against the FP64 oracle's forward and adjoint (whose gradient
property the FP64 finite-difference tests pin)."""
import numpy as np
import pytest

import synth
from oracle import filters as OF
from oracle import transform as OT

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(msg):
    print(msg, flush=True)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def test_layer_gradient_32x32(gpu):
    from paper_2006_04591_amd import ShearletLayer, ShearletSystem

    _say("case: layer 32x32 user bank K=5 B=4")
    rng = np.random.default_rng(2006)
    K, N, B = 5, 32, 4
    S = np.fft.fft2(rng.standard_normal((K, N, N)))
    x = rng.standard_normal((B, 1, N, N)).astype(np.float32)
    g = rng.standard_normal((B, K, N, N)).astype(np.float32)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as sys_:
        layer = ShearletLayer(N, N, 0, system=sys_)
        xt = _to(x, gpu).requires_grad_(True)
        c = layer(xt)
        (c * _to(g, gpu)).sum().backward()
        torch.cuda.synchronize()
        assert c.shape == (B, K, N, N) and xt.grad.shape == (B, 1, N, N)
        for b in range(B):
            assert _rel(c[b].detach().cpu().numpy(), OT.forward_plain(x[b, 0].astype(np.float64), S)) <= TOL
            assert _rel(xt.grad[b, 0].cpu().numpy(), OT.adjoint_plain(g[b].astype(np.float64), S)) <= TOL
        # dot-product test in FP32: <g, SH v> = <SH* g, v>
        v = _to(rng.standard_normal((B, N, N)), gpu)
        lhs = float((_to(g, gpu).double() * layer(v).detach().double()).sum())
        rhs = float((sys_.adjoint(_to(g, gpu)).double() * v.double()).sum())
        assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


@pytest.mark.parametrize("forward", ["panel", "whole-plane"])
def test_layer_config4(gpu, forward):
    """32 images of 256x256 (one channel), 33 filters, upstream gradient N(0, 1); the forward in its
    panel form and in the whole-plane form the autotuner may pick at this size."""
    from paper_2006_04591_amd import ShearletLayer

    _say(f"case: layer 256x256 J=3 K=33 B=32, {forward} forward")
    ref = OF.build_system(256, 256, 3)
    x = synth.cartoon_batch(32, 256, 256, config=4, sigma=0.0)[:, None]
    rng = np.random.default_rng(4)
    g = rng.standard_normal((32, 33, 256, 256)).astype(np.float32)
    layer = ShearletLayer(256, 256, 3)
    assert layer.K == 33
    layer.system.set_schedule(128 if forward == "whole-plane" else 16)
    xt = _to(x, gpu).requires_grad_(True)
    c = layer(xt)
    (c * _to(g, gpu)).sum().backward()
    torch.cuda.synchronize()
    for b in (0, 17, 31):
        assert _rel(xt.grad[b, 0].cpu().numpy(), OT.adjoint_plain(g[b].astype(np.float64), ref.spectra)) <= TOL
        x64 = x[b, 0].astype(np.float64)
        for k in (0, 20, 32):
            want = np.real(np.fft.ifft2(np.fft.fft2(x64) * np.conj(ref.spectra[k])))
            assert np.linalg.norm(c[b, k].detach().cpu().numpy() - want) <= TOL * np.linalg.norm(x64) * ref.rms[k]
    layer.system.close()


def test_layer_energy_gradient(gpu):
    """loss = ||SH x||^2 / 2 has gradient SH* SH x."""
    from paper_2006_04591_amd import ShearletLayer

    _say("case: layer energy gradient 128x128 K=17")
    ref = OF.build_system(128, 128, 2)
    x = synth.cartoon_batch(2, 128, 128, config=1, sigma=5.0)
    layer = ShearletLayer(128, 128, 2)
    xt = _to(x, gpu).requires_grad_(True)
    (0.5 * layer(xt).pow(2).sum()).backward()
    torch.cuda.synchronize()
    for b in range(2):
        x64 = x[b].astype(np.float64)
        want = OT.adjoint_plain(OT.forward_plain(x64, ref.spectra), ref.spectra)
        assert _rel(xt.grad[b].cpu().numpy(), want) <= TOL
    layer.system.close()


def test_layer_shapes_and_no_grad(gpu):
    from paper_2006_04591_amd import ShearletLayer

    layer = ShearletLayer(64, 64, 1, [0])
    x = torch.zeros((2, 64, 64), device=gpu)
    assert layer(x).shape == (2, layer.K, 64, 64)
    with pytest.raises(ValueError):
        layer(torch.zeros((2, 2, 64, 64), device=gpu))
    with torch.no_grad():
        assert not layer(x).requires_grad
    layer.system.close()
