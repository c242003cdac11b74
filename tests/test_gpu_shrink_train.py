"""GPU parity of one training step of the shrinkage network (matrix-core
forward, loss epilogue, backward-data and weight-gradient kernels) against the
oracle's analytic gradients (bfloat16 rounding at the same points; the oracle's
gradients are pinned by FP64 finite differences). Gradients are compared in
relative L2 per parameter tensor, the loss within 1e-3 relative. Both sides
round to bfloat16 at the same points, so what differs is FP32 against FP64
accumulation and the values that round to a different bfloat16 because of
it; those flips pass down the backward chain. Measured over seeds and
channel counts: W3, b3 and W2 within 3e-4 everywhere; W1 2.5e-4 at 17
filters and 3e-4 to 1.9e-3 at 56-64 filters, varying with the data (seed
to seed at one channel count) and evenly spread over W1's input and output
channels, as rounding flips are and a wrong channel would not be. Bars:
1e-3 at 17 filters, 3e-3 for the wide channel counts; a 1 % error of scale
in any gradient fails either."""
import numpy as np
import pytest

import synth
from oracle import filters as OF
from oracle import shrink as OS
from oracle import transform as OT

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(msg):
    print(msg, flush=True)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def _pairs(ref, B, N, seed, sig):
    clean = np.stack([synth.cartoon(N, N, seed=seed + b) for b in range(B)]).astype(np.float64)
    noisy = np.stack([clean[b] + synth.gaussian_noise(N, N, sig[b], seed=seed + 50 + b) for b in range(B)])
    cc = np.stack([OT.forward_plain(clean[b], ref.spectra) for b in range(B)]).astype(np.float32)
    cn = np.stack([OT.forward_plain(noisy[b], ref.spectra) for b in range(B)]).astype(np.float32)
    return cn, cc


def _net_params(K, seed):
    p = OS.init_params(K, seed=seed, tau0=2.5)
    rng = np.random.default_rng(seed + 1)
    p = OS.ShrinkParams(p.W1, p.b1 + 0.05 * rng.standard_normal(32), p.W2, p.b2 + 0.05 * rng.standard_normal(32),
                        p.W3 * 10.0, p.b3)
    return p


def test_train_step_gradients_match_oracle(gpu):
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink training gradients 128x128 K=17 B=2")
    ref = OF.build_system(128, 128, 2)
    sig = np.array([15.0, 30.0])
    cn, cc = _pairs(ref, 2, 128, 9300, sig)
    p = _net_params(ref.K, 31)
    T = 0.5
    scale = 1.0 / (2 * (ref.K - 1) * 128 * 128)
    L = 0.0
    want = {n: 0.0 for n in ("W1", "b1", "W2", "b2", "W3", "b3")}
    for b in range(2):
        Lb, gb = OS.train_loss(cn[b], cc[b], sig[b], ref.rms, p, T, scale, rounded=True)
        L += Lb
        for n in want:
            want[n] = want[n] + gb[n]
    with ShearletSystem.build(128, 128, 2) as s:
        net = ShrinkNet(s, {n: getattr(p, n) for n in ShrinkNet.NAMES})
        before = net.flat.clone()
        loss = net.train_step(_to(cn, gpu), _to(cc, gpu), _to(sig, gpu), lr=0.0, temperature=T)
        torch.cuda.synchronize()
        assert torch.equal(net.flat, before)  # a zero rate leaves the parameters alone
        assert abs(float(loss) - L) <= 1e-3 * L
        for n in want:
            e = _rel(net.grad(n).cpu().numpy(), want[n])
            print(f"grad {n}: rel L2 {e:.2e}")
            assert e <= 1e-3, n


def test_training_reduces_loss(gpu):
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink training, 40 Adam steps on a fixed batch")
    ref = OF.build_system(128, 128, 2)
    sig = np.array([20.0, 40.0, 30.0])
    cn, cc = _pairs(ref, 3, 128, 9400, sig)
    p = OS.init_params(ref.K, seed=41, tau0=3.0)
    with ShearletSystem.build(128, 128, 2) as s:
        net = ShrinkNet(s, {n: getattr(p, n) for n in ShrinkNet.NAMES})
        a, b, sg = _to(cn, gpu), _to(cc, gpu), _to(sig, gpu)
        losses = [float(net.train_step(a, b, sg, lr=2e-3)) for _ in range(40)]
        torch.cuda.synchronize()
        assert all(np.isfinite(losses))
        assert losses[-1] < 0.9 * losses[0]
        # the trained network shrinks the noisy coefficients closer to the clean ones than it did at the start
        p0 = OS.init_params(ref.K, seed=41, tau0=3.0)
        start = ShrinkNet(s, {n: getattr(p0, n) for n in ShrinkNet.NAMES})
        e1 = float(((net.apply(a, sg) - b) ** 2).sum())
        e0 = float(((start.apply(a, sg) - b) ** 2).sum())
        assert e1 < e0


@pytest.mark.parametrize("K", [40, 64])
def test_train_step_gradients_wide_channel_counts(gpu, K):
    """K above 32 (user banks, 64x128, B=2): 64 padded input channels of layer 1 (two staging
    parts in the forward and in the backward data of the last layer, 64-channel weight
    gradients) and 48 or 64 padded output channels of the last layer."""
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say(f"case: shrink training gradients 64x128 K={K} B=2")
    rng = np.random.default_rng(200 + K)
    S = np.fft.fft2(rng.standard_normal((K, 64, 128)))
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
    sig = np.array([20.0, 35.0])
    cc = (rng.standard_normal((2, K, 64, 128)) * 20.0 * rms[None, :, None, None]).astype(np.float32)
    cn = (cc + rng.standard_normal(cc.shape) * sig[:, None, None, None] * rms[None, :, None, None]).astype(np.float32)
    p = _net_params(K, 50 + K)
    T = 0.5
    scale = 1.0 / (2 * (K - 1) * 64 * 128)
    L = 0.0
    want = {n: 0.0 for n in ("W1", "b1", "W2", "b2", "W3", "b3")}
    for b in range(2):
        Lb, gb = OS.train_loss(cn[b], cc[b], sig[b], rms, p, T, scale, rounded=True)
        L += Lb
        for n in want:
            want[n] = want[n] + gb[n]
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        net = ShrinkNet(s, {n: getattr(p, n) for n in ShrinkNet.NAMES})
        loss = net.train_step(_to(cn, gpu), _to(cc, gpu), _to(sig, gpu), lr=0.0, temperature=T)
        torch.cuda.synchronize()
        assert abs(float(loss) - L) <= 1e-3 * L
        for n in want:
            e = _rel(net.grad(n).cpu().numpy(), want[n])
            print(f"grad {n}: rel L2 {e:.2e}")
            assert e <= 3e-3, n
