"""GPU parity of the learned-shrinkage network (matrix-core kernels, bfloat16
operands, FP32 accumulation) against the FP64 oracle network.

Tolerance. Both sides round the same operands to bfloat16. The oracle's
values before rounding differ from the GPU's by the FP32 accumulation error
(about 1e-7 relative), so a value that lands within that distance of a
bfloat16 rounding boundary can round to the neighbouring bfloat16 (2^-8
relative) on one side only. Such flips are rare: they change tau by far less
than 1e-3 in relative L2, the bound used here, though a single tau can move by
a few 1e-3. The keep/zero decision compares |z| with the network's own tau, so
where |z| lies within 1e-3 tau of the oracle's tau, or between the GPU's and
the oracle's tau, either decision is valid; elsewhere the decisions must be
equal, and the ambiguous set must stay a small fraction of the coefficients.
"""
import numpy as np
import pytest

import synth
from oracle import apps as OA
from oracle import filters as OF
from oracle import shrink as OS
from oracle import transform as OT

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu
TAU_TOL = 1e-3


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _say(msg):
    print(msg, flush=True)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


def _params_dict(p):
    return {"W1": p.W1, "b1": p.b1, "W2": p.W2, "b2": p.b2, "W3": p.W3, "b3": p.b3}


def _check(got_c, got_t, c32, sigma, rms, p):
    want_c, want_t = OS.shrink(c32.astype(np.float64), sigma, rms, p)
    assert _rel(got_t, want_t) <= TAU_TOL
    z = c32.astype(np.float64) / (sigma * rms[:, None, None])
    az = np.abs(z)
    lo = np.minimum(got_t, want_t) * (1 - 1e-6)
    hi = np.maximum(got_t, want_t) * (1 + 1e-6)
    between = (az >= lo) & (az <= hi)
    clear = (np.abs(az - want_t) > 1e-3 * np.maximum(want_t, 1e-3)) & ~between
    assert clear.mean() > 0.99
    assert np.array_equal(got_c[clear], want_c[clear])
    # inside the band, each output is either the coefficient or zero
    amb = ~clear
    assert np.all((got_c[amb] == c32[amb]) | (got_c[amb] == 0.0))


def _check_decision(got_c, c32, sigma, rms, p, got_c_tau, got_t):
    """The shrink without the threshold output (it decides without forming tau): against the oracle
    where _check's decisions are clear (outside the 1e-3 band around the oracle's tau and not between
    the oracle's tau and the network's own, got_t from the run that writes tau), and against the
    decisions of the run that writes tau outside a 1e-5 band around that run's tau."""
    want_c, want_t = OS.shrink(c32.astype(np.float64), sigma, rms, p)
    az = np.abs(c32.astype(np.float64) / (sigma * rms[:, None, None]))
    lo = np.minimum(got_t, want_t) * (1 - 1e-6)
    hi = np.maximum(got_t, want_t) * (1 + 1e-6)
    between = (az >= lo) & (az <= hi)
    clear = (np.abs(az - want_t) > 1e-3 * np.maximum(want_t, 1e-3)) & ~between
    assert clear.mean() > 0.99
    assert np.array_equal(got_c[clear], want_c[clear])
    assert np.all((got_c[~clear] == c32[~clear]) | (got_c[~clear] == 0.0))
    far = np.abs(az - got_t) > 1e-5 * got_t
    assert np.array_equal(got_c[far], got_c_tau[far])


def test_shrink_matches_oracle_128(gpu):
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink 128x128 K=17 B=2")
    ref = OF.build_system(128, 128, 2)
    sig = np.array([20.0, 35.0])
    x = np.stack([synth.cartoon(128, 128, seed=9100 + b) + synth.gaussian_noise(128, 128, sig[b], seed=9150 + b)
                  for b in range(2)])
    c32 = np.stack([OT.forward_plain(x[b].astype(np.float64), ref.spectra) for b in range(2)]).astype(np.float32)
    p = OS.init_params(ref.K, seed=5, tau0=3.0)
    p.W3 *= 10.0  # thresholds that vary clearly across coefficients
    p = OS.ShrinkParams(p.W1, p.b1, p.W2, p.b2, p.W3, p.b3)
    with ShearletSystem.build(128, 128, 2) as s:
        net = ShrinkNet(s, _params_dict(p))
        out, tau = net.apply(_to(c32, gpu), _to(sig, gpu), tau=True)
        out2 = net.apply(_to(c32, gpu), _to(sig, gpu))
        torch.cuda.synchronize()
        for b in range(2):
            _check(out[b].cpu().numpy(), tau[b].cpu().numpy(), c32[b], sig[b], ref.rms, p)
            _check_decision(out2[b].cpu().numpy(), c32[b], sig[b], ref.rms, p, out[b].cpu().numpy(),
                            tau[b].cpu().numpy())
        assert float(tau[:, :-1].std()) > 0.1  # the network's thresholds do vary


def test_untrained_shrink_is_hard_threshold(gpu):
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: untrained shrink = hard threshold 3 sigma RMS")
    ref = OF.build_system(128, 128, 2)
    x = synth.cartoon_batch(3, 128, 128, config=9, sigma=25.0)
    c32 = np.stack([OT.forward_plain(x[b].astype(np.float64), ref.spectra) for b in range(3)]).astype(np.float32)
    p = OS.init_params(ref.K, seed=6, tau0=3.0)
    p.W3[:] = 0.0
    with ShearletSystem.build(128, 128, 2) as s:
        net = ShrinkNet(s, _params_dict(p))
        out = net.apply(_to(c32, gpu), 25.0)
        torch.cuda.synchronize()
        delta = 3.0 * 25.0 * ref.rms
        delta[-1] = 0.0
        for b in range(3):
            want = OA.hard_threshold(c32[b].astype(np.float64), delta)
            near = np.abs(np.abs(c32[b]) - delta[:, None, None]) <= 1e-5 * delta[:, None, None]
            got = out[b].cpu().numpy()
            assert np.array_equal(got[~near], want[~near])


def test_shrink_tile_borders_user_bank(gpu):
    """A 64x128 user bank (K=5): tiles of 8x32 pixels with wrapped halos on every side."""
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink 64x128 K=5 B=3")
    rng = np.random.default_rng(12)
    S = np.fft.fft2(rng.standard_normal((5, 64, 128)))
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
    c32 = (rng.standard_normal((3, 5, 64, 128)) * 30.0 * rms[None, :, None, None]).astype(np.float32)
    sig = np.array([10.0, 30.0, 50.0])
    p = OS.init_params(5, seed=7, tau0=2.0)
    p.W3 *= 10.0
    p = OS.ShrinkParams(p.W1, p.b1 + 0.1, p.W2, p.b2 - 0.05, p.W3, p.b3)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        assert np.allclose(s.rms, rms, rtol=1e-12)
        net = ShrinkNet(s, _params_dict(p))
        out, tau = net.apply(_to(c32, gpu), _to(sig, gpu), tau=True)
        out2 = net.apply(_to(c32, gpu), _to(sig, gpu))
        torch.cuda.synchronize()
        for b in range(3):
            _check(out[b].cpu().numpy(), tau[b].cpu().numpy(), c32[b], sig[b], rms, p)
            _check_decision(out2[b].cpu().numpy(), c32[b], sig[b], rms, p, out[b].cpu().numpy(), tau[b].cpu().numpy())


def test_shrink_uneven_tile_ranges(gpu):
    """16 x 128 planes, B=3, K=5: the first layer's 12 tiles of 8 x 64 pixels split into 8 per-XCD
    ranges of one or two tiles, most blocks of its one-per-CU grid without a tile."""
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink 16x128 K=5 B=3 (uneven tile ranges)")
    rng = np.random.default_rng(14)
    S = np.fft.fft2(rng.standard_normal((5, 16, 128)))
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
    c32 = (rng.standard_normal((3, 5, 16, 128)) * 30.0 * rms[None, :, None, None]).astype(np.float32)
    sig = np.array([12.0, 25.0, 45.0])
    p = OS.init_params(5, seed=9, tau0=2.0)
    p.W3 *= 10.0
    p = OS.ShrinkParams(p.W1, p.b1 + 0.1, p.W2, p.b2 - 0.05, p.W3, p.b3)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        net = ShrinkNet(s, _params_dict(p))
        out, tau = net.apply(_to(c32, gpu), _to(sig, gpu), tau=True)
        out2 = net.apply(_to(c32, gpu), _to(sig, gpu))
        torch.cuda.synchronize()
        for b in range(3):
            _check(out[b].cpu().numpy(), tau[b].cpu().numpy(), c32[b], sig[b], rms, p)
            _check_decision(out2[b].cpu().numpy(), c32[b], sig[b], rms, p, out[b].cpu().numpy(), tau[b].cpu().numpy())


def test_shrink_sliding_window_strips(gpu):
    """512 x 256 planes, B=3, K=49 (user bank): 768 first-layer tiles of 8 x 64 pixels, so each
    block of the one-per-CU grid walks a chunk of about three tiles down a 64-column strip (the
    staged rows moved up in LDS, 8 new rows loaded), some chunks crossing from the bottom of one
    strip to the top of the next; image 0 against the oracle, both shrink epilogues."""
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say("case: shrink 512x256 K=49 B=3 (sliding window across strips)")
    rng = np.random.default_rng(15)
    K, N, M = 49, 512, 256
    S = np.fft.fft2(rng.standard_normal((K, N, M)))
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
    c32 = (rng.standard_normal((3, K, N, M)) * 30.0 * rms[None, :, None, None]).astype(np.float32)
    sig = np.array([20.0, 35.0, 15.0])
    p = OS.init_params(K, seed=11, tau0=2.0)
    p.W3 *= 10.0
    p = OS.ShrinkParams(p.W1, p.b1 + 0.1, p.W2, p.b2 - 0.05, p.W3, p.b3)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        net = ShrinkNet(s, _params_dict(p))
        out, tau = net.apply(_to(c32, gpu), _to(sig, gpu), tau=True)
        out2 = net.apply(_to(c32, gpu), _to(sig, gpu))
        torch.cuda.synchronize()
        _check(out[0].cpu().numpy(), tau[0].cpu().numpy(), c32[0], sig[0], rms, p)
        _check_decision(out2[0].cpu().numpy(), c32[0], sig[0], rms, p, out[0].cpu().numpy(), tau[0].cpu().numpy())
        # the other images: both epilogues decide alike away from the thresholds
        for b in (1, 2):
            az = np.abs(c32[b].astype(np.float64) / (sig[b] * rms[:, None, None]))
            t = tau[b].cpu().numpy()
            far = np.abs(az - t) > 1e-5 * t
            assert np.array_equal(out2[b].cpu().numpy()[far], out[b].cpu().numpy()[far])


def test_shrink_errors(gpu):
    from paper_2006_04591_amd import ShearError, ShearletSystem, ShrinkNet

    rng = np.random.default_rng(13)
    S = np.fft.fftshift(np.fft.fft2(rng.standard_normal((2, 16, 16))), axes=(1, 2))
    p = OS.init_params(2, seed=1)
    with ShearletSystem.from_spectra(S) as s:
        net = ShrinkNet(s, _params_dict(p))
        with pytest.raises(ShearError) as e:
            net.apply(_to(np.zeros((1, 2, 16, 16)), gpu), 1.0)  # 16 columns: not a multiple of 128
        assert e.value.name == "SHEAR_E_SIZE"
        with pytest.raises(ValueError):
            ShrinkNet(s, {**_params_dict(p), "W1": np.zeros((32, 3, 3, 3))})


@pytest.mark.parametrize("K", [33, 48, 64])
def test_shrink_wide_channel_counts(gpu, K):
    """K above 32 (user banks, 64x128, B=2): layer 1 stages its 64 padded input channels in two
    parts, and the shrink layer covers 48 padded output channels in three passes of 16, 64 in two
    of 32."""
    from paper_2006_04591_amd import ShearletSystem, ShrinkNet

    _say(f"case: shrink 64x128 K={K} B=2")
    rng = np.random.default_rng(100 + K)
    S = np.fft.fft2(rng.standard_normal((K, 64, 128)))
    rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
    c32 = (rng.standard_normal((2, K, 64, 128)) * 30.0 * rms[None, :, None, None]).astype(np.float32)
    sig = np.array([15.0, 40.0])
    p = OS.init_params(K, seed=K, tau0=2.0)
    p.W3 *= 10.0
    p = OS.ShrinkParams(p.W1, p.b1 + 0.1, p.W2, p.b2 - 0.05, p.W3, p.b3)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        net = ShrinkNet(s, _params_dict(p))
        out, tau = net.apply(_to(c32, gpu), _to(sig, gpu), tau=True)
        out2 = net.apply(_to(c32, gpu), _to(sig, gpu))
        torch.cuda.synchronize()
        for b in range(2):
            _check(out[b].cpu().numpy(), tau[b].cpu().numpy(), c32[b], sig[b], rms, p)
            _check_decision(out2[b].cpu().numpy(), c32[b], sig[b], rms, p, out[b].cpu().numpy(), tau[b].cpu().numpy())
