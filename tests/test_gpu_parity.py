"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded and shared (synth); the oracle never sees a GPU output.
Bar: relative L2 error <= 1e-5 (FP32 path vs FP64 oracle), also per plane
normalised by ||x|| * RMS_k.
"""
import ctypes

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


@pytest.fixture(scope="module")
def lib():
    from paper_2006_04591_amd import load_library

    return load_library()


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


# ---------------------------------------------------------------- 128x128, 17 filters (one image, FP64 workload at FP32)


@pytest.fixture(scope="module")
def cfg1(gpu, lib):
    from paper_2006_04591_amd import ShearletSystem

    _say("case: build 128x128 J=2 (K=17)")
    s = ShearletSystem.build(128, 128, 2)
    ref = OF.build_system(128, 128, 2)
    x = synth.cartoon(128, 128, synth.seed_image(1, 0))
    yield s, ref, x
    s.close()


def test_system_matches_oracle_spectra(cfg1):
    s, ref, _ = cfg1
    S, W = s.export_spectra()
    assert np.max(np.abs(S - ref.centred)) <= 1e-12 * np.max(np.abs(ref.centred))
    assert np.max(np.abs(W - np.fft.fftshift(ref.W))) <= 1e-12 * ref.W.max()
    assert np.allclose(s.rms, ref.rms, rtol=1e-12)
    assert np.array_equal(s.idx, ref.idx)


def test_forward_config1(cfg1, gpu):
    s, ref, x = cfg1
    _say("case: forward 128x128 K=17 B=1")
    c = s.forward(_to(x[None], gpu))
    torch.cuda.synchronize()
    got = c[0].double().cpu().numpy()
    want = OT.forward_plain(x.astype(np.float64), ref.spectra)
    assert _rel(got, want) <= TOL
    nx = np.linalg.norm(x.astype(np.float64))
    per = [np.linalg.norm(got[k] - want[k]) / (nx * ref.rms[k]) for k in range(ref.K)]
    assert max(per) <= TOL


def test_inverse_and_adjoint_config1(cfg1, gpu):
    s, ref, x = cfg1
    c_in = OT.forward_plain(x.astype(np.float64), ref.spectra).astype(np.float32)
    _say("case: inverse/adjoint 128x128 K=17 B=1")
    cg = _to(c_in[None], gpu)
    y = s.inverse(cg)
    a = s.adjoint(cg)
    torch.cuda.synchronize()
    cb = c_in.astype(np.float64)
    assert _rel(y[0].cpu().numpy(), OT.inverse_plain(cb, ref.spectra, ref.W)) <= TOL
    assert _rel(a[0].cpu().numpy(), OT.adjoint_plain(cb, ref.spectra)) <= TOL


def test_adjoint_random_coefficients(cfg1, gpu):
    s, ref, _ = cfg1
    rng = np.random.default_rng(11)
    c_in = rng.standard_normal((2, ref.K, 128, 128)).astype(np.float32)
    _say("case: adjoint 128x128 K=17 B=2 random coefficients")
    a = s.adjoint(_to(c_in, gpu))
    torch.cuda.synchronize()
    for b in range(2):
        assert _rel(a[b].cpu().numpy(), OT.adjoint_plain(c_in[b].astype(np.float64), ref.spectra)) <= TOL


def test_perfect_reconstruction_gpu(cfg1, gpu):
    s, _, x = cfg1
    _say("case: PR chain 128x128 K=17")
    xg = _to(x[None], gpu)
    y = s.inverse(s.forward(xg))
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), x[None]) <= TOL


def test_deterministic(cfg1, gpu):
    s, _, x = cfg1
    _say("case: determinism 128x128")
    xg = _to(np.stack([x, x[::-1].copy()]), gpu)
    a = s.forward(xg).clone()
    b = s.forward(xg)
    ya = s.inverse(a).clone()
    yb = s.inverse(b)
    torch.cuda.synchronize()
    assert torch.equal(a, b) and torch.equal(ya, yb)


# ---------------------------------------------------------------- small and ragged shapes, user filter banks


def _random_bank(rng, K, N, M, real):
    ker = rng.standard_normal((K, N, M))
    if real:  # centro-symmetric kernels -> real spectra
        ker = ker + ker[:, (-np.arange(N)) % N][:, :, (-np.arange(M)) % M]
    S = np.fft.fft2(ker)
    return S


@pytest.mark.parametrize("N,M,K,real,B", [(16, 16, 3, False, 1), (32, 64, 5, True, 3), (64, 16, 4, False, 2),
                                          (128, 32, 7, True, 5), (16, 1024, 2, False, 1), (1024, 16, 2, True, 1),
                                          (32, 1024, 5, True, 3), (2048, 2048, 2, True, 1), (2048, 32, 3, False, 2),
                                          (16, 2048, 4, True, 3)])
def test_user_bank_shapes(gpu, lib, N, M, K, real, B):
    """User filter banks of assorted shapes against the oracle. At 1024 columns the row passes run
    8-row blocks whose two halves of a 16-row tile are regrouped per 16 blocks: 32 x 1024 with 15
    coefficient planes gives 60 blocks per pass (48 regrouped, a tail of 12 in order). 2048-point
    columns are 128-thread FFT groups over two wavefronts (workgroup barriers between passes);
    2048-point rows are 1024-point half-length FFTs of 16 points per thread."""
    from paper_2006_04591_amd import ShearletSystem

    rng = np.random.default_rng(N * 7 + M + K)
    S = _random_bank(rng, K, N, M, real)
    W = np.sum(np.abs(S) ** 2, 0)
    x = rng.standard_normal((B, N, M)).astype(np.float32)
    c_in = rng.standard_normal((B, K, N, M)).astype(np.float32)
    _say(f"case: user bank N={N} M={M} K={K} real={real} B={B}")
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        c = s.forward(_to(x, gpu))
        cg = _to(c_in, gpu)
        y = s.inverse(cg)
        a = s.adjoint(cg)
        torch.cuda.synchronize()
        for b in range(B):
            assert _rel(c[b].cpu().numpy(), OT.forward_plain(x[b].astype(np.float64), S)) <= TOL
            assert _rel(y[b].cpu().numpy(), OT.inverse_plain(c_in[b].astype(np.float64), S, W)) <= TOL
            assert _rel(a[b].cpu().numpy(), OT.adjoint_plain(c_in[b].astype(np.float64), S)) <= TOL


def test_chunked_equals_unchunked(gpu, lib):
    from paper_2006_04591_amd import ShearletSystem

    rng = np.random.default_rng(5)
    N, M, K, B = 64, 128, 6, 5
    S = _random_bank(rng, K, N, M, True)
    Sc = np.fft.fftshift(S, axes=(1, 2))
    x = _to(rng.standard_normal((B, N, M)), gpu)
    one_image = B * N * (M // 2) * 8 + K * N * (M // 2) * 8
    _say("case: chunked vs unchunked 64x128 K=6 B=5")
    with ShearletSystem.from_spectra(Sc) as big, ShearletSystem.from_spectra(Sc, max_workspace_bytes=one_image + 1024) as small:
        assert small.workspace_bytes(B) == one_image
        c1 = big.forward(x)
        c2 = small.forward(x)
        y1 = big.inverse(c1)
        y2 = small.inverse(c1)
        torch.cuda.synchronize()
        assert torch.equal(c1, c2) and torch.equal(y1, y2)


def test_non_default_stream(cfg1, gpu):
    s, ref, x = cfg1
    _say("case: forward on a side stream")
    st = torch.cuda.Stream()
    xg = _to(x[None], gpu)
    torch.cuda.synchronize()
    with torch.cuda.stream(st):
        c = s.forward(xg)
    st.synchronize()
    assert _rel(c[0].cpu().numpy(), OT.forward_plain(x.astype(np.float64), ref.spectra)) <= TOL


def test_profile_counts(cfg1, gpu):
    s, _, x = cfg1
    _say("case: per-launch timing")
    xg = _to(x[None], gpu)
    s.profile(True)
    c = s.forward(xg)
    s.inverse(c)
    rec = s.profile_read()
    s.profile(False)
    assert rec["rows_r2c_images"][0] == 1 and rec["cols_fwd"][0] == 1 and rec["rows_c2r_coeffs"][0] == 1
    assert rec["rows_r2c_coeffs"][0] == 1 and rec["cols_inv"][0] == 1 and rec["rows_c2r_images"][0] == 1
    assert all(v[1] > 0 for v in rec.values() if v[0] > 0)


def test_errors(gpu, lib):
    from paper_2006_04591_amd import ShearError, ShearletSystem

    _say("case: error paths")
    with pytest.raises(ShearError) as e:
        ShearletSystem.build(4096, 4096, 4)
    assert e.value.name == "SHEAR_E_SIZE"
    with pytest.raises(ShearError) as e:
        ShearletSystem.build(32, 32, 2)  # kernels do not fit
    assert e.value.name == "SHEAR_E_SIZE"
    with pytest.raises(ShearError) as e:
        ShearletSystem.from_spectra(np.zeros((2, 16, 16), complex))
    assert e.value.name == "SHEAR_E_FRAME"
    rng = np.random.default_rng(1)
    bad = rng.standard_normal((2, 16, 16)) + 1j * rng.standard_normal((2, 16, 16))
    with pytest.raises(ShearError) as e:
        ShearletSystem.from_spectra(bad)
    assert e.value.name == "SHEAR_E_FRAME"
    S = np.fft.fftshift(np.fft.fft2(rng.standard_normal((2, 16, 16))), axes=(1, 2))
    with ShearletSystem.from_spectra(S, max_workspace_bytes=1000) as s:
        with pytest.raises(ShearError) as e:
            s.forward(_to(np.zeros((1, 16, 16)), gpu))
        assert e.value.name == "SHEAR_E_NOMEM"
        with pytest.raises(ValueError):
            s.forward(_to(np.zeros((1, 16, 8)), gpu))


def test_empty_and_negative_batches(cfg1, gpu, lib):
    """batch == 0 is an empty call: SHEAR_OK, nothing launched, no pointer read (NULL is fine); a
    negative batch is SHEAR_E_INVALID, as is batch == 0 where a size is being asked for (reserve,
    workspace size). The binding turns empty tensors into empty results."""
    from paper_2006_04591_amd import ShearError

    s, ref, x = cfg1
    _say("case: empty and negative batches")
    xb = _to(x[None], gpu)
    c_before = s.forward(xb)
    torch.cuda.synchronize()
    h = s._h
    assert lib.shear_forward(h, None, None, 0, None) == 0
    assert lib.shear_inverse(h, None, None, 0, None) == 0
    assert lib.shear_adjoint(h, None, None, 0, None) == 0
    assert lib.shear_denoise(h, None, None, 0, None, None, None) == 0
    assert lib.shear_inpaint(h, None, None, None, 0, None, 0, None) == 0
    assert lib.shear_shrink_apply(h, None, None, None, 0, None, None, None) == 0
    xp, cp = ctypes.c_void_p(xb.data_ptr()), ctypes.c_void_p(c_before.data_ptr())
    assert lib.shear_forward(h, xp, cp, -1, None) == -1
    assert lib.shear_inverse(h, cp, xp, -1, None) == -1
    assert lib.shear_forward(None, None, None, 0, None) == -1
    for fn in (s.reserve, s.workspace_bytes):
        with pytest.raises(ShearError) as e:
            fn(0)
        assert e.value.name == "SHEAR_E_INVALID"
    e0 = torch.empty((0, 128, 128), dtype=torch.float32, device=gpu)
    c = s.forward(e0)
    assert tuple(c.shape) == (0, ref.K, 128, 128)
    assert tuple(s.inverse(c).shape) == (0, 128, 128) and tuple(s.adjoint(c).shape) == (0, 128, 128)
    y, kept = s.denoise(e0, s.paper_thresholds(20.0), kept=True)
    assert tuple(y.shape) == (0, 128, 128) and tuple(kept.shape) == (0, ref.K)
    f = s.inpaint(e0, e0, np.zeros((3, 0, ref.K), np.float32))
    assert tuple(f.shape) == (0, 128, 128)
    # the empty calls left the system as it was
    c_after = s.forward(xb)
    torch.cuda.synchronize()
    assert torch.equal(c_before, c_after)


# ---------------------------------------------------------------- full-size workloads, sampled against the oracle


def _plane_forward(x64, S_k):
    return np.real(np.fft.ifft2(np.fft.fft2(x64) * np.conj(S_k)))


@pytest.fixture(scope="module")
def cfg2(gpu, lib):
    from paper_2006_04591_amd import ShearletSystem

    _say("case: build 512x512 J=4 (K=49)")
    s = ShearletSystem.build(512, 512, 4)
    ref = OF.build_system(512, 512, 4)
    yield s, ref
    s.close()


@pytest.fixture(scope="module")
def cfg2_oracle(cfg2):
    """The headline workload through the oracle, computed once: 16 noisy 512x512 cartoons (sigma 30),
    their FP64 coefficients for all 49 filters rounded to float32 (822 MB; the rounding, ~6e-8
    relative, is far below the bar), and the oracle's inverse and adjoint of those float32
    coefficients for all 16 images."""
    _, ref = cfg2
    _say("case: oracle of 16 x 512x512 x 49 (forward, inverse, adjoint)")
    x = synth.cartoon_batch(16, 512, 512, config=2, sigma=30.0)
    c32 = np.empty((16, 49, 512, 512), np.float32)
    y_ref = np.empty((16, 512, 512))
    a_ref = np.empty((16, 512, 512))
    for b in range(16):
        c32[b] = OT.forward_plain(x[b].astype(np.float64), ref.spectra)
        Sb = np.sum(np.fft.fft2(c32[b].astype(np.float64)) * ref.spectra, axis=0)
        y_ref[b] = np.real(np.fft.ifft2(Sb / ref.W))
        a_ref[b] = np.real(np.fft.ifft2(Sb))
    return x, c32, y_ref, a_ref


@pytest.mark.parametrize("schedule", ["autotuned", "fixed"])
def test_512_k49_b16_whole_tensor(cfg2, cfg2_oracle, gpu, schedule):
    """The headline configuration, whole tensors against the oracle: relative L2 over all 16 x 49
    forward planes and over all 16 inverse and adjoint images <= 1e-5, under the schedule the
    autotuner picks for this batch (as the throughput runs use) and under a fixed one. Per plane,
    the error is also bounded by 1e-5 ||x|| RMS_k (fine-scale planes carry little energy)."""
    s, ref = cfg2
    x, c32, y_ref, a_ref = cfg2_oracle
    sched = s.autotune(16) if schedule == "autotuned" else (16, 16, 1, 1)
    if schedule == "fixed":
        s.set_schedule(*sched)
    _say(f"case: 512x512 K=49 B=16 whole tensor, {schedule} schedule {sched}")
    c = s.forward(_to(x, gpu))
    y = s.inverse(_to(c32, gpu))
    a = s.adjoint(_to(c32, gpu))
    torch.cuda.synchronize()
    num = den = 0.0
    worst = 0.0
    for b in range(16):
        got = c[b].double().cpu().numpy()
        want = c32[b].astype(np.float64)
        d2 = np.sum((got - want) ** 2, axis=(1, 2))
        num += float(d2.sum())
        den += float(np.sum(want ** 2))
        worst = max(worst, float(np.max(np.sqrt(d2) / (np.linalg.norm(x[b].astype(np.float64)) * ref.rms))))
    fwd = float(np.sqrt(num / den))
    inv = _rel(y.cpu().numpy(), y_ref)
    adj = _rel(a.cpu().numpy(), a_ref)
    print(f"forward {fwd:.2e} (worst plane / (||x|| RMS_k) {worst:.2e}), inverse {inv:.2e}, adjoint {adj:.2e}")
    assert fwd <= TOL and worst <= TOL and inv <= TOL and adj <= TOL
    # perfect reconstruction of the timed chain, whole batch
    yr = s.inverse(c)
    torch.cuda.synchronize()
    assert _rel(yr.cpu().numpy(), x) <= TOL
    s.autotune(16)


def test_edge_cases_constant_and_impulse(cfg1, cfg2, gpu):
    """The method's degenerate inputs (SURVEY's pins, run on the GPU): a constant image has vanishing
    band-pass planes and a low-pass plane equal to the constant (Psi_lowpass(0) = 1); an impulse at the
    origin returns every filter's reflected kernel; both reconstruct exactly."""
    for (s, ref), N in (((cfg1[0], cfg1[1]), 128), (cfg2, 512)):
        _say(f"case: constant and impulse images {N}x{N} K={ref.K}")
        const = np.full((N, N), 77.0, np.float32)
        imp = np.zeros((N, N), np.float32)
        imp[0, 0] = 1000.0
        xs = np.stack([const, imp])
        c = s.forward(_to(xs, gpu))
        y = s.inverse(c)
        torch.cuda.synchronize()
        cc = c[0].double().cpu().numpy()
        nx = np.linalg.norm(const.astype(np.float64))
        for k in range(ref.K - 1):
            assert np.linalg.norm(cc[k]) <= TOL * nx * ref.rms[k], k
        assert _rel(cc[-1], np.full((N, N), 77.0)) <= TOL
        ci = c[1].double().cpu().numpy()
        want = 1000.0 * np.real(np.fft.ifft2(np.conj(ref.spectra)))  # c_k[n] = 1000 h_k[-n]
        assert _rel(ci, want) <= TOL
        # the kernels are centro-symmetric: the reflection is the kernel itself
        assert _rel(ci, 1000.0 * np.real(np.fft.ifft2(ref.spectra))) <= TOL
        assert _rel(y.cpu().numpy(), xs) <= TOL


@pytest.mark.parametrize("N,M", [(512, 512), (64, 128), (1024, 32)])
def test_identity_bank(gpu, lib, N, M):
    """A single all-pass filter (Psi = 1): W = 1, the forward transform is the identity (an FFT round
    trip), and so are the inverse and the adjoint."""
    from paper_2006_04591_amd import ShearletSystem

    _say(f"case: identity bank {N}x{M}")
    x = synth.cartoon_batch(3, N, M, config=8, sigma=5.0)
    with ShearletSystem.from_spectra(np.ones((1, N, M), complex)) as s:
        c = s.forward(_to(x, gpu))
        y = s.inverse(c)
        a = s.adjoint(_to(x[:, None], gpu))
        torch.cuda.synchronize()
        assert _rel(c[:, 0].cpu().numpy(), x) <= TOL
        assert _rel(y.cpu().numpy(), x) <= TOL
        assert _rel(a.cpu().numpy(), x) <= TOL


def test_forward_inverse_1024_k49_whole_tensor(gpu, lib):
    """1024 x 1024, 49 filters, two images: the 1024-point column FFTs (16 points per thread) and the
    8-row XCD-paired row tiles of 1024 columns, whole tensors against the oracle."""
    from paper_2006_04591_amd import ShearletSystem

    _say("case: 1024x1024 K=49 B=2 whole tensor")
    ref = OF.build_system(1024, 1024, 4)
    x = synth.cartoon_batch(2, 1024, 1024, config=3, sigma=20.0)
    with ShearletSystem.build(1024, 1024, 4) as s:
        c = s.forward(_to(x, gpu))
        torch.cuda.synchronize()
        num = den = 0.0
        c32 = np.empty((2, 49, 1024, 1024), np.float32)
        for b in range(2):
            want = OT.forward_plain(x[b].astype(np.float64), ref.spectra)
            got = c[b].double().cpu().numpy()
            num += float(np.sum((got - want) ** 2))
            den += float(np.sum(want ** 2))
            c32[b] = want
        assert np.sqrt(num / den) <= TOL
        y = s.inverse(_to(c32, gpu))
        a = s.adjoint(_to(c32, gpu))
        torch.cuda.synchronize()
        for b in range(2):
            cb = c32[b].astype(np.float64)
            assert _rel(y[b].cpu().numpy(), OT.inverse_plain(cb, ref.spectra, ref.W)) <= TOL
            assert _rel(a[b].cpu().numpy(), OT.adjoint_plain(cb, ref.spectra)) <= TOL


def test_config4_256_k33_b32_sampled(gpu, lib):
    from paper_2006_04591_amd import ShearletSystem

    _say("case: 256x256 K=33 B=32 forward + adjoint")
    ref = OF.build_system(256, 256, 3)
    with ShearletSystem.build(256, 256, 3) as s:
        x = synth.cartoon_batch(32, 256, 256, config=4)
        rng = np.random.default_rng(4)
        g = rng.standard_normal((32, 33, 256, 256)).astype(np.float32)
        c = s.forward(_to(x, gpu))
        a = s.adjoint(_to(g, gpu))
        torch.cuda.synchronize()
        for b in (0, 31):
            x64 = x[b].astype(np.float64)
            for k in (0, 16, 32):
                want = _plane_forward(x64, ref.spectra[k])
                assert np.linalg.norm(c[b, k].double().cpu().numpy() - want) <= TOL * np.linalg.norm(x64) * ref.rms[k]
            assert _rel(a[b].cpu().numpy(), OT.adjoint_plain(g[b].astype(np.float64), ref.spectra)) <= TOL


# ---------------------------------------------------------------- column-pass schedules and the autotuner


@pytest.mark.parametrize("N,M,J,B", [(256, 256, 3, 4), (1024, 1024, 4, 2), (512, 128, 2, 3), (512, 512, 4, 1)])
def test_schedules_agree_and_autotune(gpu, lib, N, M, J, B):
    """Every column-pass schedule transforms each column and filter with the same operations at given
    points per thread: across panel widths and filter groups the forward is bitwise identical; the
    inverse sums the filters group by group, so it agrees to rounding. The other points per thread (a
    different radix sequence: 16 at 256 and 512 points, 8 at 1024) agree to rounding and with the
    oracle. The autotuner keeps one of them."""
    from paper_2006_04591_amd import ShearletSystem

    _say(f"case: schedules {N}x{M} J={J} B={B}")
    ref = OF.build_system(N, M, J)
    alt = {256: 16, 512: 16, 1024: 8}[N]
    dflt = {256: 8, 512: 8, 1024: 16}[N]
    with ShearletSystem.build(N, M, J) as s:
        xh = synth.cartoon_batch(B, N, M, config=8, sigma=5.0)
        x = _to(xh, gpu)
        res = {}
        for pc in (dflt, alt):
            for pw in (16, 8):
                for kg in (1, 3, 8, 16):
                    s.set_schedule(pw, pw, kg, kg, pc, pc)
                    c = s.forward(x)
                    res[(pc, pw, kg)] = (c, s.inverse(c), s.adjoint(c))
        torch.cuda.synchronize()
        c0, y0, a0 = res[(dflt, 16, 1)]

        def eff(pc, pw):  # at 1024 points the alternative needs 8-column blocks (16 x 128 threads is too many)
            return dflt if (N == 1024 and pw == 16) else pc

        ref_alt = res[(alt, 8, 1)][0]
        for key, (c, y, a) in res.items():
            if eff(key[0], key[1]) == dflt:
                assert torch.equal(c, c0), key
            else:
                assert torch.equal(c, ref_alt), key
                assert _rel(c.cpu().numpy(), c0.cpu().numpy()) <= 1e-6, key
            assert _rel(y.cpu().numpy(), y0.cpu().numpy()) <= 1e-6, key
            assert _rel(a.cpu().numpy(), a0.cpu().numpy()) <= 1e-6, key
        # the split inverse and the alternative radix sequence against the oracle (one image)
        for key in ((dflt, 8, 8), (alt, 8, 8), (alt, 8, 1)):
            yk = res[key][1][0].double().cpu().numpy()
            c_in = res[key][0][0].double().cpu().numpy()
            assert _rel(yk, OT.inverse_plain(c_in, ref.spectra, ref.W)) <= TOL, key
            assert _rel(c_in, OT.forward_plain(xh[0].astype(np.float64), ref.spectra)) <= TOL, key
        assert _rel(y0.cpu().numpy(), xh) <= TOL
        pf, pi, kf, ki, qf, qi = s.autotune(B)
        # the forward may split up to 32 ways at small batches, the inverse up to 8; at 256 x 256 the
        # forward may take the whole-plane form (reported as panel width 128)
        plane = (N, M) == (256, 256) and pf == 128
        assert (pf in (8, 16) or plane) and pi in (8, 16)
        assert kf in (1, 2, 4, 8, 16, 32) and kf <= ref.K and ki in (1, 2, 4, 8)
        assert qf in (dflt, alt) and qi in (dflt, alt)
        c = s.forward(x)
        y = s.inverse(c)
        torch.cuda.synchronize()
        if plane:
            assert _rel(c.cpu().numpy(), c0.cpu().numpy()) <= 1e-6
        else:
            assert torch.equal(c, c0 if eff(qf, pf) == dflt else ref_alt)
        assert _rel(y.cpu().numpy(), y0.cpu().numpy()) <= 1e-6
        with pytest.raises(Exception):
            s.set_schedule(12, 0)
        with pytest.raises(Exception):
            s.set_schedule(0, 0, ref.K + 1, 0)
        with pytest.raises(Exception):
            s.set_schedule(0, 0, 0, 0, 4, 0)  # no 4-point-per-thread column FFTs
        s.set_schedule(0, 0, 0, 0, dflt, dflt)


def test_schedule_narrow_columns(gpu, lib):
    from paper_2006_04591_amd import ShearError, ShearletSystem

    rng = np.random.default_rng(9)
    S = np.fft.fftshift(np.fft.fft2(rng.standard_normal((2, 32, 16))), axes=(1, 2))
    with ShearletSystem.from_spectra(S) as s:
        with pytest.raises(ShearError):
            s.set_schedule(16, 0)  # 8 packed columns: one panel of 8
        assert s.autotune(2)[:2] == (8, 8)
