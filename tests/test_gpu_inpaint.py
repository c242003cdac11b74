"""GPU parity of inpainting by iterative hard thresholding (Section 4.3,
Algorithm 3) through the C ABI against the FP64 oracle.

As for denoising, each keep/zero decision is an integer decided by floating
point: the oracle runs the iterations itself and places every threshold of
every iteration in a wide gap of its own coefficient magnitudes (within 2% of
delta_i * RMS_k); the GPU runs with those thresholds, so both sides take the
same decisions in every iteration.
"""
import numpy as np
import pytest

import synth
from oracle import apps as OA
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


def _gap(mags, nominal, rel=0.02):
    if nominal <= 0.0:
        return 0.0
    lo, hi = nominal * (1 - rel), nominal * (1 + rel)
    a = np.sort(mags.ravel())
    pts = np.concatenate([[lo], a[(a > lo) & (a < hi)], [hi]])
    i = int(np.argmax(np.diff(pts)))
    return 0.5 * (pts[i] + pts[i + 1])


def oracle_schedule(ref, fm, mask, deltas):
    """Runs Algorithm 3 in FP64 with each threshold moved into a gap; returns the per-iteration
    thresholds (float32-representable, (I, K)) and the oracle's result for them."""
    fm = fm.astype(np.float64)
    mask = mask.astype(np.float64)
    f = np.zeros_like(fm)
    rows = []
    for d in deltas:
        u = mask * (fm - f) + f
        c = OT.forward_plain(u, ref.spectra)
        thr = np.array([_gap(np.abs(c[k]), d * ref.rms[k]) for k in range(ref.K)]).astype(np.float32).astype(np.float64)
        rows.append(thr)
        f = OT.inverse_plain(OA.hard_threshold(c, thr), ref.spectra, ref.W)
    rows = np.array(rows)
    assert np.array_equal(f, OA.inpaint(fm, mask, ref.spectra, ref.W, ref.rms, rows))
    return rows, f


def _d0(ref, fm):
    return float(np.max(np.abs(OT.forward_plain(fm.astype(np.float64), ref.spectra)) / ref.rms[:, None, None]))


@pytest.fixture(scope="module")
def sys128(gpu):
    from paper_2006_04591_amd import ShearletSystem

    _say("case: build 128x128 J=2 (K=17)")
    s = ShearletSystem.build(128, 128, 2)
    yield s, OF.build_system(128, 128, 2)
    s.close()


def _masked(B, N, M, config, seed0):
    f = synth.cartoon_batch(B, N, M, config=config, sigma=0.0)
    m = np.stack([synth.random_mask(N, M, 0.5, seed=seed0 + b) for b in range(B)])
    return f, m, (f * m).astype(np.float32)


def test_inpaint_matches_oracle_128(sys128, gpu):
    s, ref = sys128
    _say("case: inpaint 128x128 K=17 B=2, 6 geometric iterations")
    f, m, fm = _masked(2, 128, 128, 5, 5100)
    thr = []
    want = []
    for b in range(2):
        rows, y = oracle_schedule(ref, fm[b], m[b], OA.delta_schedule(_d0(ref, fm[b]), 2.0, 6))
        thr.append(rows)
        want.append(y)
    thr = np.stack(thr, axis=1)  # (I, B, K)
    y = s.inpaint(_to(fm, gpu), _to(m, gpu), _to(thr, gpu))
    torch.cuda.synchronize()
    for b in range(2):
        assert _rel(y[b].cpu().numpy(), want[b]) <= TOL
        # six iterations already fill part of the missing pixels
        assert OA.psnr(f[b], y[b].cpu().numpy()) > OA.psnr(f[b], fm[b]) + 3.0


def test_inpaint_graph_replays_match_direct_launches(sys128, gpu):
    """The captured graph is replayed with eager work and synchronisations in between; every replay
    equals the directly launched sequence (per-launch timing switches capture off)."""
    s, ref = sys128
    _say("case: inpaint graph replays vs direct launches")
    f, m, fm = _masked(3, 128, 128, 6, 5200)
    deltas = OA.delta_schedule(400.0, 1.0, 5)
    thr = _to(s.inpaint_thresholds(deltas, 3), gpu)
    fmg, mg = _to(fm, gpu), _to(m, gpu)
    s.profile(True)
    direct = s.inpaint(fmg, mg, thr).clone()
    s.profile_read()
    s.profile(False)
    out = torch.empty_like(fmg)
    for rep in range(3):
        s.inpaint(fmg, mg, thr, out=out)
        junk = torch.randn((1 << 20,), device=gpu).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(out, direct), rep
    # new threshold values behind the same pointer: the graph reads them when it runs
    thr2 = _to(s.inpaint_thresholds(OA.delta_schedule(200.0, 1.0, 5), 3), gpu)
    thr.copy_(thr2)
    s.inpaint(fmg, mg, thr, out=out)
    s.profile(True)
    direct2 = s.inpaint(fmg, mg, thr2)
    s.profile_read()
    s.profile(False)
    torch.cuda.synchronize()
    assert torch.equal(out, direct2) and not torch.equal(direct, direct2)


def test_grouped_graph_replays_match_direct_launches(gpu):
    """shear_inpaint_groups: the groups of three sizes in one captured graph (one branch per size),
    replayed several times with eager work and synchronisations in between; every replay equals the
    directly launched sequences (per-launch timing switches capture off) and each size's own
    shear_inpaint call."""
    from paper_2006_04591_amd import UnevenInpainter

    _say("case: grouped inpainting graph (128x128 / 256x256 / 128x256) replays vs direct launches")
    inp = UnevenInpainter(scales=lambda r, c: 2 if max(r, c) <= 128 else 3, autotune=False)
    sizes = [(128, 128), (256, 256), (128, 256), (256, 256), (128, 128)]
    fms, ms, scheds = [], [], []
    for i, (r, c) in enumerate(sizes):
        f = synth.cartoon(r, c, seed=5600 + i)
        m = synth.random_mask(r, c, 0.5, seed=5650 + i)
        fms.append(_to(f * m, gpu))
        ms.append(_to(m, gpu))
        scheds.append(OA.delta_schedule(300.0, 2.0, 4))
    for s in (inp.system(128, 128), inp.system(256, 256), inp.system(128, 256)):
        s.profile(True)
    direct = [t.clone() for t in inp.run(fms, ms, scheds)]
    torch.cuda.synchronize()
    for s in inp._systems.values():
        s.profile_read()
        s.profile(False)
    for rep in range(3):
        out = inp.run(fms, ms, scheds)
        junk = torch.randn((1 << 20,), device=gpu).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i in range(len(sizes)):
            assert torch.equal(out[i], direct[i]), (rep, i)
    # each size group alone through shear_inpaint gives the same images
    for key in ((128, 128), (256, 256), (128, 256)):
        ids = [i for i, sz in enumerate(sizes) if sz == key]
        s = inp.system(*key)
        thr = _to(s.inpaint_thresholds(scheds[ids[0]], len(ids)), gpu)
        y = s.inpaint(torch.stack([fms[i] for i in ids]), torch.stack([ms[i] for i in ids]), thr)
        torch.cuda.synchronize()
        for j, i in enumerate(ids):
            assert torch.equal(y[j], direct[i]), key
    inp.close()


def test_inpaint_linear_schedule_keeps_known_pixels(sys128, gpu):
    s, ref = sys128
    _say("case: inpaint linear decay to zero")
    f, m, fm = _masked(2, 128, 128, 7, 5300)
    deltas = OA.delta_schedule_linear(_d0(ref, fm[0]), 8)
    y = s.inpaint(_to(fm, gpu), _to(m, gpu), _to(s.inpaint_thresholds(deltas, 2), gpu))
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    for b in range(2):
        # the last iteration keeps every coefficient: the known pixels come back
        assert np.linalg.norm((yh[b] - f[b]) * m[b]) <= TOL * np.linalg.norm(f[b] * m[b])
        assert OA.psnr(f[b], yh[b]) > OA.psnr(f[b], fm[b]) + 3.0


def test_inpaint_errors(sys128, gpu):
    s, _ = sys128
    from paper_2006_04591_amd import ShearError

    x = _to(np.zeros((1, 128, 128)), gpu)
    with pytest.raises(ValueError):
        s.inpaint(x, x, np.zeros((3, 1, s.K + 1), np.float32))
    with pytest.raises(ShearError):
        s.inpaint(x, x, np.zeros((0, 1, s.K), np.float32))


def test_uneven_inpainter(gpu):
    """Mixed sizes in one call: one system and one graph per size, groups on their own streams."""
    from paper_2006_04591_amd import UnevenInpainter

    _say("case: uneven inpainting 128/256 mixed, 4 iterations")
    sizes = [128, 256, 256, 128]
    refs = {128: OF.build_system(128, 128, 2), 256: OF.build_system(256, 256, 3)}
    inp = UnevenInpainter(scales=lambda r, c: 2 if r == 128 else 3)
    fms, ms, schedules, wants, cleans = [], [], [], [], []
    for i, n in enumerate(sizes):
        f = synth.cartoon(n, n, seed=5400 + i)
        m = synth.random_mask(n, n, 0.5, seed=5450 + i)
        fm = (f * m).astype(np.float32)
        rows, y = oracle_schedule(refs[n], fm, m, OA.delta_schedule(_d0(refs[n], fm), 3.0, 4))
        fms.append(_to(fm, gpu))
        ms.append(_to(m, gpu))
        schedules.append(rows)
        wants.append(y)
        cleans.append(f)
    out = inp.run(fms, ms, schedules)
    torch.cuda.synchronize()
    for i in range(len(sizes)):
        assert out[i].shape == (sizes[i], sizes[i])
        assert _rel(out[i].cpu().numpy(), wants[i]) <= TOL
    inp.close()


def test_inpaint_uneven_full_sizes(gpu):
    """The uneven workload at full size: 256, 512 and 1024 square images, 50% masks, 100 iterations
    decaying linearly to zero; the oracle checks one 256x256 image over its first 10 iterations."""
    from paper_2006_04591_amd import UnevenInpainter

    _say("case: uneven inpainting 256/512/1024, 100 iterations")
    rng = np.random.default_rng(3)
    sizes = [int(v) for v in rng.choice([256, 512, 1024], size=8)]
    sizes[0] = 256
    inp = UnevenInpainter()
    fms, ms, schedules, cleans = [], [], [], []
    for i, n in enumerate(sizes):
        f = synth.cartoon(n, n, seed=3000 + i)
        m = synth.random_mask(n, n, 0.5, seed=3500 + i)
        fm = (f * m).astype(np.float32)
        s = inp.system(n, n)
        c = s.forward(_to(fm[None], gpu))
        d0 = float((c[0].abs().amax(dim=(1, 2)).cpu().numpy() / s.rms).max())
        fms.append(_to(fm, gpu))
        ms.append(_to(m, gpu))
        schedules.append(OA.delta_schedule_linear(d0, 100))
        cleans.append((f, m, fm))
    out = inp.run(fms, ms, schedules)
    torch.cuda.synchronize()
    for i, n in enumerate(sizes):
        f, m, fm = cleans[i]
        y = out[i].cpu().numpy()
        assert np.all(np.isfinite(y))
        assert np.linalg.norm((y - f) * m) <= TOL * np.linalg.norm(f * m)
        assert OA.psnr(f, y) > OA.psnr(f, fm) + 10.0
    # oracle sample: image 0 (256x256, 33 filters), first 10 iterations of a geometric schedule
    ref = OF.build_system(256, 256, 3)
    f, m, fm = cleans[0]
    rows, want = oracle_schedule(ref, fm, m, OA.delta_schedule(_d0(ref, fm), 2.0, 10))
    y = inp.run([fms[0]], [ms[0]], [rows])[0]
    torch.cuda.synchronize()
    assert _rel(y.cpu().numpy(), want) <= TOL
    inp.close()


@pytest.mark.parametrize("n", [512, 1024])
def test_inpaint_uneven_sizes_match_oracle(gpu, n):
    """The 512 x 512 and 1024 x 1024 members of the uneven workload (49 filters) through the uneven
    inpainter, five iterations against the oracle with gap thresholds, next to a 256 x 256 image."""
    from paper_2006_04591_amd import UnevenInpainter

    _say(f"case: uneven inpainting, {n}x{n} against the oracle, 5 iterations")
    refs = {256: OF.build_system(256, 256, 3), n: OF.build_system(n, n, 4)}
    inp = UnevenInpainter()
    fms, ms, schedules, wants = [], [], [], []
    for i, sz in enumerate((n, 256)):
        f = synth.cartoon(sz, sz, seed=3700 + i)
        m = synth.random_mask(sz, sz, 0.5, seed=3750 + i)
        fm = (f * m).astype(np.float32)
        rows, y = oracle_schedule(refs[sz], fm, m, OA.delta_schedule(_d0(refs[sz], fm), 2.0, 5))
        fms.append(_to(fm, gpu))
        ms.append(_to(m, gpu))
        schedules.append(rows)
        wants.append(y)
    out = inp.run(fms, ms, schedules)
    torch.cuda.synchronize()
    for i in range(2):
        assert _rel(out[i].cpu().numpy(), wants[i]) <= TOL
    inp.close()


def test_inpaint_2048_columns_user_bank(gpu):
    """Algorithm 3 on 16 x 2048 images (the row kernel that mixes mask, masked image and estimate at
    2048 columns) with a user filter bank, three iterations against the oracle with gap thresholds."""
    from paper_2006_04591_amd import ShearletSystem

    _say("case: inpaint 16x2048 user bank K=3 B=2, 3 iterations")
    rng = np.random.default_rng(2048)
    ker = rng.standard_normal((3, 16, 2048))
    ker = ker + ker[:, (-np.arange(16)) % 16][:, :, (-np.arange(2048)) % 2048]
    S = np.fft.fft2(ker)

    class _Ref:
        spectra = S
        W = np.sum(np.abs(S) ** 2, axis=0)
        rms = np.sqrt(np.mean(np.abs(S) ** 2, axis=(1, 2)))
        K = 3

    f = (100.0 + 50.0 * rng.standard_normal((2, 16, 2048))).astype(np.float32)
    m = (rng.random((2, 16, 2048)) < 0.5).astype(np.float32)
    fm = (f * m).astype(np.float32)
    thr, want = [], []
    for b in range(2):
        rows, y = oracle_schedule(_Ref, fm[b], m[b], OA.delta_schedule(_d0(_Ref, fm[b]), 1.0, 3))
        thr.append(rows)
        want.append(y)
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        y = s.inpaint(_to(fm, gpu), _to(m, gpu), _to(np.stack(thr, axis=1), gpu))
        torch.cuda.synchronize()
        for b in range(2):
            assert _rel(y[b].cpu().numpy(), want[b]) <= TOL
