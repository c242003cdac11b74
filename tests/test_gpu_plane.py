"""GPU parity of the whole-plane forward (256 x 256 systems with real filter sets): one workgroup
per (image, filter) plane filters the image's column spectra, runs the column IFFT as 16 x 16 (four
steps) and the row c2r on chip, and writes only the coefficients. Checked against the FP64 oracle
(relative L2 <= 1e-5 over whole tensors), against the panel form (to rounding), in chunks, and with
the schedule switching back; the inverse of its coefficients reconstructs the images."""
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


@pytest.fixture(scope="module")
def sys256(gpu):
    from paper_2006_04591_amd import ShearletSystem

    _say("case: build 256x256 J=3 (K=33)")
    s = ShearletSystem.build(256, 256, 3)
    ref = OF.build_system(256, 256, 3)
    yield s, ref
    s.close()


def test_plane_forward_matches_oracle(sys256, gpu):
    s, ref = sys256
    _say("case: whole-plane forward 256x256 K=33 B=3")
    x = synth.cartoon_batch(3, 256, 256, config=4)
    xg = _to(x, gpu)
    s.set_schedule(16, 0, 1, 0, 8, 0)
    c_panel = s.forward(xg)
    s.set_schedule(128)
    s.profile(True)
    c = s.forward(xg)
    rec = s.profile_read()
    s.profile(False)
    y = s.inverse(c)
    torch.cuda.synchronize()
    # the spectra pass counts as the forward's column pass; no exchange planes, no coefficient row pass
    assert rec["plane_fwd"][0] == 1 and rec["cols_fwd"][0] == 1 and rec["rows_c2r_coeffs"][0] == 0
    got = c.double().cpu().numpy()
    for b in range(3):
        want = OT.forward_plain(x[b].astype(np.float64), ref.spectra)
        assert _rel(got[b], want) <= TOL, b
        nx = np.linalg.norm(x[b].astype(np.float64))
        per = [np.linalg.norm(got[b, k] - want[k]) / (nx * ref.rms[k]) for k in range(ref.K)]
        assert max(per) <= TOL, b
    assert _rel(got, c_panel.cpu().numpy()) <= 1e-6
    assert _rel(y.cpu().numpy(), x) <= TOL
    # back to the panel form: the same bits as before
    s.set_schedule(16)
    c2 = s.forward(xg)
    torch.cuda.synchronize()
    assert torch.equal(c2, c_panel)


def test_plane_forward_layer_batch_sampled(sys256, gpu):
    """The differentiable layer's batch (32 images, 33 filters: 1056 workgroups, a tail of 32 past
    four per compute unit), sampled planes against the oracle and a whole-tensor check against the
    panel form."""
    s, ref = sys256
    _say("case: whole-plane forward 256x256 K=33 B=32")
    x = synth.cartoon_batch(32, 256, 256, config=4)
    xg = _to(x, gpu)
    s.set_schedule(16, 0, 1, 0, 8, 0)
    c_panel = s.forward(xg)
    s.set_schedule(128)
    c = s.forward(xg)
    torch.cuda.synchronize()
    for b in (0, 13, 31):
        x64 = x[b].astype(np.float64)
        want = OT.forward_plain(x64, ref.spectra)
        assert _rel(c[b].double().cpu().numpy(), want) <= TOL, b
    assert _rel(c.cpu().numpy(), c_panel.cpu().numpy()) <= 1e-6
    s.set_schedule(16)


def test_plane_forward_chunked(gpu):
    """A workspace cap that forces chunks of images: the chunk's column spectra reuse the room of its
    exchange planes, and the results equal the unchunked ones bit for bit."""
    from paper_2006_04591_amd import ShearletSystem

    _say("case: whole-plane forward in chunks 256x256 K=33 B=5")
    x = _to(synth.cartoon_batch(5, 256, 256, config=4), gpu)
    with ShearletSystem.build(256, 256, 3) as s:
        s.set_schedule(128)
        c_all = s.forward(x)
        torch.cuda.synchronize()
    plane = 256 * 128 * 8
    with ShearletSystem.build(256, 256, 3, max_workspace_bytes=5 * plane + 2 * 34 * plane) as s:
        s.set_schedule(128)
        c = s.forward(x)
        torch.cuda.synchronize()
    assert torch.equal(c, c_all)


def test_plane_forward_user_banks(gpu):
    """A real user bank at 256 x 256 takes the whole-plane forward; a complex one, and other sizes,
    refuse it."""
    from paper_2006_04591_amd import ShearError, ShearletSystem

    rng = np.random.default_rng(256)
    ker = rng.standard_normal((4, 256, 256))
    ker = ker + ker[:, (-np.arange(256)) % 256][:, :, (-np.arange(256)) % 256]
    S = np.fft.fft2(ker)
    x = rng.standard_normal((2, 256, 256)).astype(np.float32)
    _say("case: whole-plane forward, real user bank 256x256 K=4 B=2")
    with ShearletSystem.from_spectra(np.fft.fftshift(S, axes=(1, 2))) as s:
        s.set_schedule(128)
        c = s.forward(_to(x, gpu))
        torch.cuda.synchronize()
        for b in range(2):
            assert _rel(c[b].cpu().numpy(), OT.forward_plain(x[b].astype(np.float64), S)) <= TOL
    Sc = np.fft.fft2(rng.standard_normal((3, 256, 256)))
    with ShearletSystem.from_spectra(np.fft.fftshift(Sc, axes=(1, 2))) as s:
        with pytest.raises(ShearError):
            s.set_schedule(128)
    Sr = np.fft.fft2(rng.standard_normal((2, 128, 128)))
    Sr = Sr.real.astype(complex)
    with ShearletSystem.from_spectra(np.fft.fftshift(Sr, axes=(1, 2))) as s:
        with pytest.raises(ShearError):
            s.set_schedule(64)


def test_plane_forward_leaves_denoising_on_panels(sys256, gpu):
    """The denoising chain keeps its panel column pass with the whole-plane forward selected."""
    s, ref = sys256
    _say("case: denoise with the whole-plane forward selected 256x256 K=33 B=2")
    x = _to(synth.cartoon_batch(2, 256, 256, config=4), gpu)
    thr = torch.zeros((2, ref.K), dtype=torch.float32, device=gpu)
    s.set_schedule(16)
    y0, k0 = s.denoise(x, thr, kept=True)
    s.set_schedule(128)
    y1, k1 = s.denoise(x, thr, kept=True)
    torch.cuda.synchronize()
    assert torch.equal(y0, y1) and torch.equal(k0, k1)
    s.set_schedule(16)
