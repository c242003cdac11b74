"""The allocation-free forward (shear_forward_noalloc), through the C ABI, against shear_forward:
bitwise equal on two calls in a row, the second with a smaller input, at sizes that take one and
several scratch chunks; a size whose single image exceeds the fixed scratch is refused."""
import ctypes

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _to(x, dev):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(dev)


@pytest.mark.parametrize("N,M,J,B1,B2", [(128, 128, 2, 5, 2), (512, 512, 4, 3, 1), (256, 256, 3, 9, 4)])
def test_forward_noalloc_matches_forward(gpu, N, M, J, B1, B2):
    from paper_2006_04591_amd import ShearletSystem, load_library

    lib = load_library()
    with ShearletSystem.build(N, M, J) as s:
        for B in (B1, B2):  # two calls in a row, the second smaller: the scratch keeps the first's contents
            _say(f"case: shear_forward_noalloc {N}x{M} K={s.K} B={B}")
            x = _to(synth.cartoon_batch(B, N, M, config=9, sigma=15.0), gpu)
            want = s.forward(x)
            got = torch.full((B, s.K, N, M), float("nan"), dtype=torch.float32, device=gpu)
            torch.cuda.synchronize()
            rc = lib.shear_forward_noalloc(s._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(got.data_ptr()), B,
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
            assert rc == 0, lib.shear_last_error()
            torch.cuda.synchronize()
            assert torch.equal(got, want)
        # the empty batch is a no-op
        assert lib.shear_forward_noalloc(s._h, None, None, 0, None) == 0


def test_forward_noalloc_refuses_oversized_images(gpu):
    from paper_2006_04591_amd import ShearError, ShearletSystem

    _say("case: shear_forward_noalloc at 1024x1024 K=49 (one image exceeds the fixed scratch)")
    with ShearletSystem.build(1024, 1024, 4) as s:
        x = torch.zeros((1, 1024, 1024), dtype=torch.float32, device=gpu)
        out = torch.empty((1, s.K, 1024, 1024), dtype=torch.float32, device=gpu)
        with pytest.raises(ShearError) as e:
            s.forward_noalloc(x, out)
        assert e.value.name == "SHEAR_E_SIZE" and "scratch" in str(e.value)
