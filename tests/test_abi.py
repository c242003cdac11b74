"""CPU checks of the C ABI library: it loads, exports every declared symbol, and
its host-side FP64 filter design equals the oracle's (independent code: the
library builds spatial kernels and FFTs them, the oracle evaluates closed
forms on exact DFT grids). No GPU is needed."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import filters as OF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shear.h")


@pytest.fixture(scope="module")
def P():
    import paper_2006_04591_amd as P

    P.load_library()
    return P


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(shear_[a-z_]+)\s*\(", text)))


def test_header_symbols_exported(P):
    lib = ctypes.CDLL(P.LIB_PATH)
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(P.EXPORTED)


def test_strerror(P):
    lib = P.load_library()
    assert lib.shear_strerror(0) == b"ok"
    assert b"size" in lib.shear_strerror(-2)
    assert lib.shear_strerror(-99) == b"unknown error"


@pytest.mark.parametrize("N,M,J,levels", [(128, 128, 2, None), (256, 256, 3, None), (128, 256, 2, [1, 2]),
                                          (64, 64, 1, [0]), (256, 128, 3, [0, 1, 2])])
def test_design_matches_oracle(P, N, M, J, levels):
    S, idx = P.design_spectra(N, M, J, levels)
    ref = OF.build_system(N, M, J, levels)
    assert S.shape == ref.centred.shape
    assert np.max(np.abs(S - ref.centred)) <= 1e-12 * np.max(np.abs(ref.centred))
    assert np.array_equal(idx, ref.idx)


def test_design_512_k49_matches_oracle(P):
    S, idx = P.design_spectra(512, 512, 4)
    ref = OF.build_system(512, 512, 4)
    assert S.shape[0] == 49
    assert np.max(np.abs(S - ref.centred)) <= 1e-12 * np.max(np.abs(ref.centred))


def test_design_custom_taps_match_oracle(P):
    rng = np.random.default_rng(3)
    h = rng.standard_normal(7)  # asymmetric: complex Hermitian spectra
    p = rng.standard_normal((5, 3))
    S, idx = P.design_spectra(128, 128, 2, None, scaling_taps=h, fan_taps=p)
    ref = OF.build_system(128, 128, 2, h=h, p=p)
    assert np.max(np.abs(ref.centred.imag)) > 1e-3
    assert np.max(np.abs(S - ref.centred)) <= 1e-12 * np.max(np.abs(ref.centred))


def test_design_size_policy_matches_oracle(P):
    from paper_2006_04591_amd import ShearError

    for (N, J, levels) in [(64, 4, [1, 1, 2, 2]), (32, 2, [1, 1]), (128, 2, [1, 1]), (256, 4, [1, 1, 2, 2])]:
        fits = OF.system_fits(N, N, J, levels)
        if fits:
            P.design_spectra(N, N, J, levels)
        else:
            with pytest.raises(ShearError) as e:
                P.design_spectra(N, N, J, levels)
            assert e.value.name == "SHEAR_E_SIZE"


@pytest.mark.parametrize("kw,code", [
    (dict(rows=100, cols=128, n_scales=2), "SHEAR_E_SIZE"),
    (dict(rows=128, cols=128, n_scales=0), "SHEAR_E_INVALID"),
    (dict(rows=128, cols=128, n_scales=2, shear_levels=[1, 9]), "SHEAR_E_INVALID"),
    (dict(rows=128, cols=128, n_scales=2, scaling_taps=np.ones(4)), "SHEAR_E_INVALID"),
    (dict(rows=128, cols=128, n_scales=2, fan_taps=np.ones((2, 3))), "SHEAR_E_INVALID"),
])
def test_design_errors(P, kw, code):
    from paper_2006_04591_amd import ShearError

    with pytest.raises(ShearError) as e:
        P.design_spectra(**kw)
    assert e.value.name == code
    assert len(P.load_library().shear_last_error()) > 0


def test_null_arguments_return_invalid(P):
    lib = P.load_library()
    assert lib.shear_design_spectra(None, None, None, None) == -1
    assert lib.shear_build_system(None, None) == -1
    assert lib.shear_system_info(None, None, None, None, None, None) == -1
    assert lib.shear_export_spectra(None, None, None) == -1
    assert lib.shear_forward(None, None, None, 1, None) == -1
    assert lib.shear_inverse(None, None, None, 1, None) == -1
    assert lib.shear_adjoint(None, None, None, 1, None) == -1
    assert lib.shear_reserve(None, 1) == -1
    assert lib.shear_profile_enable(None, 1) == -1
    lib.shear_destroy_system(None)  # no-op


def test_count_query(P):
    lib = P.load_library()
    from paper_2006_04591_amd._binding import _params

    keep = []
    p = _params(512, 512, 4, None, None, None, 0, keep)
    K = ctypes.c_int(0)
    assert lib.shear_design_spectra(ctypes.byref(p), ctypes.byref(K), None, None) == 0
    assert K.value == 49


def test_delta_schedule_matches_oracle(P):
    """Algorithm 3's threshold decay, computed by the library (host only) against the oracle."""
    from oracle import apps as OA

    for (d0, dmin, it) in [(8.0, 0.5, 5), (250.0, 1.0, 100), (3.0, 1.0, 1), (1.0, 0.01, 50)]:
        got = P.delta_schedule("geometric", d0, it, dmin)
        assert np.allclose(got, OA.delta_schedule(d0, dmin, it), rtol=1e-13, atol=0)
        assert got[0] == d0
    for (d0, it) in [(120.0, 100), (5.0, 2), (7.0, 1)]:
        got = P.delta_schedule("linear", d0, it)
        assert np.allclose(got, OA.delta_schedule_linear(d0, it), rtol=1e-13, atol=1e-13)
    lib = P.load_library()
    out = (ctypes.c_double * 4)()
    assert lib.shear_delta_schedule(0, 1.0, 0.0, 4, out) == -1  # geometric decay needs delta_min > 0
    assert lib.shear_delta_schedule(7, 1.0, 0.5, 4, out) == -1
    assert lib.shear_delta_schedule(1, 1.0, 0.0, 0, out) == -1
    assert lib.shear_delta_schedule(1, 1.0, 0.0, 4, None) == -1
    assert lib.shear_denoise_thresholds(None, None, 1, None, 0, None) == -1
    assert lib.shear_inpaint_thresholds(None, None, 1, 1, None) == -1
