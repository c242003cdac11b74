"""ctypes binding of libshear.so (include/shear.h). Argument marshalling only.

Every transform step runs in the HIP library; PyTorch supplies device memory
(tensor data pointers) and the current HIP stream. There is no fallback: if
the library is missing or fails to load, using the binding raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libshear.so")

SHEAR_OK = 0
ERRORS = {
    -1: "SHEAR_E_INVALID",
    -2: "SHEAR_E_SIZE",
    -3: "SHEAR_E_FRAME",
    -4: "SHEAR_E_NOMEM",
    -5: "SHEAR_E_HIP",
    -6: "SHEAR_E_DEVICE",
}

EXPORTED = (
    "shear_design_spectra",
    "shear_build_system",
    "shear_system_from_spectra",
    "shear_system_info",
    "shear_export_spectra",
    "shear_reserve",
    "shear_workspace_bytes",
    "shear_forward",
    "shear_forward_noalloc",
    "shear_inverse",
    "shear_adjoint",
    "shear_denoise",
    "shear_denoise_thresholds",
    "shear_inpaint",
    "shear_inpaint_groups",
    "shear_inpaint_thresholds",
    "shear_delta_schedule",
    "shear_profile_enable",
    "shear_profile_read",
    "shear_set_schedule",
    "shear_autotune",
    "shear_shrink_params_bytes",
    "shear_shrink_pack",
    "shear_shrink_apply",
    "shear_shrink_param_count",
    "shear_shrink_train_step",
    "shear_destroy_system",
    "shear_strerror",
    "shear_last_error",
)


class ShearError(RuntimeError):
    """A negative status returned by libshear."""

    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        self.name = ERRORS.get(code, "UNKNOWN")
        super().__init__(f"{where}: {self.name} ({code}): {detail}")


class BuildParams(ctypes.Structure):
    _fields_ = [
        ("rows", ctypes.c_int),
        ("cols", ctypes.c_int),
        ("n_scales", ctypes.c_int),
        ("shear_levels", ctypes.POINTER(ctypes.c_int)),
        ("scaling_taps", ctypes.POINTER(ctypes.c_double)),
        ("n_scaling", ctypes.c_int),
        ("fan_taps", ctypes.POINTER(ctypes.c_double)),
        ("fan_rows", ctypes.c_int),
        ("fan_cols", ctypes.c_int),
        ("max_workspace_bytes", ctypes.c_size_t),
    ]


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libshear.so once and declares the C signatures. Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run __graft_entry__.build() (hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    pI = ctypes.POINTER(ctypes.c_int)
    pD = ctypes.POINTER(ctypes.c_double)
    lib.shear_design_spectra.argtypes = [ctypes.POINTER(BuildParams), pI, pD, pI]
    lib.shear_build_system.argtypes = [ctypes.POINTER(BuildParams), ctypes.POINTER(P)]
    lib.shear_system_from_spectra.argtypes = [I, I, I, pD, pI, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.shear_system_info.argtypes = [P, pI, pI, pI, pD, pI]
    lib.shear_export_spectra.argtypes = [P, pD, pD]
    lib.shear_reserve.argtypes = [P, I]
    lib.shear_workspace_bytes.argtypes = [P, I, ctypes.POINTER(ctypes.c_size_t)]
    for name in ("shear_forward", "shear_forward_noalloc", "shear_inverse", "shear_adjoint"):
        getattr(lib, name).argtypes = [P, P, P, I, P]
    lib.shear_denoise.argtypes = [P, P, P, I, P, P, P]
    lib.shear_inpaint.argtypes = [P, P, P, P, I, P, I, P]
    PP = ctypes.POINTER(ctypes.c_void_p)
    lib.shear_inpaint_groups.argtypes = [PP, I, PP, PP, PP, pI, PP, I, P]
    lib.shear_denoise_thresholds.argtypes = [P, pD, I, pD, I, ctypes.POINTER(ctypes.c_float)]
    lib.shear_inpaint_thresholds.argtypes = [P, pD, I, I, ctypes.POINTER(ctypes.c_float)]
    lib.shear_delta_schedule.argtypes = [I, ctypes.c_double, ctypes.c_double, I, pD]
    for name in EXPORTED:
        if name not in ("shear_destroy_system", "shear_strerror", "shear_last_error"):
            getattr(lib, name).restype = I
    lib.shear_set_schedule.argtypes = [P, I, I, I, I, I, I]
    lib.shear_shrink_params_bytes.argtypes = [I, ctypes.POINTER(ctypes.c_size_t)]
    lib.shear_shrink_pack.argtypes = [P, P, P, P, P, P, P, P, P]
    lib.shear_shrink_apply.argtypes = [P, P, P, P, I, P, P, P]
    lib.shear_shrink_param_count.argtypes = [I]
    lib.shear_shrink_train_step.argtypes = [P, P, P, I, P, P, P, P, P, I, ctypes.c_float, ctypes.c_float, P, P]
    lib.shear_autotune.argtypes = [P, I, pI, pI, pI, pI, pI, pI]
    lib.shear_profile_enable.argtypes = [P, I]
    lib.shear_profile_read.argtypes = [P, pI, pD]
    lib.shear_destroy_system.argtypes = [P]
    lib.shear_destroy_system.restype = None
    lib.shear_strerror.argtypes = [I]
    lib.shear_strerror.restype = ctypes.c_char_p
    lib.shear_last_error.argtypes = []
    lib.shear_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(rc: int, where: str) -> None:
    if rc != SHEAR_OK:
        detail = load_library().shear_last_error().decode(errors="replace")
        raise ShearError(rc, where, detail)


def _params(rows, cols, n_scales, shear_levels, scaling_taps, fan_taps, max_workspace_bytes, keep: list) -> BuildParams:
    p = BuildParams()
    p.rows, p.cols, p.n_scales = int(rows), int(cols), int(n_scales)
    if shear_levels is not None:
        arr = (ctypes.c_int * len(shear_levels))(*[int(v) for v in shear_levels])
        keep.append(arr)
        p.shear_levels = ctypes.cast(arr, ctypes.POINTER(ctypes.c_int))
    if scaling_taps is not None:
        h = np.ascontiguousarray(scaling_taps, dtype=np.float64)
        keep.append(h)
        p.scaling_taps = h.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.n_scaling = h.size
    if fan_taps is not None:
        f = np.ascontiguousarray(fan_taps, dtype=np.float64)
        keep.append(f)
        p.fan_taps = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.fan_rows, p.fan_cols = f.shape
    p.max_workspace_bytes = int(max_workspace_bytes)
    return p


def design_spectra(rows: int, cols: int, n_scales: int, shear_levels: Optional[Sequence[int]] = None,
                   scaling_taps=None, fan_taps=None):
    """Host-only filter design (shear_design_spectra). Returns (spectra_centred complex128 (K,rows,cols), idx (K,3))."""
    lib = load_library()
    keep: list = []
    p = _params(rows, cols, n_scales, shear_levels, scaling_taps, fan_taps, 0, keep)
    K = ctypes.c_int(0)
    _check(lib.shear_design_spectra(ctypes.byref(p), ctypes.byref(K), None, None), "shear_design_spectra")
    spec = np.zeros((K.value, rows, cols, 2), dtype=np.float64)
    idx = np.zeros((K.value, 3), dtype=np.int32)
    _check(lib.shear_design_spectra(ctypes.byref(p), ctypes.byref(K),
                                    spec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "shear_design_spectra")
    return spec[..., 0] + 1j * spec[..., 1], idx


def _dptr(a: np.ndarray):
    """ctypes double* of a contiguous float64 array."""
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def delta_schedule(kind: str, delta_init: float, iterations: int, delta_min: float = 0.0) -> np.ndarray:
    """Algorithm 3's threshold decay (shear_delta_schedule): kind "geometric" (delta_init to delta_min)
    or "linear" (delta_init to 0). float64 (iterations,)."""
    kinds = {"geometric": 0, "linear": 1}
    if kind not in kinds:
        raise ValueError(f"kind must be one of {sorted(kinds)}")
    out = np.empty(int(iterations), dtype=np.float64)
    _check(load_library().shear_delta_schedule(kinds[kind], float(delta_init), float(delta_min), int(iterations),
                                               _dptr(out)), "shear_delta_schedule")
    return out


def _stream_ptr(stream) -> ctypes.c_void_p:
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(int(s.cuda_stream))


class ShearletSystem:
    """A shearlet system on the current GPU (shear_build_system / shear_system_from_spectra)."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self._lib = load_library()
        K, r, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self._lib.shear_system_info(self._h, ctypes.byref(K), ctypes.byref(r), ctypes.byref(c), None, None),
               "shear_system_info")
        self.K, self.rows, self.cols = K.value, r.value, c.value

    # ------------------------------------------------------------ construction
    @classmethod
    def build(cls, rows: int, cols: int, n_scales: int, shear_levels: Optional[Sequence[int]] = None,
              scaling_taps=None, fan_taps=None, max_workspace_bytes: int = 0) -> "ShearletSystem":
        lib = load_library()
        keep: list = []
        p = _params(rows, cols, n_scales, shear_levels, scaling_taps, fan_taps, max_workspace_bytes, keep)
        h = ctypes.c_void_p()
        _check(lib.shear_build_system(ctypes.byref(p), ctypes.byref(h)), "shear_build_system")
        return cls(h)

    @classmethod
    def from_spectra(cls, spectra_centred, idx=None, max_workspace_bytes: int = 0) -> "ShearletSystem":
        lib = load_library()
        S = np.asarray(spectra_centred)
        K, rows, cols = S.shape
        buf = np.ascontiguousarray(np.stack([S.real, S.imag], axis=-1), dtype=np.float64)
        pidx = None
        if idx is not None:
            iv = np.ascontiguousarray(idx, dtype=np.int32)
            pidx = iv.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        h = ctypes.c_void_p()
        _check(lib.shear_system_from_spectra(rows, cols, K, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), pidx,
                                             int(max_workspace_bytes), ctypes.byref(h)), "shear_system_from_spectra")
        return cls(h)

    # ------------------------------------------------------------ info
    @property
    def rms(self) -> np.ndarray:
        out = np.zeros(self.K, dtype=np.float64)
        _check(self._lib.shear_system_info(self._h, None, None, None, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                           None), "shear_system_info")
        return out

    @property
    def idx(self) -> np.ndarray:
        out = np.zeros((self.K, 3), dtype=np.int32)
        _check(self._lib.shear_system_info(self._h, None, None, None, None,
                                           out.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "shear_system_info")
        return out

    def export_spectra(self):
        """(spectra_centred complex128 (K, rows, cols), W_centred float64 (rows, cols))."""
        spec = np.zeros((self.K, self.rows, self.cols, 2), dtype=np.float64)
        W = np.zeros((self.rows, self.cols), dtype=np.float64)
        _check(self._lib.shear_export_spectra(self._h, spec.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                              W.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "shear_export_spectra")
        return spec[..., 0] + 1j * spec[..., 1], W

    def reserve(self, batch: int) -> None:
        _check(self._lib.shear_reserve(self._h, int(batch)), "shear_reserve")

    def workspace_bytes(self, batch: int) -> int:
        b = ctypes.c_size_t()
        _check(self._lib.shear_workspace_bytes(self._h, int(batch), ctypes.byref(b)), "shear_workspace_bytes")
        return b.value

    # ------------------------------------------------------------ transforms
    def _check_tensor(self, t, shape, name):
        import torch

        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def forward(self, x, out=None, stream=None):
        """shear_forward: x (B, rows, cols) -> coefficients (B, K, rows, cols)."""
        import torch

        B = x.shape[0]
        self._check_tensor(x, (B, self.rows, self.cols), "x")
        if out is None:
            out = torch.empty((B, self.K, self.rows, self.cols), dtype=torch.float32, device=x.device)
        self._check_tensor(out, (B, self.K, self.rows, self.cols), "out")
        _check(self._lib.shear_forward(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), B,
                                       _stream_ptr(stream)), "shear_forward")
        return out

    def forward_noalloc(self, x, out):
        """shear_forward_noalloc: as forward, through the library's fixed device scratch (no allocation in
        the call); ``out`` (B, K, rows, cols) must be given."""
        B = x.shape[0]
        self._check_tensor(x, (B, self.rows, self.cols), "x")
        self._check_tensor(out, (B, self.K, self.rows, self.cols), "out")
        _check(self._lib.shear_forward_noalloc(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                               B, _stream_ptr(None)), "shear_forward_noalloc")
        return out

    def _inv(self, fn, name, c, out, stream):
        import torch

        B = c.shape[0]
        self._check_tensor(c, (B, self.K, self.rows, self.cols), "coeffs")
        if out is None:
            out = torch.empty((B, self.rows, self.cols), dtype=torch.float32, device=c.device)
        self._check_tensor(out, (B, self.rows, self.cols), "out")
        _check(fn(self._h, ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(out.data_ptr()), B, _stream_ptr(stream)), name)
        return out

    def inverse(self, coeffs, out=None, stream=None):
        """shear_inverse: coefficients (B, K, rows, cols) -> images (B, rows, cols)."""
        return self._inv(self._lib.shear_inverse, "shear_inverse", coeffs, out, stream)

    def adjoint(self, coeffs, out=None, stream=None):
        """shear_adjoint: coefficients (B, K, rows, cols) -> images (B, rows, cols)."""
        return self._inv(self._lib.shear_adjoint, "shear_adjoint", coeffs, out, stream)

    # ------------------------------------------------------------ denoising
    def paper_thresholds(self, sigma, factors=None) -> np.ndarray:
        """Thresholds of the denoising rule of Section 4.2 (shear_denoise_thresholds): K_j sigma RMS_k for
        filter k of scale j, the low-pass taking K_1. sigma: a scalar -> float32 (K,), or B values ->
        (B, K). factors: J values K_1..K_J (coarse to fine), or None for the paper's [2.5, ..., 3.8]."""
        sig = np.ascontiguousarray(np.atleast_1d(np.asarray(sigma, dtype=np.float64)))
        out = np.empty((sig.shape[0], self.K), dtype=np.float32)
        f = None if factors is None else np.ascontiguousarray(factors, dtype=np.float64)
        _check(self._lib.shear_denoise_thresholds(self._h, _dptr(sig), int(sig.shape[0]),
                                                  None if f is None else _dptr(f), 0 if f is None else int(f.size),
                                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "shear_denoise_thresholds")
        return out[0] if np.ndim(sigma) == 0 else out

    def denoise(self, x, thresholds, out=None, kept=False, stream=None):
        """shear_denoise: y = SH^-1 T SH x with hard thresholds (B, K) or (K,) (float32, on x's device).
        Returns y, or (y, kept counts (B, K) int64 tensor) when kept is True."""
        import torch

        B = x.shape[0]
        self._check_tensor(x, (B, self.rows, self.cols), "x")
        thr = torch.as_tensor(thresholds, dtype=torch.float32, device=x.device)
        if thr.dim() == 1:
            if thr.shape[0] != self.K:
                raise ValueError(f"thresholds has {thr.shape[0]} entries, expected K = {self.K}")
            thr = thr.expand(B, self.K)
        thr = thr.contiguous()
        self._check_tensor(thr, (B, self.K), "thresholds")
        if out is None:
            out = torch.empty((B, self.rows, self.cols), dtype=torch.float32, device=x.device)
        self._check_tensor(out, (B, self.rows, self.cols), "out")
        cnt = torch.empty((B, self.K), dtype=torch.int32, device=x.device) if kept else None
        _check(self._lib.shear_denoise(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), B,
                                       ctypes.c_void_p(thr.data_ptr()),
                                       ctypes.c_void_p(cnt.data_ptr()) if kept else None, _stream_ptr(stream)),
               "shear_denoise")
        if kept:
            # the library writes uint32 counts; a plane has at most 2^20 coefficients
            return out, cnt.to(torch.int64)
        return out

    # ------------------------------------------------------------ inpainting
    def inpaint_thresholds(self, deltas, batch: int) -> np.ndarray:
        """Algorithm 3's per-filter thresholds (shear_inpaint_thresholds): thresholds[i][b][k] =
        deltas[i] * RMS_k for a schedule of I scalars (every image alike), or deltas[i][b] for an
        (I, batch) schedule. float32 (I, batch, K)."""
        d = np.asarray(deltas, dtype=np.float64)
        if d.ndim == 1:
            d = np.repeat(d[:, None], batch, axis=1)
        if d.ndim != 2 or d.shape[1] != batch:
            raise ValueError(f"deltas must be (iterations,) or (iterations, {batch}), got {d.shape}")
        d = np.ascontiguousarray(d)
        out = np.empty((d.shape[0], batch, self.K), dtype=np.float32)
        _check(self._lib.shear_inpaint_thresholds(self._h, _dptr(d), int(d.shape[0]), int(batch),
                                                  out.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               "shear_inpaint_thresholds")
        return out

    def inpaint(self, f_masked, mask, thresholds, out=None, stream=None):
        """shear_inpaint: Algorithm 3 on a batch (B, rows, cols); thresholds (iterations, B, K) float32."""
        import torch

        B = f_masked.shape[0]
        self._check_tensor(f_masked, (B, self.rows, self.cols), "f_masked")
        self._check_tensor(mask, (B, self.rows, self.cols), "mask")
        thr = torch.as_tensor(thresholds, dtype=torch.float32, device=f_masked.device).contiguous()
        if thr.dim() != 3 or thr.shape[1:] != (B, self.K):
            raise ValueError(f"thresholds must be (iterations, {B}, {self.K}), got {tuple(thr.shape)}")
        if out is None:
            out = torch.empty((B, self.rows, self.cols), dtype=torch.float32, device=f_masked.device)
        self._check_tensor(out, (B, self.rows, self.cols), "out")
        _check(self._lib.shear_inpaint(self._h, ctypes.c_void_p(f_masked.data_ptr()), ctypes.c_void_p(mask.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()), B, ctypes.c_void_p(thr.data_ptr()),
                                       int(thr.shape[0]), _stream_ptr(stream)), "shear_inpaint")
        # the graph reads the thresholds when it runs: keep them alive with the output
        self._keep = thr
        return out

    # ------------------------------------------------------------ column-pass schedule
    def set_schedule(self, pw_fwd: int = 0, pw_inv: int = 0, kg_fwd: int = 0, kg_inv: int = 0, pc_fwd: int = 0,
                     pc_inv: int = 0) -> None:
        """Columns per block, filter groups and points per thread (radix sequence) of the forward and
        inverse column passes (shear_set_schedule); 0 keeps a value."""
        _check(self._lib.shear_set_schedule(self._h, int(pw_fwd), int(pw_inv), int(kg_fwd), int(kg_inv), int(pc_fwd),
                                            int(pc_inv)), "shear_set_schedule")

    def autotune(self, batch: int):
        """Times the compiled column-pass schedules at this batch size and keeps the fastest
        (shear_autotune); returns (pw_fwd, pw_inv, kg_fwd, kg_inv, pc_fwd, pc_inv)."""
        v = [ctypes.c_int() for _ in range(6)]
        _check(self._lib.shear_autotune(self._h, int(batch), *[ctypes.byref(x) for x in v]), "shear_autotune")
        return tuple(x.value for x in v)

    # ------------------------------------------------------------ tracing
    KERNEL_KINDS = ("rows_r2c_images", "cols_fwd", "rows_c2r_coeffs", "rows_r2c_coeffs", "cols_inv", "rows_c2r_images",
                    "rows_thresh", "plane_fwd")

    def profile(self, on: bool = True) -> None:
        """Brackets every launch with hipEvents on the caller's stream (shear_profile_enable)."""
        _check(self._lib.shear_profile_enable(self._h, 1 if on else 0), "shear_profile_enable")

    def profile_read(self) -> dict:
        """{kind: (launches, total_ms)} since the last read (shear_profile_read); waits for the events."""
        n = (ctypes.c_int * len(self.KERNEL_KINDS))()
        ms = (ctypes.c_double * len(self.KERNEL_KINDS))()
        _check(self._lib.shear_profile_read(self._h, n, ms), "shear_profile_read")
        return {k: (n[i], ms[i]) for i, k in enumerate(self.KERNEL_KINDS)}

    # ------------------------------------------------------------ lifetime
    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.shear_destroy_system(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class ShrinkNet:
    """Learned shrinkage network of a system (shear_shrink_pack / shear_shrink_apply): FP32 parameters
    W1 (32, K, 3, 3), b1 (32,), W2 (32, 32, 3, 3), b2 (32,), W3 (K, 32, 3, 3), b3 (K,) as CUDA tensors,
    and their packed bfloat16 block."""

    NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, system: ShearletSystem, params: dict, device=None):
        import torch

        self.system = system
        self._lib = system._lib
        dev = device if device is not None else torch.device("cuda")
        K = system.K
        shapes = {"W1": (32, K, 3, 3), "b1": (32,), "W2": (32, 32, 3, 3), "b2": (32,), "W3": (K, 32, 3, 3), "b3": (K,)}
        n = self._lib.shear_shrink_param_count(K)
        if n < 0:
            raise ShearError(n, "shear_shrink_param_count", f"unsupported filter count {K}")
        # one flat FP32 buffer in the library's order; the named tensors are views of it
        self.flat = torch.empty(n, dtype=torch.float32, device=dev)
        self.params = {}
        o = 0
        for name in self.NAMES:
            t = torch.as_tensor(params[name], dtype=torch.float32, device=dev)
            if tuple(t.shape) != shapes[name]:
                raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shapes[name]}")
            view = self.flat[o:o + t.numel()].view(shapes[name])
            view.copy_(t)
            self.params[name] = view
            o += t.numel()
        assert o == n
        self.grads = torch.zeros(n, dtype=torch.float32, device=dev)
        self.adam = torch.zeros(2 * n, dtype=torch.float32, device=dev)
        self.steps = 0
        nb = ctypes.c_size_t()
        _check(self._lib.shear_shrink_params_bytes(K, ctypes.byref(nb)), "shear_shrink_params_bytes")
        self.packed = torch.empty(nb.value, dtype=torch.uint8, device=dev)
        self.pack()

    def pack(self, stream=None) -> None:
        """Re-packs the FP32 parameters (after they change) into the bfloat16 block."""
        p = [ctypes.c_void_p(self.params[n].data_ptr()) for n in self.NAMES]
        _check(self._lib.shear_shrink_pack(self.system._h, *p, ctypes.c_void_p(self.packed.data_ptr()),
                                           _stream_ptr(stream)), "shear_shrink_pack")

    def apply(self, coeffs, sigma, out=None, tau: bool = False, stream=None):
        """Shrunk coefficients (and the thresholds tau, noise units, when tau is True)."""
        import torch

        s = self.system
        B = coeffs.shape[0]
        s._check_tensor(coeffs, (B, s.K, s.rows, s.cols), "coeffs")
        sig = torch.as_tensor(sigma, dtype=torch.float32, device=coeffs.device)
        if sig.dim() == 0:
            sig = sig.expand(B)
        sig = sig.contiguous()
        s._check_tensor(sig, (B,), "sigma")
        if out is None:
            out = torch.empty_like(coeffs)
        s._check_tensor(out, (B, s.K, s.rows, s.cols), "out")
        t = torch.empty_like(coeffs) if tau else None
        _check(self._lib.shear_shrink_apply(s._h, ctypes.c_void_p(coeffs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                            ctypes.c_void_p(t.data_ptr()) if tau else None, B,
                                            ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(self.packed.data_ptr()),
                                            _stream_ptr(stream)), "shear_shrink_apply")
        return (out, t) if tau else out

    def train_step(self, c_noisy, c_clean, sigma, lr: float, temperature: float = 0.5, stream=None):
        """One Adam step on a batch of (noisy, clean) coefficient pairs (shear_shrink_train_step); returns the
        step's loss as a one-element CUDA tensor (not synchronised)."""
        import torch

        s = self.system
        B = c_noisy.shape[0]
        s._check_tensor(c_noisy, (B, s.K, s.rows, s.cols), "c_noisy")
        s._check_tensor(c_clean, (B, s.K, s.rows, s.cols), "c_clean")
        sig = torch.as_tensor(sigma, dtype=torch.float32, device=c_noisy.device)
        if sig.dim() == 0:
            sig = sig.expand(B)
        sig = sig.contiguous()
        loss = torch.empty(1, dtype=torch.float32, device=c_noisy.device)
        self.steps += 1
        _check(self._lib.shear_shrink_train_step(
            s._h, ctypes.c_void_p(c_noisy.data_ptr()), ctypes.c_void_p(c_clean.data_ptr()), B,
            ctypes.c_void_p(sig.data_ptr()), ctypes.c_void_p(self.flat.data_ptr()), ctypes.c_void_p(self.grads.data_ptr()),
            ctypes.c_void_p(self.adam.data_ptr()), ctypes.c_void_p(self.packed.data_ptr()), self.steps, float(lr),
            float(temperature), ctypes.c_void_p(loss.data_ptr()), _stream_ptr(stream)), "shear_shrink_train_step")
        return loss

    def grad(self, name: str):
        """The last step's gradient of one parameter (a view of the flat gradient buffer)."""
        o = 0
        for n in self.NAMES:
            t = self.params[n]
            if n == name:
                return self.grads[o:o + t.numel()].view(t.shape)
            o += t.numel()
        raise KeyError(name)
