"""Oracle: learned shrinkage of shearlet coefficients, FP64 (test infrastructure only).

A small convolutional network maps the coefficients of a noisy image to one
threshold per coefficient; coefficients below their threshold are set to zero
and the image is reconstructed (the hard thresholding of Section 4.2 with
learned, spatially varying thresholds). The paper has no such network; its
definition here is the workload's:

  z_k   = c_k / (sigma RMS_k)                       noise-normalised coefficients
  h1    = relu(conv3x3(z;  W1 [32 x K  x 3 x 3]) + b1)
  h2    = relu(conv3x3(h1; W2 [32 x 32 x 3 x 3]) + b2)
  o     = conv3x3(h2; W3 [K x 32 x 3 x 3]) + b3
  tau_k = softplus(o_k)   (0 for the low-pass plane, which is kept)
  c'_k  = c_k if |z_k| >= tau_k else 0

conv3x3 is a cross-correlation with circular boundary (the coefficient planes
are periodic): out[co](y, x) = sum_{ci, dy, dx} W[co, ci, dy, dx] in[ci](y+dy-1, x+dx-1).
The network computes with bfloat16 operands and FP32 accumulation; the
oracle rounds the same operands to bfloat16 (z, the weights, h1, h2) and
accumulates in FP64. Biases, o and tau are not rounded.

Training objective (not in the paper; the workload's): the hard threshold is
replaced by a smooth gate so that it can be differentiated,
  g = sigmoid((|z| - tau) / T),   z_hat = z g,
  L = scale * sum over images, band planes (not the low-pass) and pixels of (z_hat - z_clean)^2,
z_clean the noise-normalised coefficients of the clean image. ``train_loss``
returns L and its gradients by the chain rule (rounding points treated as the
identity, as the kernels do; with ``rounded`` the gradients flowing back are
rounded to bfloat16 where the kernels store them).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "to_bf16",
    "softplus",
    "conv3x3_circular",
    "ShrinkParams",
    "init_params",
    "thresholds",
    "shrink",
    "conv3x3_adjoint",
    "train_loss",
]


def to_bf16(x: np.ndarray) -> np.ndarray:
    """Rounds to the nearest bfloat16 (8-bit exponent, 8-bit significand), ties to even; returned as
    float64 (exact). Goes through float32 first, as the kernels do."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def softplus(x: np.ndarray) -> np.ndarray:
    """log(1 + e^x), computed without overflow."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def conv3x3_circular(x: np.ndarray, W: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """out[co](y, x) = b[co] + sum_{ci,dy,dx} W[co, ci, dy, dx] x[ci]((y + dy - 1) mod N, (x + dx - 1) mod M)."""
    x = np.asarray(x, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    cout = W.shape[0]
    out = np.zeros((cout,) + x.shape[1:])
    for dy in range(3):
        for dx in range(3):
            shifted = np.roll(x, shift=(1 - dy, 1 - dx), axis=(1, 2))  # shifted[ci](y, x) = x[ci](y+dy-1, x+dx-1)
            out += np.einsum("oc,cyx->oyx", W[:, :, dy, dx], shifted)
    if b is not None:
        out += np.asarray(b, dtype=np.float64)[:, None, None]
    return out


class ShrinkParams:
    """Weights (bfloat16-representable) and biases of the three layers."""

    def __init__(self, W1, b1, W2, b2, W3, b3):
        self.W1, self.W2, self.W3 = (to_bf16(w) for w in (W1, W2, W3))
        self.b1, self.b2, self.b3 = (np.asarray(v, dtype=np.float32).astype(np.float64) for v in (b1, b2, b3))

    @property
    def K(self) -> int:
        return self.W1.shape[1]


def init_params(K: int, hidden: int = 32, seed: int = 0, tau0: float = 3.0) -> ShrinkParams:
    """Seeded initial parameters: small random weights and an output bias with softplus(b3) = tau0,
    so the untrained network is close to hard thresholding at tau0."""
    rng = np.random.default_rng(seed)

    def he(cout, cin):
        return rng.standard_normal((cout, cin, 3, 3)) * np.sqrt(2.0 / (9 * cin))

    b3 = np.full(K, np.log(np.expm1(tau0)))
    return ShrinkParams(he(hidden, K), np.zeros(hidden), he(hidden, hidden), np.zeros(hidden),
                        0.1 * he(K, hidden), b3)


def thresholds(c: np.ndarray, sigma: float, rms: np.ndarray, p: ShrinkParams, lowpass: int | None = None) -> np.ndarray:
    """tau (K, N, M) in noise units for the coefficients c (K, N, M) of one image; the low-pass plane
    (index ``lowpass``, default the last) gets 0."""
    c = np.asarray(c, dtype=np.float64)
    K = c.shape[0]
    lp = K - 1 if lowpass is None else lowpass
    scale = 1.0 / (float(sigma) * np.asarray(rms, dtype=np.float64))
    z = to_bf16(c * scale[:, None, None])
    h1 = to_bf16(np.maximum(conv3x3_circular(z, p.W1, p.b1), 0.0))
    h2 = to_bf16(np.maximum(conv3x3_circular(h1, p.W2, p.b2), 0.0))
    o = conv3x3_circular(h2, p.W3, p.b3)
    tau = softplus(o)
    tau[lp] = 0.0
    return tau


def shrink(c: np.ndarray, sigma: float, rms: np.ndarray, p: ShrinkParams, lowpass: int | None = None):
    """(c', tau): c'_k = c_k where |c_k| / (sigma RMS_k) >= tau_k, else 0."""
    c = np.asarray(c, dtype=np.float64)
    tau = thresholds(c, sigma, rms, p, lowpass)
    z = c / (float(sigma) * np.asarray(rms, dtype=np.float64))[:, None, None]
    return np.where(np.abs(z) >= tau, c, 0.0), tau


def conv3x3_adjoint(d: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of conv3x3_circular in its input: out[ci](y, x) = sum_{co,dy,dx} W[co, ci, dy, dx] d[co](y-dy+1, x-dx+1)."""
    d = np.asarray(d, dtype=np.float64)
    W = np.asarray(W, dtype=np.float64)
    out = np.zeros((W.shape[1],) + d.shape[1:])
    for dy in range(3):
        for dx in range(3):
            out += np.einsum("oc,oyx->cyx", W[:, :, dy, dx], np.roll(d, shift=(dy - 1, dx - 1), axis=(1, 2)))
    return out


def _wgrad(d: np.ndarray, x: np.ndarray) -> np.ndarray:
    """dW[co, ci, dy, dx] = sum_{y,x} d[co](y, x) x[ci](y+dy-1, x+dx-1)."""
    out = np.zeros((d.shape[0], x.shape[0], 3, 3))
    for dy in range(3):
        for dx in range(3):
            out[:, :, dy, dx] = np.einsum("oyx,cyx->oc", d, np.roll(x, shift=(1 - dy, 1 - dx), axis=(1, 2)))
    return out


def _sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def train_loss(c_noisy, c_clean, sigma, rms, p: ShrinkParams, temperature: float, scale: float,
               rounded: bool = True, lowpass: int | None = None):
    """(L, grads dict W1, b1, W2, b2, W3, b3) for one image (K, N, M) of noise level sigma."""
    r = (lambda v: to_bf16(v)) if rounded else (lambda v: v)
    c_noisy = np.asarray(c_noisy, dtype=np.float64)
    K = c_noisy.shape[0]
    lp = K - 1 if lowpass is None else lowpass
    sc = 1.0 / (float(sigma) * np.asarray(rms, dtype=np.float64))[:, None, None]
    z = c_noisy * sc
    zc = np.asarray(c_clean, dtype=np.float64) * sc
    zb = r(z)
    a1 = conv3x3_circular(zb, p.W1, p.b1)
    h1 = r(np.maximum(a1, 0.0))
    a2 = conv3x3_circular(h1, p.W2, p.b2)
    h2 = r(np.maximum(a2, 0.0))
    o = conv3x3_circular(h2, p.W3, p.b3)
    tau = softplus(o)
    g = _sigmoid((np.abs(z) - tau) / temperature)
    res = z * g - zc
    band = np.ones(K, dtype=bool)
    band[lp] = False
    L = float(scale * np.sum(res[band] ** 2))
    do = 2.0 * scale * res * z * g * (1.0 - g) * (-1.0 / temperature) * _sigmoid(o)
    do[lp] = 0.0
    do = r(do)
    grads = {"W3": _wgrad(do, h2), "b3": do.sum(axis=(1, 2))}
    dh2 = r(conv3x3_adjoint(do, p.W3) * (h2 > 0))
    grads["W2"] = _wgrad(dh2, h1)
    grads["b2"] = dh2.sum(axis=(1, 2))
    dh1 = r(conv3x3_adjoint(dh2, p.W2) * (h1 > 0))
    grads["W1"] = _wgrad(dh1, zb)
    grads["b1"] = dh1.sum(axis=(1, 2))
    return L, grads
