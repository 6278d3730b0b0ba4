"""Learned surrogate forecast (float64 reference on BF16-rounded operands).

The paper has no learned component; the surrogate is a small convolutional network that
stands in for the 5-minute model forecast between analyses, with the plain solver as its
fallback.  Definition (the reference for the GPU kernels):

  input      psi = (eta, hu, hv) per cell, normalised x = (psi - mu) / sigma per channel
  network    six 3x3 convolutions with periodic padding, 3 -> 48 -> 48 -> 48 -> 48 -> 48 -> 3,
             ReLU after the first five; operands (weights, layer inputs) rounded to BF16
             (round to nearest even), sums and bias in FP32 on the GPU / FP64 here
  output     psi' = psi + s * net(x), s per channel
  loss       MSE of net(x) against (psi_target - psi) / s over cells and channels
  training   Adam (lr, beta1 0.9, beta2 0.999, eps 1e-8) on FP32 master weights
  guard      relative mass drift |sum h' - sum h| / sum h, h = H + eta; above a threshold the
             particle is re-stepped by the plain solver

Layouts: activations [C][H][W] here (NHWC on the GPU); weights [C_out][C_in][3][3], tap
(ky, kx) applies to input cell (y + ky - 1, x + kx - 1) (cross-correlation, as torch).
"""
from __future__ import annotations

import numpy as np

CHANNELS = (3, 48, 48, 48, 48, 48, 3)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest BF16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[o, y, x] = b[o] + sum_{c, ky, kx} w[o, c, ky, kx] x[c, y + ky - 1, x + kx - 1]
    with periodic indices.  x [C_in, H, W], w [C_out, C_in, 3, 3], b [C_out]."""
    cin, H, W = x.shape
    out = np.zeros((w.shape[0], H, W)) + b[:, None, None]
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(np.roll(x, -(ky - 1), axis=1), -(kx - 1), axis=2)  # xs[c,y,x] = x[c,y+ky-1,x+kx-1]
            out += np.einsum("oc,chw->ohw", w[:, :, ky, kx], xs)
    return out


def conv3x3_input_grad(gy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient of sum(gy * conv3x3(x, w, b)) with respect to x (periodic)."""
    cout, H, W = gy.shape
    gx = np.zeros((w.shape[1], H, W))
    for ky in range(3):
        for kx in range(3):
            t = np.einsum("oc,ohw->chw", w[:, :, ky, kx], gy)
            gx += np.roll(np.roll(t, ky - 1, axis=1), kx - 1, axis=2)
    return gx


def conv3x3_weight_grad(gy: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Gradient of sum(gy * conv3x3(x, w, b)) with respect to w."""
    gw = np.zeros((gy.shape[0], x.shape[0], 3, 3))
    for ky in range(3):
        for kx in range(3):
            xs = np.roll(np.roll(x, -(ky - 1), axis=1), -(kx - 1), axis=2)
            gw[:, :, ky, kx] = np.einsum("ohw,chw->oc", gy, xs)
    return gw


def init_params(rng: np.random.Generator, last_scale: float = 0.1):
    """He-style initial weights (FP32 master copies) and zero biases."""
    params = []
    for i in range(6):
        cin, cout = CHANNELS[i], CHANNELS[i + 1]
        std = np.sqrt(2.0 / (9 * cin)) * (last_scale if i == 5 else 1.0)
        w = (rng.normal(size=(cout, cin, 3, 3)) * std).astype(np.float32).astype(np.float64)
        params.append((w, np.zeros(cout)))
    return params


def forward(params, x: np.ndarray):
    """Network on a normalised input x [3, H, W].  Returns (output, cache) where cache holds
    the BF16-rounded input of every layer and the pre-activations."""
    a = bf16_round(x)
    cache = []
    for i, (w, b) in enumerate(params):
        wq = bf16_round(w)
        z = conv3x3(a, wq, b)
        cache.append((a, wq, z))
        if i < 5:
            a = bf16_round(np.maximum(z, 0.0))
        else:
            a = z
    return a, cache


def backward(params, cache, gout: np.ndarray, round_grads: bool = False):
    """Gradients of sum(gout * net(x)) for every (w, b); the BF16 rounding of the
    operands is treated as identity (straight-through), as in mixed-precision training.
    round_grads: the gradient with respect to every layer's pre-activation (and the loss
    gradient) is rounded to BF16 before it multiplies weights or activations, which is the
    mixed-precision backward the GPU kernels implement."""
    grads = [None] * 6
    g = bf16_round(gout) if round_grads else gout
    for i in reversed(range(6)):
        a, wq, z = cache[i]
        if i < 5:
            g = g * (z > 0)
            if round_grads:
                g = bf16_round(g)
        gw = conv3x3_weight_grad(g, a)
        gb = g.sum(axis=(1, 2))
        grads[i] = (gw, gb)
        if i > 0:
            g = conv3x3_input_grad(g, wq)
    return grads


def mse_loss_and_grad(pred: np.ndarray, target: np.ndarray):
    """L = mean((pred - target)^2) and dL/dpred."""
    d = pred - target
    n = d.size
    return float(np.sum(d * d) / n), 2.0 * d / n


class Adam:
    """Adam on FP32 master weights: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
    p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [[np.zeros_like(w), np.zeros_like(b)] for w, b in params]
        self.v = [[np.zeros_like(w), np.zeros_like(b)] for w, b in params]

    def step(self, params, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for i, (pw, gw) in enumerate(zip(params, grads)):
            new = []
            for j in range(2):
                g = gw[j]
                self.m[i][j] = self.b1 * self.m[i][j] + (1 - self.b1) * g
                self.v[i][j] = self.b2 * self.v[i][j] + (1 - self.b2) * g * g
                new.append(pw[j] - self.lr * (self.m[i][j] / c1) /
                           (np.sqrt(self.v[i][j] / c2) + self.eps))
            out.append(tuple(new))
        return out


def apply(params, psi: np.ndarray, mu, sigma, s):
    """psi' = psi + s * net((psi - mu) / sigma) for one state [3, H, W]."""
    x = (psi - np.asarray(mu)[:, None, None]) / np.asarray(sigma)[:, None, None]
    y, _ = forward(params, x)
    return psi + np.asarray(s)[:, None, None] * y


def mass_drift(psi_in: np.ndarray, psi_out: np.ndarray, H: float) -> float:
    """|sum (H + eta_out) - sum (H + eta_in)| / sum (H + eta_in)."""
    a = np.sum(H + psi_in[0])
    b = np.sum(H + psi_out[0])
    return float(abs(b - a) / a)
