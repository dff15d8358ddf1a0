"""1D convolutional network of the learned preconditioner stage (oracle; test infrastructure only).

The paper has no learned component; this is the FP64 reference of the small
network the GPU library trains and applies as an extra flexible-GMRES stage:
L layers of 1D convolution along the interface coordinate (kernel K, stride
1, dilation d_l of layer l: taps at offsets (k - K//2) d_l, zero padding),
ReLU after every layer but the last.  Shapes: activations (batch, channels,
n); weights (c_out, c_in, K); biases (c_out,).

Functions: forward (keeping the activations), backward (gradients of the
loss with respect to every weight and bias), and the loss used for training,
the mean over samples of ||y_b - t_b||^2 / (||t_b||^2 + tiny).

Pinned by tests/test_oracle_cnn.py: central finite differences of the loss
on 3-layer toys (with and without dilation), a one-layer network against a
direct convolution with numpy's correlate (dilated: against the correlation
with the zero-stuffed kernel), and translation properties.
"""
from __future__ import annotations

import numpy as np

TINY = 1e-30


def conv1d(x: np.ndarray, w: np.ndarray, b: np.ndarray, d: int = 1) -> np.ndarray:
    """y[b, o, i] = bias[o] + sum_{c,k} w[o, c, k] x[b, c, i + (k - K//2) d] (zero outside 0..n-1)."""
    B, C, n = x.shape
    O, C2, K = w.shape
    assert C == C2
    p = (K // 2) * d
    xp = np.zeros((B, C, n + 2 * p), dtype=np.float64)
    xp[:, :, p:p + n] = x
    y = np.zeros((B, O, n), dtype=np.float64) + b[None, :, None]
    for k in range(K):
        y += np.einsum("oc,bcn->bon", w[:, :, k], xp[:, :, k * d:k * d + n])
    return y


def forward(params, x: np.ndarray, dil=None):
    """params: list of (w, b); dil: dilation per layer (default 1).  Returns the output and the list of
    layer inputs/outputs."""
    dil = dil or [1] * len(params)
    acts = [x]
    h = x
    for li, (w, b) in enumerate(params):
        h = conv1d(h, w, b, dil[li])
        if li < len(params) - 1:
            h = np.maximum(h, 0.0)
        acts.append(h)
    return h, acts


def loss(y: np.ndarray, t: np.ndarray) -> float:
    B = y.shape[0]
    num = ((y - t) ** 2).reshape(B, -1).sum(axis=1)
    den = (t ** 2).reshape(B, -1).sum(axis=1) + TINY
    return float(np.mean(num / den))


def loss_grad(y: np.ndarray, t: np.ndarray) -> np.ndarray:
    B = y.shape[0]
    den = (t ** 2).reshape(B, -1).sum(axis=1) + TINY
    return 2.0 * (y - t) / den[:, None, None] / B


def backward(params, acts, dy: np.ndarray, dil=None):
    """Gradients [(dw, db), ...] of the loss given dL/d(output) = dy (dil as in forward)."""
    dil = dil or [1] * len(params)
    grads = [None] * len(params)
    g = dy
    for li in range(len(params) - 1, -1, -1):
        w, b = params[li]
        x = acts[li]
        d = dil[li]
        if li < len(params) - 1:
            g = g * (acts[li + 1] > 0.0)  # ReLU'(pre) = [post > 0]
        O, C, K = w.shape
        p = (K // 2) * d
        n = x.shape[2]
        xp = np.zeros((x.shape[0], C, n + 2 * p))
        xp[:, :, p:p + n] = x
        dw = np.zeros_like(w)
        for k in range(K):
            dw[:, :, k] = np.einsum("bon,bcn->oc", g, xp[:, :, k * d:k * d + n])
        db = g.sum(axis=(0, 2))
        gp = np.zeros((x.shape[0], C, n + 2 * p))
        for k in range(K):
            gp[:, :, k * d:k * d + n] += np.einsum("oc,bon->bcn", w[:, :, k], g)
        grads[li] = (dw, db)
        g = gp[:, :, p:p + n]
    return grads


def init_params(channels=(8, 32, 32, 32, 8), K=5, seed=0):
    rng = np.random.default_rng(seed)
    ps = []
    for ci, co in zip(channels[:-1], channels[1:]):
        ps.append((rng.standard_normal((co, ci, K)) * np.sqrt(2.0 / (ci * K)), np.zeros(co)))
    return ps


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (round half to even on the float32 bits)."""
    f = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (f >> 16) & 1
    r = ((f + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
