"""FP64 reference of the dispersion-corrector CNN -- TEST INFRASTRUCTURE ONLY.

A 3x3x3 convolution with zero padding on channel-last volumes x[z, y, x, ci]:
    y[v, co] = bias[co] + sum over taps t and ci of w[t, co, ci] x[v + d_t, ci],
tap t = 9 (dz+1) + 3 (dy+1) + (dx+1).  The network is three such layers, with ReLU after the first
two or none at all (a linear network); the loss is
    L = 1/2 sum over voxels v and the first two output channels of w_v (out - target)^2,
    w_v = weight * mask[v]   (mask: None for 1 everywhere, else a per-voxel array >= 0).
Gradients follow the chain rule: dL/dout = w_v (out - target) on those channels, then per layer
dW_t[co, ci] = sum_v dz[v, co] x[v + d_t, ci], db = sum_v dz, the data gradient
dx[v, ci] = sum_t sum_co dz[v - d_t, co] w[t, co, ci], and the ReLU derivative (y > 0) where a
ReLU follows the layer.  Plain numpy; no code shared with the HIP path.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def _shift(x, d):
    """x shifted so that result[v] = x[v + d] with zeros outside (x: [nz, ny, nx, c])."""
    dz, dy, dx = d
    nz, ny, nx = x.shape[:3]
    p = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    return p[1 + dz:1 + dz + nz, 1 + dy:1 + dy + ny, 1 + dx:1 + dx + nx]


def conv3d(x, w, bias=None, relu=False):
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, d in enumerate(TAPS):
        y += _shift(x, d) @ w[t].T
    if bias is not None:
        y += np.asarray(bias, dtype=np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv3d_wgrad(x, dz):
    """dW[t, co, ci] = sum_v dz[v, co] x[v + d_t, ci];  db[co] = sum_v dz[v, co]."""
    x = np.asarray(x, dtype=np.float64)
    dz = np.asarray(dz, dtype=np.float64)
    c_out, c_in = dz.shape[-1], x.shape[-1]
    dw = np.zeros((27, c_out, c_in))
    for t, d in enumerate(TAPS):
        dw[t] = dz.reshape(-1, c_out).T @ _shift(x, d).reshape(-1, c_in)
    return dw, dz.reshape(-1, c_out).sum(axis=0)


def conv3d_dgrad(dz, w):
    """dx[v, ci] = sum_t sum_co dz[v - d_t, co] w[t, co, ci]."""
    dz = np.asarray(dz, dtype=np.float64)
    dx = np.zeros(dz.shape[:3] + (w.shape[2],))
    for t, (a, b, c) in enumerate(TAPS):
        dx += _shift(dz, (-a, -b, -c)) @ np.asarray(w[t], dtype=np.float64)
    return dx


def forward(x, params, relu: bool = True):
    """params: [(w1, b1), (w2, b2), (w3, b3)]; ReLU after the first two layers when relu is True.
    Returns (out, activations)."""
    acts = [np.asarray(x, dtype=np.float64)]
    h = acts[0]
    for li, (w, b) in enumerate(params):
        h = conv3d(h, w, b, relu=relu and li < 2)
        acts.append(h)
    return h, acts


def loss_and_grads(x, target, params, channels: int = 2, relu: bool = True, mask=None, weight: float = 1.0):
    """L = 1/2 sum_v w_v sum over the first `channels` outputs of (out - target)^2, with
    w_v = weight * mask[v] (mask None: 1), and its parameter gradients."""
    out, acts = forward(x, params, relu)
    wv = np.full(out.shape[:3], float(weight))
    if mask is not None:
        wv = wv * np.asarray(mask, dtype=np.float64).reshape(out.shape[:3])
    err = np.zeros_like(out)
    err[..., :channels] = out[..., :channels] - np.asarray(target, dtype=np.float64)[..., :channels]
    loss = 0.5 * float(np.sum(wv[..., None] * err * err))
    dy = wv[..., None] * err
    grads = [None] * 3
    dz = dy
    for li in (2, 1, 0):
        if li < 2 and relu:
            dz = dz * (acts[li + 1] > 0)
        dw, db = conv3d_wgrad(acts[li], dz)
        grads[li] = (dw, db)
        if li > 0:
            dz = conv3d_dgrad(dz, params[li][0])
    return loss, grads
