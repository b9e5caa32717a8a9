"""Convolutional surrogate of the lattice update: a U-Net, forward and backward, numpy FP64.

TEST INFRASTRUCTURE (part of the oracle).  Only tests and the benchmark's CPU baseline use it.

The paper itself has no network; this is the learned part that advances the order parameter and
the velocity of the hybrid lattice Boltzmann / finite-difference method by a fixed number of
lattice steps.  The network maps the normalised fields (phi, u_x, u_y, T, a) on an H x W lattice
to the increments of (phi, u_x, u_y) over those steps (the channel counts are parameters of the
functions below; the tests also use other counts).

Architecture (L levels, widths w_1 .. w_L, default 4 levels of 32, 64, 128, 256 channels):
  encoder level l:   two 3x3 convolutions w_{l-1} -> w_l -> w_l, each followed by SiLU;
                     between levels a 2x2 average pool;
  decoder level l:   nearest-neighbour 2x upsampling of level l+1, concatenated (upsampled
                     channels first, then the encoder output of level l), then two 3x3
                     convolutions w_{l+1} + w_l -> w_l -> w_l with SiLU;
  head:              1x1 convolution w_1 -> 3, no activation.
Convolutions are cross-correlations: out[y, x] = b + sum over taps (dy, dx) in {-1, 0, 1}^2 of
W[tap] in[y + dy, x + dx], tap = 3 (dy + 1) + (dx + 1).  The lattice is periodic in x (as the
solver is); across y = 0 and y = H - 1 (the walls) the input is padded with zeros.

Parameter vector (FP32 on the device, FP64 here), in this order: for each 3x3 layer in the order
e1a, e1, e2a, e2, ..., eLa, eL, d(L-1)a, d(L-1), ..., d1a, d1: W as [9][C_out][C_in] then b as
[C_out]; then the head W as [3][w_1] and b as [3].

Loss: mean over all H * W * 3 outputs of (out - target)^2.

BF16 emulation (q=True): the device stores weights, activations and activation gradients in
bfloat16 and accumulates in FP32.  With q=True the same values are rounded to bfloat16 (round to
nearest, ties to even) at the same places: the packed input, the 3x3 weights, each convolution's
pre-activation z and output silu(z), pooled maps, and the activation gradients; the head weights
and the output stay FP32.  Sums are FP64 here, so what remains between the two is the order and
precision of the FP32 accumulation.
"""
from __future__ import annotations

import numpy as np

WIDTHS = (32, 64, 128, 256)
IN_CH = 5
OUT_CH = 3


def layers(widths=WIDTHS, in_ch=IN_CH):
    """(name, C_in, C_out) of the 3x3 layers in parameter order."""
    L = len(widths)
    out = []
    prev = in_ch
    for l in range(L):
        out.append((f"e{l + 1}a", prev, widths[l]))
        out.append((f"e{l + 1}", widths[l], widths[l]))
        prev = widths[l]
    for l in range(L - 2, -1, -1):
        out.append((f"d{l + 1}a", widths[l + 1] + widths[l], widths[l]))
        out.append((f"d{l + 1}", widths[l], widths[l]))
    return out


def param_count(widths=WIDTHS, in_ch=IN_CH, out_ch=OUT_CH) -> int:
    n = sum(9 * ci * co + co for _, ci, co in layers(widths, in_ch))
    return n + out_ch * widths[0] + out_ch


def split(theta, widths=WIDTHS, in_ch=IN_CH, out_ch=OUT_CH) -> dict:
    """Views of the parameter vector: name -> (W, b)."""
    theta = np.asarray(theta)
    p, o = {}, 0
    for name, ci, co in layers(widths, in_ch):
        W = theta[o:o + 9 * co * ci].reshape(9, co, ci)
        o += 9 * co * ci
        p[name] = (W, theta[o:o + co])
        o += co
    Wh = theta[o:o + out_ch * widths[0]].reshape(out_ch, widths[0])
    o += out_ch * widths[0]
    p["head"] = (Wh, theta[o:o + out_ch])
    o += out_ch
    assert o == theta.size
    return p


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.ascontiguousarray(np.asarray(x, np.float64).astype(np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64).reshape(a.shape)


def _shift(x, dy, dx):
    """s[y, x] = x[y + dy, (x + dx) mod W], zero where y + dy is outside [0, H)."""
    H = x.shape[0]
    s = np.roll(x, -dx, axis=1)
    out = np.zeros_like(x)
    lo, hi = max(0, -dy), min(H, H - dy)
    out[lo:hi] = s[lo + dy:hi + dy]
    return out


def conv3x3(x, W, b):
    """x [H, W, C_in], W [9, C_out, C_in], b [C_out] -> [H, W, C_out]."""
    out = np.broadcast_to(b, x.shape[:2] + (W.shape[1],)).copy()
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            out += _shift(x, dy, dx) @ W[3 * (dy + 1) + (dx + 1)].T
    return out


def conv3x3_input_grad(g, W):
    """Adjoint of conv3x3 with respect to its input: g [H, W, C_out] -> [H, W, C_in]."""
    out = np.zeros(g.shape[:2] + (W.shape[2],))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            out += _shift(g, -dy, -dx) @ W[3 * (dy + 1) + (dx + 1)]
    return out


def conv3x3_weight_grad(x, g):
    """Gradient of <g, conv3x3(x, W, b)> with respect to W and b."""
    dW = np.empty((9, g.shape[2], x.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            s = _shift(x, dy, dx)
            dW[3 * (dy + 1) + (dx + 1)] = g.reshape(-1, g.shape[2]).T @ s.reshape(-1, s.shape[2])
    return dW, g.sum(axis=(0, 1))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def pool(x):
    H, W, C = x.shape
    return x.reshape(H // 2, 2, W // 2, 2, C).mean(axis=(1, 3))


def up(x):
    return np.repeat(np.repeat(x, 2, axis=0), 2, axis=1)


def forward(theta, x, widths=WIDTHS, q=False, out_ch=OUT_CH):
    """x [H, W, C_in] -> (out [H, W, out_ch], cache for backward)."""
    r = bf16 if q else (lambda v: v)
    P = split(theta, widths, x.shape[2], out_ch)
    L = len(widths)
    cache = {"x": r(x)}

    def conv(name, inp):
        W, b = P[name]
        z = conv3x3(inp, r(W), b)
        y = r(silu(z))
        cache[name] = (inp, r(z))
        return y

    h = cache["x"]
    skips = []
    for l in range(L):
        h = conv(f"e{l + 1}", conv(f"e{l + 1}a", h))
        skips.append(h)
        if l < L - 1:
            h = r(pool(h))
    for l in range(L - 2, -1, -1):
        h = np.concatenate([up(h), skips[l]], axis=2)
        h = conv(f"d{l + 1}", conv(f"d{l + 1}a", h))
    Wh, bh = P["head"]
    cache["head"] = h
    return h @ Wh.T + bh, cache


def loss(out, target):
    return float(np.mean((out - target) ** 2))


def backward(theta, cache, out, target, widths=WIDTHS, q=False, g_extra=None):
    """Gradient of loss(out, target) with respect to theta and the input x.  With g_extra
    ([H, W, out_ch]) the gradient is that of loss(out, target) + sum(g_extra * out): g_extra is the
    gradient of a later use of the output (the chain rule through several surrogate steps)."""
    r = bf16 if q else (lambda v: v)
    in_ch = cache["x"].shape[2]
    out_ch = out.shape[2]
    P = split(theta, widths, in_ch, out_ch)
    grad = np.zeros_like(np.asarray(theta, np.float64))
    G = split(grad, widths, in_ch, out_ch)
    L = len(widths)
    g_out = 2.0 * (out - target) / out.size
    if g_extra is not None:
        g_out = g_out + g_extra
    Wh, _ = P["head"]
    h = cache["head"]
    G["head"][0][...] = g_out.reshape(-1, out_ch).T @ h.reshape(-1, h.shape[2])
    G["head"][1][...] = g_out.sum(axis=(0, 1))
    g = g_out @ Wh  # gradient with respect to the output of d1 (or eL when L = 1)

    def conv_back(name, g_y):
        """g_y: gradient w.r.t. silu(z) of layer `name`; returns the gradient w.r.t. its input
        (unrounded)."""
        inp, z = cache[name]
        W, _ = P[name]
        g_z = r(g_y * dsilu(z))
        dW, db = conv3x3_weight_grad(inp, g_z)
        G[name][0][...] = dW
        G[name][1][...] = db
        return conv3x3_input_grad(g_z, r(W))

    # Rounding points follow the device: a 3x3 input gradient that feeds a SiLU layer is multiplied
    # by silu'(z) before it is stored (one rounding); one that feeds a concatenation or a pool is
    # stored as it is and combined afterwards.
    skip_grads = [None] * L
    for l in range(L - 1):
        g = r(conv_back(f"d{l + 1}a", conv_back(f"d{l + 1}", g)))
        c_up = widths[l + 1]
        skip_grads[l] = g[:, :, c_up:]
        g_up = g[:, :, :c_up]
        H, W_, C = g_up.shape
        g = g_up.reshape(H // 2, 2, W_ // 2, 2, C).sum(axis=(1, 3))
    for l in range(L - 1, -1, -1):
        if l < L - 1:
            # output of level l feeds the pool (to level l + 1) and the skip connection
            g = skip_grads[l] + up(g) / 4.0
        g = r(conv_back(f"e{l + 1}a", conv_back(f"e{l + 1}", g)))
    return grad, g


def adam(theta, m, v, grad, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba, 2015) with bias correction; t counts from 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
