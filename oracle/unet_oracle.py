"""Plain FP64 numpy reference of the warm-start 3D U-Net (forward, backward,
Adam).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the HIP network kernels
(on identical BF16-rounded operands) and pinned by finite differences and
brute-force loops in tests/test_unet_oracle.py.  Shares nothing with the
HIP implementation.

Layout: activations are channels-last arrays [D, H, W, C]; a 3x3x3 convolution
has weights W[tap, c_out, c_in] with tap = 9 (dz+1) + 3 (dy+1) + (dx+1),
zero padding 1, stride 1, and a bias b[c_out].

Network (3 levels, base width B): two 3x3x3 conv+ReLU per level, 2x2x2
average pooling down, nearest x2 upsampling up with the skip activation
concatenated after the upsampled channels, and a final 1x1x1 convolution.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def layer_specs(cin: int = 3, cout: int = 5, base: int = 32):
    """(name, c_in, c_out, kernel taps, relu) of every convolution, in order."""
    b1, b2, b3 = base, 2 * base, 4 * base
    return [
        ("e1a", cin, b1, 27, True), ("e1b", b1, b1, 27, True),
        ("e2a", b1, b2, 27, True), ("e2b", b2, b2, 27, True),
        ("b1", b2, b3, 27, True), ("b2", b3, b3, 27, True),
        ("d2a", b3 + b2, b2, 27, True), ("d2b", b2, b2, 27, True),
        ("d1a", b2 + b1, b1, 27, True), ("d1b", b1, b1, 27, True),
        ("out", b1, cout, 1, False),
    ]


def param_count(specs) -> int:
    return sum(t * co * ci + co for _, ci, co, t, _ in specs)


def unpack(theta, specs):
    """Flat parameter vector -> list of (W[taps, co, ci], b[co])."""
    out, o = [], 0
    for _, ci, co, t, _ in specs:
        n = t * co * ci
        W = theta[o:o + n].reshape(t, co, ci)
        o += n
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    return out


def init_params(specs, seed: int):
    """He-normal weights, zero biases, from a seeded generator (the random
    numbers are an input of both implementations)."""
    rng = np.random.default_rng(seed)
    parts = []
    for _, ci, co, t, _ in specs:
        std = np.sqrt(2.0 / (t * ci))
        parts.append(rng.standard_normal(t * co * ci) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)


# ------------------------------------------------------------------ ops

def conv3d(x, W, b):
    """y[v, o] = b[o] + sum_tap sum_i W[tap, o, i] x[v + tap, i] (zero outside)."""
    D, H, Wd, _ = x.shape
    taps = TAPS if W.shape[0] == 27 else [(0, 0, 0)]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((D, H, Wd, W.shape[1])) + b
    for t, (dz, dy, dx) in enumerate(taps):
        xs = xp[1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + Wd]
        y += np.einsum("dhwi,oi->dhwo", xs, W[t])
    return y


def conv3d_backward(x, W, gy):
    """Gradients of conv3d w.r.t. x, W, b for the upstream gradient gy."""
    D, H, Wd, _ = x.shape
    taps = TAPS if W.shape[0] == 27 else [(0, 0, 0)]
    xp = np.pad(x, ((1, 1), (1, 1), (1, 1), (0, 0)))
    gxp = np.zeros_like(xp)
    gW = np.zeros_like(W)
    for t, (dz, dy, dx) in enumerate(taps):
        sl = (slice(1 + dz, 1 + dz + D), slice(1 + dy, 1 + dy + H), slice(1 + dx, 1 + dx + Wd))
        gW[t] = np.einsum("dhwo,dhwi->oi", gy, xp[sl])
        gxp[sl] += np.einsum("dhwo,oi->dhwi", gy, W[t])
    gx = gxp[1:-1, 1:-1, 1:-1]
    gb = gy.sum(axis=(0, 1, 2))
    return gx, gW, gb


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    D, H, W, C = x.shape
    return x.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_backward(gy):
    return np.repeat(np.repeat(np.repeat(gy, 2, 0), 2, 1), 2, 2) / 8.0


def upsample2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, 0), 2, 1), 2, 2)


def upsample2_backward(gy):
    D, H, W, C = gy.shape
    return gy.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def mse(y, t, mask):
    """Mean over masked cells and channels of (y - t)^2, and its gradient."""
    n = mask.sum() * y.shape[-1]
    d = (y - t) * mask[..., None]
    return (d * d).sum() / n, 2.0 * d / n


# ------------------------------------------------------------ network

def forward(theta, x, specs, keep: bool = False):
    """Forward pass; returns the output and (if keep) the tape for backward."""
    P = unpack(theta, specs)
    tape = {}

    def conv(i, inp):
        W, b = P[i]
        pre = conv3d(inp, W, b)
        out = relu(pre) if specs[i][4] else pre
        tape[i] = (inp, pre)
        return out

    a = conv(0, x)
    s1 = conv(1, a)
    a = conv(2, avgpool2(s1))
    s2 = conv(3, a)
    a = conv(4, avgpool2(s2))
    a = conv(5, a)
    a = conv(6, np.concatenate([upsample2(a), s2], axis=-1))
    a = conv(7, a)
    a = conv(8, np.concatenate([upsample2(a), s1], axis=-1))
    a = conv(9, a)
    y = conv(10, a)
    return (y, tape) if keep else y


def backward(theta, tape, gy, specs):
    """Gradient of a scalar loss w.r.t. theta given dL/dy of the output."""
    P = unpack(theta, specs)
    grads = [None] * len(specs)

    def bconv(i, g):
        inp, pre = tape[i]
        if specs[i][4]:
            g = g * (pre > 0)
        gx, gW, gb = conv3d_backward(inp, P[i][0], g)
        grads[i] = (gW, gb)
        return gx

    b1, b2, b3 = specs[1][2], specs[3][2], specs[5][2]
    g = bconv(10, gy)
    g = bconv(9, g)
    g = bconv(8, g)                       # d1a input: [up(d2b), s1]
    g_up, g_s1 = g[..., :b2], g[..., b2:]
    g = bconv(7, upsample2_backward(g_up))
    g = bconv(6, g)                       # d2a input: [up(b2), s2]
    g_up, g_s2 = g[..., :b3], g[..., b3:]
    g = bconv(5, upsample2_backward(g_up))
    g = bconv(4, g)
    g = bconv(3, avgpool2_backward(g) + g_s2)
    g = bconv(2, g)
    g = bconv(1, avgpool2_backward(g) + g_s1)
    bconv(0, g)
    return np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected); returns new theta, m, v."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)
