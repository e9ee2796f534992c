"""Plain FP64 numpy reference of the learned warm start's network (test infrastructure only).

The network is not part of the paper: it is the added form that proposes a starting velocity for
the Newton--Krylov solve.  This module writes it out directly from its definition so that the
GPU kernels can be checked element by element:

  * 3x3 convolution with periodic padding (the images live on the torus):
        y[b, i, j, o] = bias[o] + sum_{dy, dx in {-1,0,1}} sum_c x[b, i+dy, j+dx, c] w[t, o, c],
    t = 3 (dy + 1) + (dx + 1), indices modulo the grid;
  * ReLU, 2x2 average pooling, nearest-neighbour upsampling by 2, channel concatenation;
  * a U-Net: `levels` resolutions, `base` channels doubling per level, two conv + ReLU per level,
    skips concatenated as (upsampled, skip), a linear 3x3 output convolution to 2 channels;
  * mean squared error against a target velocity, its gradient by hand-written backpropagation
    (chain rule, layer by layer), and one Adam step (Kingma & Ba, bias-corrected).

Parameters are one flat array laid out as the C ABI documents it: per layer (encoder levels
fine to coarse, then decoder levels coarse to fine, then the output layer) W[9][cout][cin] then
bias[cout], each padded to a multiple of 64 values; then the scalar head (w[2 C_top], bias[1],
each padded to 64), which maps the per-channel pixel means and maxima of the coarsest level's
output to one number per item (the learned log(beta (e_max - 1)) of the two-level
preconditioner).  The input has 32 channels (m_R, m_T,
m_R - m_T, zeros) and the output layer 32 (two used); a network built for small tests may use
any channel counts.

With bf16=True every value the GPU stores in BF16 (inputs, weights, each layer's output, each
activation gradient) is rounded to BF16 (round to nearest even) at the same point, so that the
remaining difference to the GPU is the order of its FP32 sums.  With bf16=False everything is
FP64: that is the form the pins (finite differences, scipy correlation) check.
"""

from __future__ import annotations

import math

import numpy as np

IN_C = 32
OUT_C = 32


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    x32 = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = x32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _pad64(n):
    return (n + 63) // 64 * 64


class Arch:
    """Layer table of the U-Net: (cin, cout, relu, level) per layer and parameter offsets."""

    def __init__(self, height, width, levels=4, base=32, in_c=IN_C, out_c=OUT_C):
        self.H, self.W, self.L, self.base = height, width, levels, base
        self.C = [base << l for l in range(levels)]
        self.layers = []   # dict(cin, cout, relu, level, woff, boff)
        self.n = 0
        self.enc_a, self.enc_b, self.dec_a, self.dec_b = {}, {}, {}, {}
        for l in range(levels):
            self.enc_a[l] = self._add(in_c if l == 0 else self.C[l - 1], self.C[l], True, l)
            self.enc_b[l] = self._add(self.C[l], self.C[l], True, l)
        for l in range(levels - 2, -1, -1):
            self.dec_a[l] = self._add(self.C[l + 1] + self.C[l], self.C[l], True, l)
            self.dec_b[l] = self._add(self.C[l], self.C[l], True, l)
        self.out = self._add(self.C[0], out_c, False, 0)
        self.in_c, self.out_c = in_c, out_c
        # scalar head after the convolution layers: w[2 C_top] (means, maxima), bias[1], each padded
        self.trunk_n = self.n
        self.hw_off = self.n
        self.n += _pad64(2 * self.C[-1])
        self.hb_off = self.n
        self.n += 64

    def _add(self, cin, cout, relu, level):
        woff = self.n
        self.n += _pad64(9 * cout * cin)
        boff = self.n
        self.n += _pad64(cout)
        self.layers.append(dict(cin=cin, cout=cout, relu=relu, level=level, woff=woff, boff=boff))
        return len(self.layers) - 1

    def weights(self, params, k):
        ly = self.layers[k]
        w = params[ly["woff"]: ly["woff"] + 9 * ly["cout"] * ly["cin"]].reshape(9, ly["cout"], ly["cin"])
        b = params[ly["boff"]: ly["boff"] + ly["cout"]]
        return w, b


def _shift(x, dy, dx):
    """s[b, i, j] = x[b, i + dy, j + dx] (periodic)."""
    return np.roll(x, shift=(-dy, -dx), axis=(1, 2))


def conv3x3(x, w, b):
    """Periodic 3x3 convolution of x [B, H, W, cin] with w [9, cout, cin] plus bias [cout]."""
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        y += np.einsum("bhwc,oc->bhwo", _shift(x, dy, dx), w[t])
    return y + b


def conv3x3_backward(x, w, dy_):
    """Gradients of conv3x3: (dx, dw, db) for upstream gradient dy_ [B, H, W, cout]."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t in range(9):
        dy, dxs = t // 3 - 1, t % 3 - 1
        xs = _shift(x, dy, dxs)
        dw[t] = np.einsum("bhwo,bhwc->oc", dy_, xs)
        # y[p] gets x[p + d] w: so x[q] receives dy_[q - d] w
        dx += _shift(np.einsum("bhwo,oc->bhwc", dy_, w[t]), -dy, -dxs)
    return dx, dw, dy_.sum(axis=(0, 1, 2))


def pool(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_backward(dy_):
    return 0.25 * np.repeat(np.repeat(dy_, 2, axis=1), 2, axis=2)


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_backward(dy_):
    B, H, W, C = dy_.shape
    return dy_.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def make_input(mR, mT, in_c=IN_C):
    """Network input [B, H, W, in_c]: (m_R, m_T, m_R - m_T, zeros)."""
    mR = np.asarray(mR, dtype=np.float64)
    mT = np.asarray(mT, dtype=np.float64)
    x = np.zeros(mR.shape + (in_c,))
    x[..., 0] = mR
    x[..., 1] = mT
    if in_c > 2:
        x[..., 2] = mR.astype(np.float32) - mT.astype(np.float32)  # formed in FP32, as on the GPU
    return x


def forward(arch, params, mR, mT, bf16=False):
    """Velocity v [B, 2, H, W] and the cache of every activation (for backward)."""
    rnd = bf16_round if bf16 else (lambda a: a)
    p = rnd(params) if bf16 else params
    x0 = rnd(make_input(mR, mT, arch.in_c))
    cache = {"x0": x0, "params": p}

    def layer(k, x):
        w, b = arch.weights(p, k)
        bb = arch.weights(params, k)[1]  # biases are applied from the FP32 master copy
        z = conv3x3(x, w, bb)
        return np.maximum(z, 0.0) if arch.layers[k]["relu"] else z

    L = arch.L
    feats = {}
    x = x0
    for l in range(L):
        xin = x
        ea = rnd(layer(arch.enc_a[l], xin))
        eb = rnd(layer(arch.enc_b[l], ea))
        feats[l] = (xin, ea, eb)
        if l < L - 1:
            x = rnd(pool(eb))
    low = feats[L - 1][2]
    dec = {}
    for l in range(L - 2, -1, -1):
        cat = np.concatenate([up(low), feats[l][2]], axis=-1)
        da = rnd(layer(arch.dec_a[l], cat))
        db = rnd(layer(arch.dec_b[l], da))
        dec[l] = (cat, da, db)
        low = db
    out = layer(arch.out, low)  # FP32 output, no rounding
    top = feats[L - 1][2]
    f = np.concatenate([top.mean(axis=(1, 2)), top.max(axis=(1, 2))], axis=1)   # [B, 2 C_top]
    head = f @ params[arch.hw_off: arch.hw_off + 2 * arch.C[-1]] + params[arch.hb_off]
    cache.update(feats=feats, dec=dec, last=low, pooled=f, head=head)
    v = np.moveaxis(out[..., :2], -1, 1)
    return v, cache


def head_grad(arch, cache, y):
    """Loss mean_b (head_b - y_b)^2 and its gradient with respect to the head's parameters only
    (flat, arch layout; the convolution layers get none)."""
    d = cache["head"] - np.asarray(y, dtype=np.float64)
    g = np.zeros(arch.n)
    B = d.size
    g[arch.hw_off: arch.hw_off + 2 * arch.C[-1]] = (2.0 * d / B) @ cache["pooled"]
    g[arch.hb_off] = np.sum(2.0 * d / B)
    return float(np.mean(d * d)), g


def mse(v, target):
    d = np.asarray(v, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def backward(arch, cache, dv, bf16=False):
    """Gradient of a scalar loss with respect to every parameter (flat, arch layout), given
    dL/dv [B, 2, H, W]."""
    rnd = bf16_round if bf16 else (lambda a: a)
    p = cache["params"]
    grads = np.zeros(arch.n)
    L = arch.L
    feats, dec = cache["feats"], cache["dec"]

    def back(k, x, y, g):
        ly = arch.layers[k]
        w, _ = arch.weights(p, k)
        if ly["relu"]:
            g = g * (y > 0)
        dx, dw, db = conv3x3_backward(x, w, g)
        grads[ly["woff"]: ly["woff"] + dw.size] = dw.ravel()
        grads[ly["boff"]: ly["boff"] + db.size] = db
        return dx

    gout = np.zeros(cache["last"].shape[:3] + (arch.out_c,))
    gout[..., :2] = np.moveaxis(dv, 1, -1)
    gout = rnd(gout)
    g = rnd(back(arch.out, cache["last"], None, gout))
    for l in range(0, L - 1):
        cat, da, db = dec[l]
        g = rnd(back(arch.dec_b[l], da, db, g))
        gcat = rnd(back(arch.dec_a[l], cat, da, g))
        c_low = arch.C[l + 1]
        dec[l] = (cat, da, db, gcat[..., c_low:])
        g = rnd(up_backward(gcat[..., :c_low]))
    # g: gradient of the bottleneck output
    gin_next = None
    for l in range(L - 1, -1, -1):
        xin, ea, eb = feats[l]
        if l < L - 1:
            g = rnd(dec[l][3] + pool_backward(gin_next))
        gea = rnd(back(arch.enc_b[l], ea, eb, g))
        gx = back(arch.enc_a[l], xin, ea, gea)
        gin_next = rnd(gx)
        g = None
    return grads


def adam_step(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** step)
    vh = v / (1.0 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


def random_params(arch, rng, scale=1.0):
    """He-scaled normal parameters (real channels only; padded channels zero) for tests."""
    w = np.zeros(arch.n)
    for k, ly in enumerate(arch.layers):
        cin_real = 3 if k == arch.enc_a[0] else ly["cin"]
        cout_real = 2 if k == arch.out else ly["cout"]
        a = scale * math.sqrt(2.0 / (9.0 * cin_real))
        W = np.zeros((9, ly["cout"], ly["cin"]))
        W[:, :cout_real, :cin_real] = a * rng.standard_normal((9, cout_real, cin_real))
        w[ly["woff"]: ly["woff"] + W.size] = W.ravel()
        b = np.zeros(ly["cout"])
        b[:cout_real] = 0.05 * rng.standard_normal(cout_real)
        w[ly["boff"]: ly["boff"] + b.size] = b
    return w
