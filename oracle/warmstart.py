"""Oracle: the learned warm start's encoder-decoder, its gradient and Adam.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The network maps a source sampled on a G x G grid of the interior box (two
channels: real and imaginary part) to a guess of k^2 u on the same grid
(two channels); the guess divided by k^2 starts GMRES.  Five levels:

    e0 = relu(conv(x, We0))                  G      c0
    el = relu(conv(pool(e_{l-1}), Wel))      G/2^l  cl      l = 1..4
    d3 = relu(conv(up(e4) + e3, Wd3))        G/8    c2      (c3 == c4)
    d2 = relu(conv(up(d3) + e2, Wd2))        G/4    c1
    d1 = relu(conv(up(d2) + e1, Wd1))        G/2    c0
    d0 = relu(conv(up(d1) + e0, Wd0))        G      c0
    y  = conv(d0, Wh)                        G      2

conv: 3 x 3, zero padding, no bias; weights W[ky][kx][cin][cout] with
out[y, x] = sum_{ky,kx} in[y + ky - 1, x + kx - 1] W[ky, kx]; pool: mean of
2 x 2 blocks; up: nearest-neighbour doubling.  Tensors are (batch, y, x, c).
Loss: mean squared error over every output value.  Everything in float64;
the backward pass is written out by hand (reverse order of the forward).
"""
from __future__ import annotations

import numpy as np

NAMES = ("e0", "e1", "e2", "e3", "e4", "d3", "d2", "d1", "d0", "head")


def shapes(channels):
    """(cin, cout) of every convolution for level widths c0..c4 (c3 == c4)."""
    c0, c1, c2, c3, c4 = channels
    assert c3 == c4, "the deepest skip adds e3 to the upsampled e4"
    return {"e0": (2, c0), "e1": (c0, c1), "e2": (c1, c2), "e3": (c2, c3), "e4": (c3, c4),
            "d3": (c4, c2), "d2": (c2, c1), "d1": (c1, c0), "d0": (c0, c0), "head": (c0, 2)}


def conv(x, W):
    """out[b, y, x, o] = sum_{ky, kx, i} x[b, y + ky - 1, x + kx - 1, i] W[ky, kx, i, o]."""
    B, H, Wd, _ = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, x.shape[3]))
    xp[:, 1:-1, 1:-1, :] = x
    out = np.zeros((B, H, Wd, W.shape[3]))
    for ky in range(3):
        for kx in range(3):
            out += np.einsum("byxi,io->byxo", xp[:, ky:ky + H, kx:kx + Wd, :], W[ky, kx])
    return out


def conv_grad_input(dout, W):
    """d loss / d x of conv: dx[b, y, x, i] = sum_{ky, kx, o} dout[b, y - ky + 1, x - kx + 1, o] W[ky, kx, i, o]."""
    B, H, Wd, _ = dout.shape
    dxp = np.zeros((B, H + 2, Wd + 2, W.shape[2]))
    for ky in range(3):
        for kx in range(3):
            dxp[:, ky:ky + H, kx:kx + Wd, :] += np.einsum("byxo,io->byxi", dout, W[ky, kx])
    return dxp[:, 1:-1, 1:-1, :]


def conv_grad_weight(x, dout):
    """d loss / d W of conv: dW[ky, kx, i, o] = sum_{b, y, x} x[b, y + ky - 1, x + kx - 1, i] dout[b, y, x, o]."""
    B, H, Wd, ci = x.shape
    xp = np.zeros((B, H + 2, Wd + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    dW = np.zeros((3, 3, ci, dout.shape[3]))
    for ky in range(3):
        for kx in range(3):
            dW[ky, kx] = np.einsum("byxi,byxo->io", xp[:, ky:ky + H, kx:kx + Wd, :], dout)
    return dW


def pool(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool_grad(dout):
    return np.repeat(np.repeat(dout, 2, axis=1), 2, axis=2) / 4.0


def up(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up_grad(dout):
    B, H, W, C = dout.shape
    return dout.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def relu(z):
    return np.maximum(z, 0.0)


def forward(params, x):
    """Returns the output and every intermediate the backward pass needs."""
    t = {"x": x}
    t["e0"] = relu(conv(x, params["e0"]))
    prev = t["e0"]
    for l in range(1, 5):
        t["p%d" % l] = pool(prev)
        t["e%d" % l] = relu(conv(t["p%d" % l], params["e%d" % l]))
        prev = t["e%d" % l]
    skips = {3: "e3", 2: "e2", 1: "e1", 0: "e0"}
    for l in (3, 2, 1, 0):
        t["s%d" % l] = up(prev) + t[skips[l]]
        t["d%d" % l] = relu(conv(t["s%d" % l], params["d%d" % l]))
        prev = t["d%d" % l]
    t["y"] = conv(prev, params["head"])
    return t["y"], t


def loss(y, target):
    return float(np.mean((y - target) ** 2))


def backward(params, t, target):
    """Gradient of the mean squared error with respect to every weight."""
    g = {}
    dy = 2.0 * (t["y"] - target) / t["y"].size
    g["head"] = conv_grad_weight(t["d0"], dy)
    dprev = conv_grad_input(dy, params["head"])            # d loss / d d0
    dskip = {}
    skips = {3: "e3", 2: "e2", 1: "e1", 0: "e0"}
    below = {3: "e4", 2: "d3", 1: "d2", 0: "d1"}
    for l in (0, 1, 2, 3):
        dz = dprev * (t["d%d" % l] > 0)
        g["d%d" % l] = conv_grad_weight(t["s%d" % l], dz)
        ds = conv_grad_input(dz, params["d%d" % l])
        dskip[skips[l]] = ds
        dprev = up_grad(ds)                                # d loss / d (level below)
    # dprev is now d loss / d e4 (through the decoder); encoder from the bottom
    de = dprev
    for l in (4, 3, 2, 1):
        if l < 4:
            de = de + dskip["e%d" % l]
        dz = de * (t["e%d" % l] > 0)
        g["e%d" % l] = conv_grad_weight(t["p%d" % l], dz)
        dp = conv_grad_input(dz, params["e%d" % l])
        de = pool_grad(dp)                                 # d loss / d e_{l-1}
    de = de + dskip["e0"]
    dz = de * (t["e0"] > 0)
    g["e0"] = conv_grad_weight(t["x"], dz)
    return g


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, with bias correction); step counts from 1."""
    out_p, out_m, out_v = {}, {}, {}
    for k in params:
        out_m[k] = beta1 * m[k] + (1 - beta1) * grads[k]
        out_v[k] = beta2 * v[k] + (1 - beta2) * grads[k] ** 2
        mh = out_m[k] / (1 - beta1 ** step)
        vh = out_v[k] / (1 - beta2 ** step)
        out_p[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
    return out_p, out_m, out_v
