"""FP64 oracle of the warm-start network's building blocks.  Test infrastructure only.

Not part of the paper: the warm start is a convolutional network that maps a normalised
backprojection to an initial image for Algorithm 2.  These are the plain definitions the
GPU kernels are compared with, written as explicit sums (channel-last volumes
[y][x][z][C], 3x3x3 kernels with zero padding, tap = (dy+1)*9 + (dx+1)*3 + (dz+1),
weights [tap][co][ci]).
"""
from __future__ import annotations

import numpy as np

TAPS = [(dy, dx, dz) for dy in (-1, 0, 1) for dx in (-1, 0, 1) for dz in (-1, 0, 1)]


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _shifted(x, dy, dx, dz):
    """s[v] = x[v + (dy, dx, dz)], zero outside."""
    ny, nx, nz = x.shape[:3]
    out = np.zeros_like(x)
    ys, yd = slice(max(0, dy), ny + min(0, dy)), slice(max(0, -dy), ny + min(0, -dy))
    xs, xd = slice(max(0, dx), nx + min(0, dx)), slice(max(0, -dx), nx + min(0, -dx))
    zs, zd = slice(max(0, dz), nz + min(0, dz)), slice(max(0, -dz), nz + min(0, -dz))
    out[yd, xd, zd] = x[ys, xs, zs]
    return out


def conv3d(x, w, b=None, relu=False):
    """y[v, co] = b[co] + sum_{tap, ci} w[tap, co, ci] x[v + off(tap), ci]."""
    x = np.asarray(x, np.float64)
    w = np.asarray(w, np.float64)
    y = np.zeros(x.shape[:3] + (w.shape[1],))
    for t, (dy, dx, dz) in enumerate(TAPS):
        y += _shifted(x, dy, dx, dz) @ w[t].T
    if b is not None:
        y += np.asarray(b, np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv3d_input_grad(dy, w):
    """Adjoint of conv3d in x: dx[u, ci] = sum_{tap, co} w[tap, co, ci] dy[u - off(tap), co]."""
    dy = np.asarray(dy, np.float64)
    w = np.asarray(w, np.float64)
    dx = np.zeros(dy.shape[:3] + (w.shape[2],))
    for t, (a, b, c) in enumerate(TAPS):
        dx += _shifted(dy, -a, -b, -c) @ w[t]
    return dx


def conv3d_weight_grad(x, dy):
    """dw[tap, co, ci] = sum_v dy[v, co] x[v + off(tap), ci]; db[co] = sum_v dy[v, co]."""
    x = np.asarray(x, np.float64)
    dy = np.asarray(dy, np.float64)
    ci, co = x.shape[3], dy.shape[3]
    dw = np.zeros((27, co, ci))
    for t, (a, b, c) in enumerate(TAPS):
        dw[t] = dy.reshape(-1, co).T @ _shifted(x, a, b, c).reshape(-1, ci)
    return dw, dy.reshape(-1, co).sum(axis=0)


def pool2(x):
    """2x2x2 average pooling (even sizes)."""
    ny, nx, nz, c = x.shape
    return np.asarray(x, np.float64).reshape(ny // 2, 2, nx // 2, 2, nz // 2, 2, c).mean(axis=(1, 3, 5))


def pool2_adjoint(g):
    return np.repeat(np.repeat(np.repeat(np.asarray(g, np.float64), 2, 0), 2, 1), 2, 2) / 8.0


def up2(x):
    """Nearest 2x upsampling."""
    return np.repeat(np.repeat(np.repeat(np.asarray(x, np.float64), 2, 0), 2, 1), 2, 2)


def up2_adjoint(g):
    ny, nx, nz, c = g.shape
    return np.asarray(g, np.float64).reshape(ny // 2, 2, nx // 2, 2, nz // 2, 2, c).sum(axis=(1, 3, 5))


def adam(p, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma & Ba 2015, Algorithm 1)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- the encoder-decoder
# (name, cin, cout, relu): the same layer list as the network under test
LAYERS = [("c1", 16, 16, 1), ("c2", 16, 16, 1), ("c3", 16, 32, 1), ("c4", 32, 32, 1),
          ("c5", 32, 64, 1), ("c6", 64, 64, 1), ("c7", 64, 32, 1), ("c8", 32, 32, 1),
          ("c9", 32, 16, 1), ("c10", 16, 16, 1), ("c11", 16, 16, 0)]


def network_forward(img, scale, w, b, rnd=bf16_round):
    """Forward pass of the 3-level encoder-decoder on an image [y][x][z]; activations are
    rounded with `rnd` where the network stores them.  Returns (output image, activations)."""
    spec = {n: (ci, co, relu) for n, ci, co, relu in LAYERS}
    a = {}
    x = np.zeros(img.shape + (16,))
    x[..., 0] = rnd(scale * np.asarray(img, np.float64))
    a["in"] = x

    def conv(n, inp):
        return rnd(conv3d(inp, w[n], b[n], relu=bool(spec[n][2])))

    a["c1"] = conv("c1", a["in"]); a["e1"] = conv("c2", a["c1"])
    a["p1"] = rnd(pool2(a["e1"])); a["c3"] = conv("c3", a["p1"]); a["e2"] = conv("c4", a["c3"])
    a["p2"] = rnd(pool2(a["e2"])); a["c5"] = conv("c5", a["p2"]); a["b"] = conv("c6", a["c5"])
    a["u2"] = up2(a["b"]); a["c7"] = conv("c7", a["u2"]); a["s2"] = rnd(a["c7"] + a["e2"])
    a["d2"] = conv("c8", a["s2"]); a["u1"] = up2(a["d2"]); a["c9"] = conv("c9", a["u1"])
    a["s1"] = rnd(a["c9"] + a["e1"]); a["d1"] = conv("c10", a["s1"]); a["out"] = conv("c11", a["d1"])
    out = (a["out"][..., 0] + scale * np.asarray(img, np.float64)) / scale
    return out, a


def network_gradients(img, target, scale, w, b, rnd=bf16_round):
    """Loss 0.5 sum (p - scale target)^2, p = out channel 0 + scale img, and its exact
    gradients (FP64 backpropagation through the forward activations of network_forward)."""
    spec = {n: (ci, co, relu) for n, ci, co, relu in LAYERS}
    _, a = network_forward(img, scale, w, b, rnd)
    p = a["out"][..., 0] + scale * np.asarray(img, np.float64)
    res = p - scale * np.asarray(target, np.float64)
    loss = 0.5 * float(np.sum(res * res))
    grads = {}
    g = np.zeros(a["out"].shape)
    g[..., 0] = res

    def back(n, inp, outp, gout):
        if spec[n][2]:
            gout = gout * (outp > 0)
        grads[n + ".w"], grads[n + ".b"] = conv3d_weight_grad(inp, gout)
        return conv3d_input_grad(gout, w[n])

    g = back("c11", a["d1"], a["out"], g)
    g_s1 = back("c10", a["s1"], a["d1"], g)
    g = up2_adjoint(back("c9", a["u1"], a["c9"], g_s1))
    g_s2 = back("c8", a["s2"], a["d2"], g)
    g = up2_adjoint(back("c7", a["u2"], a["c7"], g_s2))
    g = back("c6", a["c5"], a["b"], g)
    g = pool2_adjoint(back("c5", a["p2"], a["c5"], g)) + g_s2
    g = back("c4", a["c3"], a["e2"], g)
    g = pool2_adjoint(back("c3", a["p1"], a["c3"], g)) + g_s1
    g = back("c2", a["c1"], a["e1"], g)
    back("c1", a["in"], a["c1"], g)
    return loss, grads
