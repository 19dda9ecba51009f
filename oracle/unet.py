"""FP64 reference of the denoiser network -- test infrastructure only.

The paper has no denoiser: this network is the project's addition (a learned
filter over low-sample accumulation tiles, with plain accumulation as the
fallback where the per-tile variance is high).  Its architecture is a
project choice, written out here as the definition the GPU kernels must
reproduce:

  input  x = [mean R, G, B, A, log(tile variance), 1/n]      (6 channels)
  enc1   conv3x3  6->32, ReLU; conv3x3 32->32, ReLU          -> s1
  enc2   avgpool2; conv3x3 32->64, ReLU; conv3x3 64->64, ReLU -> s2
  enc3   avgpool2; conv3x3 64->128, ReLU; conv3x3 128->128, ReLU
  dec2   nearest-up2; conv3x3 128->64, ReLU; concat [., s2];
         conv3x3 128->64, ReLU; conv3x3 64->64, ReLU
  dec1   nearest-up2; conv3x3 64->32, ReLU; concat [., s1];
         conv3x3 64->32, ReLU; conv3x3 32->32, ReLU
  out    conv1x1 32->3, added to the mean RGB (a residual)
  loss   mean squared error over pixels and RGB

conv3x3 is the plain definition (cross-correlation, zero padding 1):
  y[n, r, c, o] = b[o] + sum_{dr, dc in 0..2, i} x[n, r + dr - 1, c + dc - 1, i] W[dr, dc, i, o]
Every step below is that definition or its derivative, with a matrix
product (numpy) per tap as the only library primitive.

With ``bf16=True`` values are rounded to bfloat16 exactly where the GPU
stores or multiplies bfloat16: the network input, the conv3x3 weights, every
conv3x3 output, every pooled map, and the gradient operands of the backward
products (dY of dgrad and wgrad).  Rounding: float64 -> float32 (nearest
even) -> bfloat16 (nearest even), by bit manipulation.
"""
from __future__ import annotations

import numpy as np

CONV3 = [  # (name, c_in, c_out)
    ("enc1a", 6, 32), ("enc1b", 32, 32),
    ("enc2a", 32, 64), ("enc2b", 64, 64),
    ("enc3a", 64, 128), ("enc3b", 128, 128),
    ("up2", 128, 64), ("dec2a", 128, 64), ("dec2b", 64, 64),
    ("up1", 64, 32), ("dec1a", 64, 32), ("dec1b", 32, 32),
]
OUT = ("out", 32, 3)
IN_CH = 6


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def init_params(seed=0):
    """He-normal conv3x3 weights, zero biases, small 1x1 output weights, as
    float32 master values (the GPU keeps the same)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, ci, co in CONV3:
        p[name + ".w"] = (rng.standard_normal((3, 3, ci, co)) * np.sqrt(2.0 / (9 * ci))).astype(np.float32)
        p[name + ".b"] = np.zeros(co, dtype=np.float32)
    name, ci, co = OUT
    p[name + ".w"] = (rng.standard_normal((ci, co)) * 0.01).astype(np.float32)
    p[name + ".b"] = np.zeros(co, dtype=np.float32)
    return p


def _round(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def conv3x3(x, w, b):
    """Definition above; x [N,H,W,Ci], w [3,3,Ci,Co], b [Co] -> [N,H,W,Co]."""
    N, H, W, _ = x.shape
    xp = np.zeros((N, H + 2, W + 2, x.shape[3]))
    xp[:, 1:H + 1, 1:W + 1] = x
    y = np.broadcast_to(np.asarray(b, dtype=np.float64), (N, H, W, w.shape[3])).copy()
    for dr in range(3):
        for dc in range(3):
            y += xp[:, dr:dr + H, dc:dc + W, :] @ w[dr, dc]
    return y


def conv3x3_backward(x, w, dy):
    """Gradients of conv3x3 w.r.t. x, w and b for upstream dy."""
    N, H, W, Ci = x.shape
    xp = np.zeros((N, H + 2, W + 2, Ci))
    xp[:, 1:H + 1, 1:W + 1] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w, dtype=np.float64)
    for dr in range(3):
        for dc in range(3):
            dxp[:, dr:dr + H, dc:dc + W, :] += dy @ w[dr, dc].T
            dw[dr, dc] = np.tensordot(xp[:, dr:dr + H, dc:dc + W, :], dy, axes=([0, 1, 2], [0, 1, 2]))
    return dxp[:, 1:H + 1, 1:W + 1], dw, dy.sum(axis=(0, 1, 2))


def avgpool2(x):
    N, H, W, C = x.shape
    return x.reshape(N, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(dy):
    N, H, W, C = dy.shape
    return dy.reshape(N, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


def forward(params, x, mean_rgb, *, bf16_on=True):
    """Returns (output RGB [N,H,W,3], cache of every activation by name)."""
    r = lambda a: _round(a, bf16_on)
    wq = {n: r(params[n + ".w"]) for n, _, _ in CONV3}
    c = {"x": r(x)}

    def cr(name, inp):
        y = conv3x3(inp, wq[name], params[name + ".b"])
        y = r(np.maximum(y, 0.0))
        c[name] = y
        return y

    s1 = cr("enc1b", cr("enc1a", c["x"]))
    c["pool1"] = r(avgpool2(s1))
    s2 = cr("enc2b", cr("enc2a", c["pool1"]))
    c["pool2"] = r(avgpool2(s2))
    h3 = cr("enc3b", cr("enc3a", c["pool2"]))
    u2 = cr("up2", up2(h3))
    c["cat2"] = np.concatenate([u2, s2], axis=3)
    d2 = cr("dec2b", cr("dec2a", c["cat2"]))
    u1 = cr("up1", up2(d2))
    c["cat1"] = np.concatenate([u1, s1], axis=3)
    d1 = cr("dec1b", cr("dec1a", c["cat1"]))
    out = np.asarray(mean_rgb, dtype=np.float64) + d1 @ params["out.w"].astype(np.float64) \
        + params["out.b"].astype(np.float64)
    c["out"] = out
    return out, c


def mse(out, target):
    return float(np.mean((out - np.asarray(target, dtype=np.float64)) ** 2))


def backward(params, cache, target, *, bf16_on=True):
    """Gradients of the MSE loss w.r.t. every parameter (dict like params)."""
    r = lambda a: _round(a, bf16_on)
    wq = {n: r(params[n + ".w"]) for n, _, _ in CONV3}
    g = {}
    out = cache["out"]
    dout = 2.0 * (out - np.asarray(target, dtype=np.float64)) / out.size
    d1 = cache["dec1b"]
    g["out.w"] = np.tensordot(d1, dout, axes=([0, 1, 2], [0, 1, 2]))
    g["out.b"] = dout.sum(axis=(0, 1, 2))
    dh = dout @ params["out.w"].astype(np.float64).T

    def back(name, inp, dy):
        dy = dy * (cache[name] > 0)            # ReLU
        g[name + ".b"] = dy.sum(axis=(0, 1, 2))
        dyq = r(dy)
        dx, dw, _ = conv3x3_backward(inp, wq[name], dyq)
        g[name + ".w"] = dw
        return dx

    dh = back("dec1b", cache["dec1a"], dh)
    dcat1 = back("dec1a", cache["cat1"], dh)
    du1, ds1 = dcat1[..., :32], dcat1[..., 32:]
    dd2 = up2_backward(back("up1", up2(cache["dec2b"]), du1))
    dh = back("dec2b", cache["dec2a"], dd2)
    dcat2 = back("dec2a", cache["cat2"], dh)
    du2, ds2 = dcat2[..., :64], dcat2[..., 64:]
    dh3 = up2_backward(back("up2", up2(cache["enc3b"]), du2))
    dh = back("enc3b", cache["enc3a"], dh3)
    dp2 = back("enc3a", cache["pool2"], dh)
    ds2 = ds2 + avgpool2_backward(dp2)
    dh = back("enc2b", cache["enc2a"], ds2)
    dp1 = back("enc2a", cache["pool1"], dh)
    ds1 = ds1 + avgpool2_backward(dp1)
    dh = back("enc1b", cache["enc1a"], ds1)
    back("enc1a", cache["x"], dh)
    return g


def adam_step(params, grads, state, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of float32 master values (Kingma & Ba), bias-corrected
    with step t >= 1.  ``state`` holds m and v per parameter (float64)."""
    out = {}
    for k, w in params.items():
        m, v = state.get(k, (np.zeros(w.shape), np.zeros(w.shape)))
        gk = np.asarray(grads[k], dtype=np.float64)
        m = beta1 * m + (1 - beta1) * gk
        v = beta2 * v + (1 - beta2) * gk * gk
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        out[k] = (w.astype(np.float64) - lr * mh / (np.sqrt(vh) + eps)).astype(np.float32)
        state[k] = (m, v)
    return out


# ---------------------------------------------------------------- frame glue
def frame_input(mu_tiles, tile_var, n, width, height, tile_w, tile_h):
    """Network input of a compositor accumulation: per image pixel
    [mean R, G, B, A, log(v_t), 1/n], log(v_t) with v_t floored at 1e-12 and
    0 while n < 2 (no variance measured yet).  mu_tiles [T, P, 4]."""
    tiles_x = -(-width // tile_w)
    out = np.zeros((height, width, 6))
    for y in range(height):
        for x in range(width):
            t = (y // tile_h) * tiles_x + x // tile_w
            q = (y % tile_h) * tile_w + x % tile_w
            out[y, x, :4] = mu_tiles[t, q]
            out[y, x, 4] = np.log(max(tile_var[t], 1e-12)) if n >= 2 else 0.0
            out[y, x, 5] = 1.0 / n
    return out


def select(mu_tiles, tile_var, out_rgb, n, tau, width, height, tile_w, tile_h):
    """Per tile: the plain mean where the measured variance exceeds tau
    (n >= 2 and v_t > tau), else the network's RGB with the mean's alpha."""
    tiles_x = -(-width // tile_w)
    res = np.array(mu_tiles, dtype=np.float64, copy=True)
    for t in range(res.shape[0]):
        if n >= 2 and tile_var[t] > tau:
            continue
        for q in range(res.shape[1]):
            y = (t // tiles_x) * tile_h + q // tile_w
            x = (t % tiles_x) * tile_w + q % tile_w
            if x < width and y < height:
                res[t, q, :3] = out_rgb[y, x]
    return res
