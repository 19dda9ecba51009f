"""Pins of the FP64 denoiser oracle (oracle/unet.py): the conv definition
against scipy's 2-D correlation, the analytic backward against central
finite differences (no bfloat16 rounding), the bfloat16 rounding against
torch's float32 -> bfloat16 conversion, Adam against its constant-gradient
limit and two hand-worked steps, and the frame glue (network input and the
per-tile fallback) on a hand-built ragged tile grid."""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import unet


def test_conv3x3_is_zero_padded_cross_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    y = unet.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(signal.correlate2d(x[n, :, :, i], w[:, :, i, o], mode="same", boundary="fill")
                             for i in range(3))
            np.testing.assert_allclose(y[n, :, :, o], ref, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 65504.0, 1e-30]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)
    assert np.array_equal(unet.bf16(x32), ref)
    assert unet.bf16(1.0 + 2 ** -8) == 1.0           # tie -> even
    assert unet.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6


def test_backward_matches_central_differences():
    rng = np.random.default_rng(2)
    p = unet.init_params(3)
    for k in p:
        if k.endswith(".b"):
            p[k] = (rng.standard_normal(p[k].shape) * 0.05).astype(np.float32)
    p["out.w"] = (rng.standard_normal(p["out.w"].shape) * 0.3).astype(np.float32)
    p64 = {k: v.astype(np.float64) for k, v in p.items()}
    x = rng.standard_normal((2, 8, 8, unet.IN_CH))
    mean_rgb = rng.standard_normal((2, 8, 8, 3))
    target = rng.standard_normal((2, 8, 8, 3))
    out, cache = unet.forward(p64, x, mean_rgb, bf16_on=False)
    g = unet.backward(p64, cache, target, bf16_on=False)
    h = 1e-6
    checked = 0
    for k in sorted(p64):
        flat = p64[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp = unet.mse(unet.forward(p64, x, mean_rgb, bf16_on=False)[0], target)
            flat[idx] = old - h
            lm = unet.mse(unet.forward(p64, x, mean_rgb, bf16_on=False)[0], target)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(abs(fd), 1e-3), (k, idx, fd, an)
            checked += 1
    assert checked >= 70


def test_adam_constant_gradient_moves_by_lr():
    p = {"a": np.array([1.0, -2.0, 0.5], dtype=np.float32)}
    gr = {"a": np.array([0.3, -5.0, 1e-3])}
    state = {}
    q = p
    for t in range(1, 6):
        q = unet.adam_step(q, gr, state, t, lr=0.01)
    np.testing.assert_allclose(q["a"], p["a"] - 5 * 0.01 * np.sign(gr["a"]), rtol=0, atol=2e-5)


def test_architecture_parameter_count():
    p = unet.init_params(0)
    n = sum(v.size for v in p.values())
    assert 500_000 < n < 540_000


# ---------------------------------------------------------------- Adam, two steps
def test_adam_two_steps_distinguish_the_moments():
    """Two Adam steps with different gradients (1, then -2) on one scalar,
    beta1 = 0.9, beta2 = 0.999, lr = 0.01, eps = 1e-8 (Kingma & Ba's
    definition).  The moments, worked out by hand:
      step 1: m = 0.1, v = 0.001; corrected m = 0.1/0.1 = 1, v = 0.001/0.001 = 1
      step 2: m = 0.9*0.1 + 0.1*(-2) = -0.11,  v = 0.999*0.001 + 0.001*4 = 0.004999
              corrected m = -0.11/(1 - 0.81) = -11/19
              corrected v = 0.004999/(1 - 0.998001) = 4999/1999
    With beta1 and beta2 swapped, step 1 is the same but step 2 gives
    corrected m = -0.001001/0.001999 and v = 0.49/0.19, a different update."""
    p = {"a": np.array([0.5], dtype=np.float32)}
    state = {}
    q = unet.adam_step(p, {"a": np.array([1.0])}, state, 1, lr=0.01)
    w1 = np.float32(0.5 - 0.01 * 1.0 / (1.0 + 1e-8))
    assert q["a"][0] == w1
    m, v = state["a"]
    assert abs(m[0] - 0.1) < 1e-15 and abs(v[0] - 0.001) < 1e-15
    q = unet.adam_step(q, {"a": np.array([-2.0])}, state, 2, lr=0.01)
    m, v = state["a"]
    assert abs(m[0] - (-0.11)) < 1e-15 and abs(v[0] - 0.004999) < 1e-15
    w2 = np.float32(np.float64(w1) - 0.01 * (-11 / 19) / (math.sqrt(4999 / 1999) + 1e-8))
    assert q["a"][0] == w2
    swapped = np.float32(np.float64(w1) - 0.01 * (-0.001001 / 0.001999) / (math.sqrt(0.49 / 0.19) + 1e-8))
    assert abs(float(swapped) - float(w2)) > 1e-4     # the pin separates the two readings


# ---------------------------------------------------------------- frame glue
# A 5 x 3 frame in 2 x 2 tiles: 3 x 2 tiles, the right column and the bottom
# row cut by the image edge.  Tile ids are row-major, pixels row-major inside
# a tile.  Every image pixel's (tile, pixel-in-tile), written out by hand:
GLUE_W, GLUE_H, GLUE_TW, GLUE_TH = 5, 3, 2, 2
GLUE_MAP = {  # (y, x): (t, q)
    (0, 0): (0, 0), (0, 1): (0, 1), (0, 2): (1, 0), (0, 3): (1, 1), (0, 4): (2, 0),
    (1, 0): (0, 2), (1, 1): (0, 3), (1, 2): (1, 2), (1, 3): (1, 3), (1, 4): (2, 2),
    (2, 0): (3, 0), (2, 1): (3, 1), (2, 2): (4, 0), (2, 3): (4, 1), (2, 4): (5, 0),
}


def _glue_tiles():
    # mean of tile t, pixel q, channel c = 1000 t + 10 q + c: every entry distinct
    mu = np.zeros((6, 4, 4))
    for t in range(6):
        for q in range(4):
            for c in range(4):
                mu[t, q, c] = 1000 * t + 10 * q + c
    return mu


def test_frame_input_places_every_tile_pixel():
    mu = _glue_tiles()
    var = np.array([1.0, np.exp(2.0), 1e-15, 0.0, np.exp(-3.0), 7.0])
    x = unet.frame_input(mu, var, 2, GLUE_W, GLUE_H, GLUE_TW, GLUE_TH)
    assert x.shape == (3, 5, 6)
    # log of the tile's variance, floored at 1e-12 (tiles 2 and 3)
    log_v = [0.0, 2.0, math.log(1e-12), math.log(1e-12), -3.0, math.log(7.0)]
    for (y, xx), (t, q) in GLUE_MAP.items():
        assert list(x[y, xx, :4]) == [1000 * t + 10 * q + c for c in range(4)], (y, xx)
        assert abs(x[y, xx, 4] - log_v[t]) < 1e-12, (y, xx)
        assert x[y, xx, 5] == 0.5


def test_frame_input_has_no_variance_channel_before_two_frames():
    mu = _glue_tiles()
    var = np.array([np.inf, 3.0, 1e-15, 0.0, 5.0, 7.0])   # n = 1: nothing is measured yet
    x = unet.frame_input(mu, var, 1, GLUE_W, GLUE_H, GLUE_TW, GLUE_TH)
    assert np.all(x[..., 4] == 0.0)
    assert np.all(x[..., 5] == 1.0)
    x4 = unet.frame_input(mu, var, 4, GLUE_W, GLUE_H, GLUE_TW, GLUE_TH)
    assert np.all(x4[..., 5] == 0.25)


def test_select_falls_back_per_tile_above_the_threshold():
    mu = _glue_tiles()
    net = np.full((GLUE_H, GLUE_W, 3), -1.0)
    for (y, xx) in GLUE_MAP:
        net[y, xx] = [-(100 * y + 10 * xx + c) - 1 for c in range(3)]
    # tau = 1: tile 1 sits exactly at the threshold (not above: denoised),
    # tiles 2 (1.5), 3 (inf) and 5 (2.0) fall back to the plain mean
    var = np.array([0.5, 1.0, 1.5, np.inf, 0.0, 2.0])
    res = unet.select(mu, var, net, 2, 1.0, GLUE_W, GLUE_H, GLUE_TW, GLUE_TH)
    denoised_tiles = {0, 1, 4}
    for (y, xx), (t, q) in GLUE_MAP.items():
        if t in denoised_tiles:
            assert list(res[t, q, :3]) == [-(100 * y + 10 * xx + c) - 1 for c in range(3)], (y, xx)
        else:
            assert list(res[t, q, :3]) == [1000 * t + 10 * q + c for c in range(3)], (y, xx)
        assert res[t, q, 3] == 1000 * t + 10 * q + 3          # alpha is always the mean's
    # pixels of a tile past the image edge keep the mean (tile 4: q = 2, 3)
    assert list(res[4, 2]) == [4020, 4021, 4022, 4023]
    assert list(res[4, 3]) == [4030, 4031, 4032, 4033]
    # n = 1: no variance is measured, no tile falls back
    res1 = unet.select(mu, var, net, 1, 1.0, GLUE_W, GLUE_H, GLUE_TW, GLUE_TH)
    for (y, xx), (t, q) in GLUE_MAP.items():
        assert list(res1[t, q, :3]) == [-(100 * y + 10 * xx + c) - 1 for c in range(3)], (y, xx)
