"""Pins of the FP64 denoiser oracle (oracle/unet.py): the conv definition
against scipy's 2-D correlation, the analytic backward against central
finite differences (no bfloat16 rounding), the bfloat16 rounding against
torch's float32 -> bfloat16 conversion, and Adam's constant-gradient limit."""
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
