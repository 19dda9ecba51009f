"""The accumulation tolerance used by the GPU parity tests is a derived
bound (gpu_helpers.WelfordBound), not a chosen constant.  Here it is checked
on the CPU against an emulation of the GPU's FP32 arithmetic: frames
perturbed by up to the colour bar, folded in with n = 1 copying the frame and
d = fl(x - mu), mu = fma(d, fl(1/k), mu), q = fma(d, fl(x - mu), q) in binary32
(fma emulated by one float64 evaluation rounded to binary32).  The emulated
error must stay inside the bound, and the bound must not be vacuous."""
import numpy as np

import oracle
from gpu_helpers import WelfordBound


def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32)


def fma32(a, b, c):
    return f32(a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64))


def emulate(xs):
    mu = None
    q = None
    for k, x in enumerate(xs, start=1):
        x = f32(x)
        if k == 1:
            mu = x.copy()
            q = np.zeros(x.shape[:-1] + (3,), dtype=np.float32)
            continue
        inv = f32(1.0 / np.float32(k))
        d = f32(x.astype(np.float64) - mu.astype(np.float64))
        mu = fma32(d, np.broadcast_to(inv, d.shape), mu)
        g = f32(x.astype(np.float64) - mu.astype(np.float64))
        q = fma32(d[..., :3], g[..., :3], q)
    return mu, q


def test_bound_covers_emulated_fp32_welford():
    rng = np.random.default_rng(3)
    T, P, frames = 4, 512, 16
    base = rng.random((T, P, 4)) * rng.choice([1e-3, 0.3, 1.0], size=(T, P, 1))
    mu = np.zeros((T, P, 4))
    m2 = np.zeros((T, P, 3))
    bound = WelfordBound(T, P)
    gpu_in = []
    worst = [0.0, 0.0]
    for k in range(frames):
        x = base.copy()
        x[..., :3] += rng.normal(0.0, 0.1, (T, P, 3))
        mag = np.abs(x) + rng.random((T, P, 4)) * 0.5      # S_p >= |x|
        # a composite error near the edge of the colour bar, either sign (0.99
        # of it: rounding x + eps to binary32 below adds up to u |x|, which
        # the GPU's own binary32 composite does not have on top of its error)
        eps = 0.99e-5 * mag * rng.choice([-1.0, 1.0], size=x.shape)
        gpu_in.append(x + eps)
        mu_prev = mu.copy()
        oracle.accumulate(mu, m2, x, k + 1)
        bound.step(x, mag, mu_prev, mu, m2)
        g_mu, g_q = emulate(gpu_in)
        w = bound.check(g_mu, g_q, mu, m2, "frame %d" % (k + 1))
        worst = [max(worst[0], w[0]), max(worst[1], w[1])]
    # not vacuous: the emulated error reaches a sizeable part of the bound
    assert worst[0] > 0.3 and worst[1] > 0.05, worst


def test_bound_is_zero_width_only_where_nothing_can_differ():
    # one frame: mean within the colour bar of the frame, M2 exactly zero
    bound = WelfordBound(1, 4)
    x = np.array([[[0.1, 0.2, 0.3, 0.4]] * 4])
    mag = np.abs(x)
    mu = np.zeros((1, 4, 4))
    m2 = np.zeros((1, 4, 3))
    mu_prev = mu.copy()
    oracle.accumulate(mu, m2, x, 1)
    bound.step(x, mag, mu_prev, mu, m2)
    assert np.allclose(bound.r, 1e-5 * mag) and np.all(bound.q == 0)
