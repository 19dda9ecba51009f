"""Shared helpers of the GPU parity tests: run a frame through the C ABI and
compare with the FP64 oracle."""
import numpy as np

import oracle

TOL_REL = 1e-5  # |gpu - oracle| <= 1e-5 * sum_i T_i |c_i| + T |bg|, per channel


def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a HIP device"
    return torch


def upload(frag):
    torch = torch_dev()
    return torch.from_numpy(np.ascontiguousarray(frag)).to("cuda:0")


def stream_handle():
    torch = torch_dev()
    return torch.cuda.current_stream().cuda_stream


def sorted_sources(layers, tile):
    s = np.sort(np.asarray(layers["source_id"])[np.asarray(layers["tile_id"]) == tile])
    return s


def order_as_sources(order_flat, layers, tiles, counts, P):
    """GPU order buffer (per tile [K][P] layer indices in source order) ->
    per tile [P, K] source ids, nearest first."""
    out = []
    pos = 0
    for t in tiles:
        K = int(counts[t])
        blk = order_flat[pos:pos + K * P].reshape(K, P).T.astype(np.int64)
        pos += K * P
        out.append(sorted_sources(layers, t)[blk] if K else np.zeros((P, 0), dtype=np.uint32))
    return out


def assert_colour(got, ref, mag, what=""):
    got = np.asarray(got, dtype=np.float64)
    err = np.abs(got - ref)
    bound = TOL_REL * mag
    bad = err > bound
    if bad.any():
        i = np.argwhere(bad)[0]
        raise AssertionError("%s colour mismatch at %s: gpu %r oracle %r bound %r (%d bad)"
                             % (what, tuple(i), got[tuple(i)], ref[tuple(i)], bound[tuple(i)], int(bad.sum())))


def assert_rgba8(got, ref_rgba, gamma=1.0, what=""):
    code = oracle.tonemap(ref_rgba, gamma).astype(np.int32)
    d = np.abs(np.asarray(got, dtype=np.int32) - code)
    assert d.max() <= 1, "%s RGBA8 differs by %d LSB" % (what, d.max())


U32 = 2.0 ** -24   # unit roundoff of binary32


class WelfordBound:
    """Per-pixel bounds on how far the GPU's FP32 running mean and M2 may be
    from the oracle's FP64 Welford recurrence, carried frame by frame.

    The GPU folds its composite x~_k = x_k + eps_k, |eps_k| <= e_k = 1e-5 S_k
    (the colour bar), into the mean with n = 1 copying the frame exactly and,
    for k >= 2, d = fl(x~ - mu~), mu~ = fma(d, fl(1/k), mu~),
    q~ = fma(d, fl(x~ - mu~), q~) -- each operation rounded once (relative
    error <= u = 2^-24).  Writing r_k for the bound on |mu~_k - mu_k| and
    d_k = x_k - mu_{k-1}, g_k = x_k - mu_k (oracle values), first-order error
    propagation gives
        r_1 = e_1,
        r_k = (1 - 1/k) r_{k-1} + e_k / k + 2u |d_k| / k + u |mu_k|,
    and for M2 (q_1 = 0 exactly)
        Q_k = Q_{k-1} + |d_k| (e_k + r_k) + |g_k| (e_k + r_{k-1})
              + 2u |d_k g_k| + u q_k + (e_k + r_k)(e_k + r_{k-1}).
    Second-order rounding terms (u^2 and u e) are covered by a 1 % margin."""

    def __init__(self, n_tiles, P):
        self.k = 0
        self.r = np.zeros((n_tiles, P, 4))
        self.q = np.zeros((n_tiles, P, 3))

    def step(self, x, mag, mu_prev, mu, m2):
        """x, mag: this frame's oracle composite and magnitude sum; mu_prev /
        mu, m2: the oracle's mean before and after folding x in, and its M2."""
        self.k += 1
        k = self.k
        e = 1e-5 * mag
        if k == 1:
            self.r = e.copy()
            self.q = np.zeros_like(self.q)
            return
        d = x - mu_prev
        g = x - mu
        r_prev = self.r
        r = (1.0 - 1.0 / k) * r_prev + e / k + 2.0 * U32 * np.abs(d) / k + U32 * np.abs(mu)
        e3, r3, rp3, d3, g3 = e[..., :3], r[..., :3], r_prev[..., :3], d[..., :3], g[..., :3]
        self.q = (self.q + np.abs(d3) * (e3 + r3) + np.abs(g3) * (e3 + rp3) + 2.0 * U32 * np.abs(d3 * g3)
                  + U32 * np.abs(m2) + (e3 + r3) * (e3 + rp3))
        self.r = r

    def check(self, g_mu, g_m2, mu, m2, what=""):
        """|gpu - oracle| within the bounds (1 % margin, 1e-30 floor)."""
        for name, got, ref, bound in (("mean", g_mu, mu, self.r), ("M2", g_m2, m2, self.q)):
            err = np.abs(np.asarray(got, dtype=np.float64) - ref)
            bad = err > bound * 1.01 + 1e-30
            if bad.any():
                i = tuple(np.argwhere(bad)[0])
                raise AssertionError("%s %s: gpu %r oracle %r bound %r (%d of %d values outside)"
                                     % (what, name, got[i], ref[i], bound[i], int(bad.sum()), bad.size))
        return float((np.abs(g_mu - mu) / (self.r + 1e-30)).max()), float((np.abs(g_m2 - m2) / (self.q + 1e-30)).max())

    def variance_bound(self, m2, tiles, width, height, tile_w, tile_h, n, reduce_depth):
        """Bound on |v_gpu - v_oracle| per tile: the GPU sums the in-image M2
        values of a tile in FP32 along reduction paths of at most
        ``reduce_depth`` additions (|error| <= gamma_D sum |M2|, gamma_D =
        D u / (1 - D u)), plus each M2 value's own bound Q; the variance is
        linear in M2, so the oracle's per-tile reduction of Q + gamma_D (M2 +
        Q) bounds it, and the final division adds u |v|."""
        gam = reduce_depth * U32 / (1.0 - reduce_depth * U32)
        mass = np.ascontiguousarray(self.q + gam * (m2 + self.q))
        b = oracle.tile_variance(mass, tiles, width, height, tile_w, tile_h, n)
        v = oracle.tile_variance(m2, tiles, width, height, tile_w, tile_h, n)
        return b * 1.01 + U32 * np.abs(v)


def reduce_depth(info, tile_px, unfused=False):
    """Longest chain of FP32 additions in a tile's M2 sum for a launch shape:
    per lane 3 per pixel it handles in a work unit, 6 in the wave reduction,
    3 across at most 4 waves, and one per further unit of the tile in the
    variance combine.  The unfused pass runs one 256-lane workgroup per
    tile."""
    if unfused:
        return 3 * (-(-tile_px // 256)) + 6 + 3
    work_px = info.work_w * info.work_h
    per_lane = -(-work_px // (64 * info.waves_per_tile))
    return 3 * per_lane + 6 + 3 + tile_px // work_px
