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
