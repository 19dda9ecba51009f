"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned work unit and waves per unit):

* 2048x2048, 4x4x4 bricks: every pixel of every tile, sort order bit-exact;
* 4096x1024, 8x8x4 bricks, fp32 and fp16, 16 progressive frames with
  N(0, 0.1) colour noise: running mean, M2, per-tile variance and RGBA8 at
  every pixel after every frame, sort order bit-exact on frame 1;
* 8192x8192, 128x128 tiles, truncated-Zipf(1.2) layer counts up to 512 per
  tile, values drawn on the device: a K-stratified sample of tiles (including
  the largest K) copied back and composited by the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (WelfordBound, assert_colour, assert_rgba8, order_as_sources, reduce_depth,
                         stream_handle, torch_dev, upload)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfb():
    torch_dev()
    import paper_2305_07083_amd as m
    m.load()
    return m


def stratified_tiles(counts, n, rng):
    order = np.argsort(counts, kind="stable")
    picks = set([int(order[-1]), int(order[0])])
    for q in np.linspace(0, len(order) - 1, n):
        picks.add(int(order[int(q)]))
    extra = rng.choice(len(counts), size=min(4, len(counts)), replace=False)
    picks.update(int(t) for t in extra)
    return np.array(sorted(picks), dtype=np.int32)


@pytest.mark.timeout(300)
def test_bricks_2048_every_pixel(dfb):
    f = workloads.c2()
    cfg = dfb.make_config(2048, 2048, 64, work=0, waves=0, flags=dfb.DFB_KEEP_FINISHED | dfb.DFB_KEEP_SORT_ORDER)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(upload(f.frag), f.frag.shape[0], f.layers, f.expected)
        c.composite()
        info = c.info()
        got = c.read(dfb.DFB_BUF_FINISHED_F32)
        final = c.read(dfb.DFB_BUF_FINAL)
        order = c.read(dfb.DFB_BUF_SORT_ORDER)
    assert info.work_w in (16, 32, 64) and info.waves_per_tile in (1, 2, 4)
    ref = oracle.composite(f.frag, f.layers, 2048, 2048, 64, 64, expected=f.expected, want_mag=True,
                           want_order=True)
    assert_colour(got, ref["rgba"], ref["mag"], "2048x2048")
    assert_rgba8(final, ref["rgba"], what="2048x2048")
    gord = order_as_sources(order, f.layers, np.arange(f.n_tiles), f.expected, f.P)
    for t in range(f.n_tiles):
        assert np.array_equal(gord[t], ref["order"][t, :, :f.expected[t]]), t


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", ["f32", "f16"])
def test_bricks_4096x1024_progressive_16_frames(dfb, dtype):
    """Every pixel of every tile after each of the 16 frames: the running
    mean and M2 within the FP32 Welford bound around the oracle's FP64
    recurrence, RGBA8 within 1 LSB, the per-tile variance within its
    reduction bound; frame 1's sort order bit-exact at every pixel.  Frames
    are drawn on the device (N(0, 0.1) colour noise per covered fragment) and
    the oracle reads back the exact bytes the GPU composited."""
    torch = torch_dev()
    f = workloads.c3()
    noise = workloads.DeviceNoise(f, 0.1, 77)
    half = dtype == "f16"
    cfg = dfb.make_config(4096, 1024, 64, work=0, waves=0, dtype=dfb.DFB_F16 if half else dfb.DFB_F32,
                          flags=dfb.DFB_KEEP_SORT_ORDER)
    tiles = np.arange(f.n_tiles)
    mu = np.zeros((f.n_tiles, f.P, 4))
    m2 = np.zeros((f.n_tiles, f.P, 3))
    bound = WelfordBound(f.n_tiles, f.P)
    worst = [0.0, 0.0]
    with dfb.Compositor(cfg, stream_handle()) as c:
        for k in range(16):
            x = noise.next()
            if half:
                x = x.to(torch.float16)
            c.set_fragments(x, x.shape[0], f.layers, f.expected)
            c.composite(accumulate=True)
            xh = x.cpu().numpy()
            r = oracle.composite(xh, f.layers, 4096, 1024, 64, 64, expected=f.expected, want_mag=True,
                                 want_order=(k == 0))
            mu_prev = mu.copy()
            oracle.accumulate(mu, m2, r["rgba"], k + 1)
            bound.step(r["rgba"], r["mag"], mu_prev, mu, m2)
            g_mu = c.read(dfb.DFB_BUF_ACCUM_F32)
            g_m2 = c.read(dfb.DFB_BUF_M2_F32).transpose(0, 2, 1)
            g_v = c.read(dfb.DFB_BUF_TILE_VARIANCE)
            g_8 = c.read(dfb.DFB_BUF_FINAL)
            info = c.info()
            w = bound.check(g_mu, g_m2, mu, m2, "%s frame %d" % (dtype, k + 1))
            worst = [max(worst[0], w[0]), max(worst[1], w[1])]
            assert_rgba8(g_8, mu, what="%s frame %d" % (dtype, k + 1))
            if k == 0:
                assert np.all(np.isinf(g_v))
                order = c.read(dfb.DFB_BUF_SORT_ORDER)
                gord = order_as_sources(order, f.layers, tiles, f.expected, f.P)
                for t in tiles:
                    assert np.array_equal(gord[t], r["order"][t, :, :f.expected[t]]), "order, tile %d" % t
                del order, gord
            else:
                v_ref = oracle.tile_variance(m2, tiles, 4096, 1024, 64, 64, k + 1)
                vb = bound.variance_bound(m2, tiles, 4096, 1024, 64, 64, k + 1, reduce_depth(info, f.P))
                assert np.all(np.abs(g_v - v_ref) <= vb), "%s variance, frame %d" % (dtype, k + 1)
            del xh, r
        assert c.info().accumulation_id == 16
    print("%s: largest error / bound: mean %.3g, M2 %.3g" % (dtype, worst[0], worst[1]))


@pytest.mark.timeout(600)
def test_zipf_8192_sampled_tiles(dfb):
    torch = torch_dev()
    layers, K = workloads.zipf_layout(8192, 8192, 128, 512, 1.2, 512, seed=0)
    n_blocks = len(layers)
    P = 128 * 128
    frag = workloads.uniform_values_torch(n_blocks, P, seed=0, device="cuda:0")
    expected = K.astype(np.int32)
    cfg = dfb.make_config(8192, 8192, 128, work=0, waves=0,
                          flags=dfb.DFB_KEEP_FINISHED | dfb.DFB_KEEP_SORT_ORDER)
    rng = np.random.default_rng(2)
    tiles = stratified_tiles(K, 10, rng)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(frag, n_blocks, layers, expected)
        c.composite()
        info = c.info()
        assert info.max_layers_per_tile == int(K.max())
        got = np.stack([c.read(dfb.DFB_BUF_FINISHED_F32, int(t), 1)[0] for t in tiles])
        final = np.stack([c.read(dfb.DFB_BUF_FINAL, int(t), 1)[0] for t in tiles])
        orders = [c.read(dfb.DFB_BUF_SORT_ORDER, int(t), 1) for t in tiles]
    sel = np.isin(layers["tile_id"], tiles)
    sub = layers[sel].copy()
    idx = torch.from_numpy(sub["block"].copy()).to("cuda:0")
    host = frag[idx].cpu().numpy()
    del idx
    sub["block"] = np.arange(len(sub))
    ref = oracle.composite(host, sub, 8192, 8192, 128, 128, tiles=tiles, want_mag=True, want_order=True)
    assert_colour(got, ref["rgba"], ref["mag"], "8192^2 zipf")
    assert_rgba8(final, ref["rgba"], what="8192^2 zipf")
    for i, t in enumerate(tiles):
        gord = order_as_sources(orders[i], layers, [t], expected, P)[0]
        assert np.array_equal(gord, ref["order"][i, :, :K[t]]), t
    del frag
    torch.cuda.empty_cache()


@pytest.mark.timeout(300)
def test_list_2048_every_pixel(dfb):
    """The 2048x2048 brick frame as a generation list, in the benchmark's
    launch configuration: every pixel against the oracle's list operation,
    and (the rank order being correct for this view) against its sort."""
    f = workloads.bricks_2048_list()
    cfg = dfb.make_config(2048, 2048, 64, work=0, waves=0, op=dfb.DFB_OP_LIST,
                          flags=dfb.DFB_KEEP_FINISHED | dfb.DFB_KEEP_SORT_ORDER)
    buf = upload(f.frag)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        got = c.read(dfb.DFB_BUF_FINISHED_F32)
        final = c.read(dfb.DFB_BUF_FINAL)
        order = c.read(dfb.DFB_BUF_SORT_ORDER)
    ref = oracle.composite(f.frag, f.layers, 2048, 2048, 64, 64, expected=f.expected, want_mag=True,
                           want_order=True, op="list")
    assert_colour(got, ref["rgba"], ref["mag"], "list 2048")
    assert_rgba8(final, ref["rgba"], what="list 2048")
    gord = order_as_sources(order, f.layers, np.arange(f.n_tiles), f.expected, f.P)
    for t in range(f.n_tiles):
        assert np.array_equal(gord[t], ref["order"][t, :, :f.expected[t]]), t
    srt = oracle.composite(f.frag, workloads.c2().layers, 2048, 2048, 64, 64, want_mag=True)
    assert_colour(got, srt["rgba"], srt["mag"], "list 2048 vs per-pixel sort")


@pytest.mark.timeout(300)
def test_average_2048_every_pixel(dfb):
    f = workloads.redundant_2048()
    cfg = dfb.make_config(2048, 2048, 64, work=0, waves=0, op=dfb.DFB_OP_AVERAGE, flags=dfb.DFB_KEEP_FINISHED)
    buf = upload(f.frag)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        got = c.read(dfb.DFB_BUF_FINISHED_F32)
        final = c.read(dfb.DFB_BUF_FINAL)
    ref = oracle.composite(f.frag, f.layers, 2048, 2048, 64, 64, expected=f.expected, want_mag=True, op="average")
    assert_colour(got, ref["rgba"], ref["mag"], "average 2048")
    assert_rgba8(final, ref["rgba"], what="average 2048")
