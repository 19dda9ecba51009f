"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times (autotuned work unit and waves per unit):

* 2048x2048, 4x4x4 bricks: every pixel of every tile, sort order bit-exact;
* 4096x1024, 8x8x4 bricks, fp32 and fp16, 16 progressive frames with
  N(0, 0.1) colour noise: running mean, M2-based per-tile variance and RGBA8
  on a K-stratified sample of tiles after frames 1, 2, 8 and 16;
* 8192x8192, 128x128 tiles, truncated-Zipf(1.2) layer counts up to 512 per
  tile, values drawn on the device: a K-stratified sample of tiles (including
  the largest K) copied back and composited by the oracle.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (assert_colour, assert_rgba8, order_as_sources, stream_handle, torch_dev,
                         upload)

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


@pytest.mark.timeout(300)
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_bricks_4096x1024_progressive_16_frames(dfb, dtype):
    f = workloads.c3()
    rng = np.random.default_rng(1)
    tiles = stratified_tiles(f.expected, 24, rng)
    sel = np.isin(f.layers["tile_id"], tiles)
    sub_layers = f.layers[sel].copy()
    sub_blocks = sub_layers["block"].copy()
    sub_layers["block"] = np.arange(len(sub_layers))
    cfg = dfb.make_config(4096, 1024, 64, work=0, waves=0,
                          dtype=dfb.DFB_F16 if dtype == np.float16 else dfb.DFB_F32)
    mu = np.zeros((len(tiles), f.P, 4))
    m2 = np.zeros((len(tiles), f.P, 3))
    with dfb.Compositor(cfg, stream_handle()) as c:
        for k in range(16):
            x = workloads.noisy_colour(f, 0.1, 77, k, dtype=dtype)
            c.set_fragments(upload(x), x.shape[0], f.layers, f.expected)
            c.composite(accumulate=True)
            r = oracle.composite(x[sub_blocks], sub_layers, 4096, 1024, 64, 64, tiles=tiles, want_mag=True)
            oracle.accumulate(mu, m2, r["rgba"], k + 1)
            if k + 1 in (1, 2, 8, 16):
                g_mu = np.stack([c.read(dfb.DFB_BUF_ACCUM_F32, int(t), 1)[0] for t in tiles])
                g_v = np.concatenate([c.read(dfb.DFB_BUF_TILE_VARIANCE, int(t), 1) for t in tiles])
                g_8 = np.stack([c.read(dfb.DFB_BUF_FINAL, int(t), 1)[0] for t in tiles])
                scale = np.maximum(r["mag"], np.abs(mu)) + 1e-6
                assert np.all(np.abs(g_mu - mu) <= 4e-5 * scale), k
                assert_rgba8(g_8, mu, what="frame %d" % (k + 1))
                v_ref = oracle.tile_variance(m2, tiles, 4096, 1024, 64, 64, k + 1)
                if k == 0:
                    assert np.all(np.isinf(g_v))
                else:
                    np.testing.assert_allclose(g_v, v_ref, rtol=1e-4)
        assert c.info().accumulation_id == 16


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
