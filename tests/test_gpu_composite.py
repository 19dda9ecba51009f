"""GPU parity of the compositing path (through the C ABI) against the FP64
oracle: sort order bit-exact, colour within 1e-5 of the per-pixel magnitude
sum, RGBA8 within 1 LSB, accumulation / variance against the oracle's
Welford.  Inputs come from the seeded generators in ``workloads``."""
import json
import os

import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import (WelfordBound, assert_colour, assert_rgba8, order_as_sources, reduce_depth,
                         stream_handle, torch_dev, upload)

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def dfb():
    torch_dev()
    import paper_2305_07083_amd as m
    m.load()
    return m


def composite_gpu(dfb, f, *, work=64, waves=4, bg=(0, 0, 0, 0), flags=None, fmt=None, dtype=None,
                  gamma=1.0, layers=None):
    flags = (dfb.DFB_KEEP_FINISHED | dfb.DFB_KEEP_SORT_ORDER) if flags is None else flags
    fmt = dfb.DFB_FMT_RGBA8 if fmt is None else fmt
    dt = dfb.DFB_F16 if f.frag.dtype == np.float16 else dfb.DFB_F32
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=work, waves=waves, dtype=dt,
                          fmt=fmt, background=bg, gamma=gamma, flags=flags)
    frag = upload(f.frag)
    out = {}
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(frag, f.frag.shape[0], f.layers if layers is None else layers, f.expected)
        c.composite()
        if flags & dfb.DFB_KEEP_FINISHED:
            out["finished"] = c.read(dfb.DFB_BUF_FINISHED_F32)
        if flags & dfb.DFB_KEEP_SORT_ORDER:
            out["order"] = c.read(dfb.DFB_BUF_SORT_ORDER)
        if fmt != dfb.DFB_FMT_NONE:
            out["final"] = c.read(dfb.DFB_BUF_FINAL)
        out["info"] = c.info()
    return out


def check_frame(dfb, f, bg=(0, 0, 0, 0), **kw):
    g = composite_gpu(dfb, f, bg=bg, **kw)
    ref = oracle.composite(f.frag, f.layers, f.width, f.height, f.tile_w, f.tile_h,
                           expected=f.expected, background=bg, want_mag=True, want_order=True)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], f.name)
    assert_rgba8(g["final"], ref["rgba"], what=f.name)
    counts = f.expected
    tiles = np.arange(f.n_tiles)
    gord = order_as_sources(g["order"], f.layers, tiles, counts, f.P)
    for t in tiles:
        K = int(counts[t])
        assert np.array_equal(gord[t], ref["order"][t, :, :K]), "sort order differs in tile %d" % t
    return g, ref


# ----------------------------------------------------------------- frames
def test_worked_example_bit_exact(dfb):
    ex = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    K = len(ex["fragments"])
    frag = np.zeros((K, 5, 1), dtype=np.float32)
    layers = np.empty(K, dtype=workloads.LAYER_DTYPE)
    for l, fr in enumerate(ex["fragments"]):
        frag[l, :, 0] = (fr["colour"], fr["colour"], fr["colour"], fr["alpha"], fr["depth"])
        layers[l] = (0, fr["source_id"], l)
    f = workloads.Frame(1, 1, 1, 1, frag, layers, np.array([K], np.int32), name="worked example")
    for bg in [(0, 0, 0, 0), (1, 0.5, 0.25, 1)]:
        g = composite_gpu(dfb, f, work=0, waves=1, bg=bg)
        assert list(g["finished"][0, 0]) == ex["final_rgba"]
        assert list(g["final"][0, 0]) == ex["final_rgba8"]
        srcs = order_as_sources(g["order"], layers, [0], [K], 1)[0][0]
        assert list(srcs) == ex["sorted_source_ids"]


def test_uniform_256_four_ranks(dfb):
    check_frame(dfb, workloads.c1(), bg=(0.1, 0.2, 0.3, 0.4))


@pytest.mark.parametrize("work,waves", [(32, 1), (32, 2), (64, 1), (64, 4)])
def test_launch_shapes_give_identical_results(dfb, work, waves):
    f = workloads.brick_frame(256, 256, (4, 4, 4), 64, seed=1)
    base = composite_gpu(dfb, f, work=64, waves=4)
    g = composite_gpu(dfb, f, work=work, waves=waves)
    assert np.array_equal(base["finished"], g["finished"])
    assert np.array_equal(base["order"], g["order"])
    assert np.array_equal(base["final"], g["final"])


def test_bricks_512_and_arrival_order_invariance(dfb):
    f = workloads.brick_frame(512, 512, (4, 4, 4), 64, seed=2)
    g, _ = check_frame(dfb, f, bg=(0.0, 0.0, 0.2, 0.5))
    rng = np.random.default_rng(9)
    g2 = composite_gpu(dfb, f, bg=(0.0, 0.0, 0.2, 0.5), layers=f.layers[rng.permutation(len(f.layers))])
    assert np.array_equal(g["finished"], g2["finished"])
    assert np.array_equal(g["order"], g2["order"])


def test_ragged_frame_edges(dfb):
    f = workloads.brick_frame(200, 136, (4, 4, 4), 64, seed=4, name="200x136 ragged")
    check_frame(dfb, f, work=32, waves=2)


def test_small_tiles_ragged_rows(dfb):
    f = workloads.uniform_frame(96, 80, 32, ranks=5, seed=8)
    f = workloads.Frame(96, 80, 32, 32, f.frag, f.layers, f.expected, f.covered, "96x80 tiles 32")
    check_frame(dfb, f, work=32, waves=1)


def test_fp16_planes(dfb):
    f = workloads.brick_frame(512, 128, (8, 8, 4), 64, seed=5, name="512x128 8x8x4 fp16").as_dtype(np.float16)
    check_frame(dfb, f)


@pytest.mark.parametrize("ranks", [9, 17, 31, 32, 33, 64, 100, 257])
def test_layer_counts_across_register_and_lds_paths(dfb, ranks):
    f = workloads.uniform_frame(128, 64, 64, ranks=ranks, seed=ranks)
    check_frame(dfb, f, bg=(0.3, 0.2, 0.1, 0.9))


@pytest.mark.parametrize("ranks", [1500, 2048, 2100, 4096])
def test_thousands_of_layers(dfb, ranks):
    """Padded layer counts of 2048 and 4096 in the LDS sort, up to the
    largest tile the library takes (4096 layers, no padding): against the
    oracle, order bit-exact."""
    f = workloads.uniform_frame(16, 16, 16, ranks=ranks, seed=ranks)
    check_frame(dfb, f, work=0, waves=0, bg=(0.1, 0.1, 0.1, 1.0))


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("work", [(64, 16), (64, 4)])
def test_strip_work_units(dfb, dtype, work):
    """Full-width strip work units (the autotuner's other shape family):
    against the oracle, and the same finished colour and order as square
    units (a pixel's arithmetic does not depend on the unit's shape)."""
    f = workloads.brick_frame(512, 256, (4, 4, 4), 64, seed=7, name="strips").as_dtype(dtype)
    g, _ = check_frame(dfb, f, work=work, waves=4)
    sq = composite_gpu(dfb, f, work=32, waves=4)
    assert np.array_equal(g["finished"], sq["finished"])
    assert np.array_equal(g["order"], sq["order"])


@pytest.mark.parametrize("work", [16, 32, 64, (64, 16)])
def test_work_units_identical_for_many_layers(dfb, work):
    """With the waves per unit fixed, the LDS path splits each pixel's
    colour sum over the same lanes for every work-unit size: identical
    results (across waves per unit the split differs, so only the oracle's
    tolerance applies there)."""
    f = workloads.uniform_frame(128, 128, 64, ranks=100, seed=21)
    base = composite_gpu(dfb, f, work=32, waves=4)
    g = composite_gpu(dfb, f, work=work, waves=4)
    assert np.array_equal(base["finished"], g["finished"])
    assert np.array_equal(base["order"], g["order"])


def test_fixed_work_unit_is_honoured_after_autotuning(dfb):
    """A caller's fixed work unit and wave count are used even after another
    context with the same frame geometry was autotuned: tuned shapes are
    cached per geometry and per fixed unit / wave count.  More than 128
    layers, so even a fixed unit leaves the LDS budget to the autotuner."""
    f = workloads.uniform_frame(128, 128, 64, ranks=140, seed=5)
    tuned = composite_gpu(dfb, f, work=0, waves=0)
    for work, waves in ((16, 4), ((64, 16), 4), (32, 2), (16, 1)):
        g, _ = check_frame(dfb, f, work=work, waves=waves)
        ww, wh = (work, work) if isinstance(work, int) else work
        assert (g["info"].work_w, g["info"].work_h, g["info"].waves_per_tile) == (ww, wh, waves)
    again = composite_gpu(dfb, f, work=0, waves=0)
    assert (again["info"].work_w, again["info"].work_h) == (tuned["info"].work_w, tuned["info"].work_h)


@pytest.mark.parametrize("ranks", [6, 40])
def test_depth_ties_break_by_source(dfb, ranks):
    f = workloads.uniform_frame(64, 64, 64, ranks=ranks, seed=3)
    frag = f.frag.copy()
    frag[:, 4, :] = np.round(frag[:, 4, :] * 4) / 4   # five depth values: many ties
    check_frame(dfb, workloads.Frame(64, 64, 64, 64, frag, f.layers, f.expected, None, "ties"))


@pytest.mark.parametrize("ranks", [12, 40, 300])
def test_special_depth_values(dfb, ranks):
    """NaN, signed zeros, infinities and denormals in the register sort and
    in the LDS sort (ranks > 32)."""
    f = workloads.uniform_frame(64, 64, 64, ranks=ranks, seed=12)
    frag = f.frag.copy()
    rng = np.random.default_rng(0)
    special = np.array([np.nan, 0.0, -0.0, np.inf, -np.inf, 1e-40, -1e-40, -1.0], dtype=np.float32)
    mask = rng.random(frag[:, 4, :].shape) < 0.3
    frag[:, 4, :][mask] = special[rng.integers(0, len(special), int(mask.sum()))]
    check_frame(dfb, workloads.Frame(64, 64, 64, 64, frag, f.layers, f.expected, None, "special depths"))


def test_empty_tiles_show_background(dfb):
    f = workloads.brick_frame(256, 256, (4, 4, 4), 64, seed=6)
    keep = f.layers["tile_id"] % 3 != 0
    layers = f.layers[keep]
    expected = np.zeros(f.n_tiles, np.int32)
    np.add.at(expected, layers["tile_id"], 1)
    g = workloads.Frame(f.width, f.height, 64, 64, f.frag, layers, expected, None, "holes")
    _, ref = check_frame(dfb, g, bg=(0.25, 0.5, 0.75, 1.0))
    for t in range(f.n_tiles):
        if expected[t] == 0:
            assert np.all(ref["rgba"][t] == [0.25, 0.5, 0.75, 1.0])


def test_opaque_and_transparent_fragments(dfb):
    f = workloads.uniform_frame(64, 64, 64, ranks=7, seed=21)
    frag = f.frag.copy()
    frag[2, 3, :2048] = 1.0      # an opaque layer over half the tile
    frag[4, :4, 1000:3000] = 0.0  # an empty layer over another part
    check_frame(dfb, workloads.Frame(64, 64, 64, 64, frag, f.layers, f.expected, None, "opaque"))


def test_gamma_and_float_formats(dfb):
    f = workloads.c1()
    g = composite_gpu(dfb, f, gamma=2.2)
    ref = oracle.composite(f.frag, f.layers, 256, 256, 64, 64)
    assert_rgba8(g["final"], ref["rgba"], gamma=2.2, what="gamma 2.2")
    g = composite_gpu(dfb, f, fmt=dfb.DFB_FMT_RGBAF32)
    assert np.array_equal(g["final"], g["finished"])
    g = composite_gpu(dfb, f, fmt=dfb.DFB_FMT_NONE)
    assert "final" not in g


# -------------------------------------------------------------- accumulation
def run_progressive(dfb, f, sigma, frames, seed, *, fused=True, dtype=np.float32, work=64, waves=4):
    dt = dfb.DFB_F16 if dtype == np.float16 else dfb.DFB_F32
    cfg = dfb.make_config(f.width, f.height, 64, work=work, waves=waves, dtype=dt,
                          flags=dfb.DFB_KEEP_FINISHED)
    mu = np.zeros((f.n_tiles, f.P, 4))
    m2 = np.zeros((f.n_tiles, f.P, 3))
    tiles = np.arange(f.n_tiles)
    bound = WelfordBound(f.n_tiles, f.P)
    with dfb.Compositor(cfg, stream_handle()) as c:
        for k in range(frames):
            x = workloads.noisy_colour(f, sigma, seed, k, dtype=dtype)
            c.set_fragments(upload(x), x.shape[0], f.layers, f.expected)
            if fused:
                c.composite(accumulate=True)
            else:
                c.composite()
                c.accumulate()
            ref = oracle.composite(x, f.layers, f.width, f.height, 64, 64, want_mag=True)
            mu_prev = mu.copy()
            oracle.accumulate(mu, m2, ref["rgba"], k + 1)
            bound.step(ref["rgba"], ref["mag"], mu_prev, mu, m2)
            g_mu = c.read(dfb.DFB_BUF_ACCUM_F32)
            g_m2 = c.read(dfb.DFB_BUF_M2_F32).transpose(0, 2, 1)
            g_v = c.read(dfb.DFB_BUF_TILE_VARIANCE)
            g_8 = c.read(dfb.DFB_BUF_FINAL)
            info = c.info()
            assert info.accumulation_id == k + 1
            # mean and M2 within the FP32 Welford bound around the oracle
            bound.check(g_mu, g_m2, mu, m2, "frame %d" % (k + 1))
            assert_rgba8(g_8, mu, what="frame %d" % k)
            if k == 0:
                assert np.all(np.isinf(g_v))
                assert np.all(g_m2 == 0)
            else:
                v_ref = oracle.tile_variance(m2, tiles, f.width, f.height, 64, 64, k + 1)
                vb = bound.variance_bound(m2, tiles, f.width, f.height, 64, 64, k + 1,
                                          reduce_depth(info, f.P, unfused=not fused))
                assert np.all(np.abs(g_v - v_ref) <= vb), "variance differs at frame %d" % (k + 1)
    return mu


def test_progressive_fused_fp32(dfb):
    f = workloads.brick_frame(512, 128, (8, 8, 4), 64, seed=7)
    run_progressive(dfb, f, 0.1, 16, seed=100)


def test_progressive_fused_fp16(dfb):
    f = workloads.brick_frame(512, 128, (8, 8, 4), 64, seed=7)
    run_progressive(dfb, f, 0.1, 16, seed=101, dtype=np.float16)


def test_progressive_with_sub_tile_units(dfb):
    f = workloads.brick_frame(256, 192, (4, 4, 4), 64, seed=9)
    run_progressive(dfb, f, 0.1, 5, seed=102, work=32, waves=1)


def test_unfused_accumulate_matches_fused(dfb):
    f = workloads.brick_frame(256, 256, (4, 4, 4), 64, seed=10)
    res = []
    for fused in (True, False):
        cfg = dfb.make_config(256, 256, 64, work=64, waves=2, flags=dfb.DFB_KEEP_FINISHED)
        with dfb.Compositor(cfg, stream_handle()) as c:
            for k in range(4):
                x = workloads.noisy_colour(f, 0.1, 5, k)
                c.set_fragments(upload(x), x.shape[0], f.layers, f.expected)
                if fused:
                    c.composite(accumulate=True)
                else:
                    c.composite()
                    c.accumulate()
            res.append((c.read(dfb.DFB_BUF_ACCUM_F32), c.read(dfb.DFB_BUF_M2_F32),
                        c.read(dfb.DFB_BUF_TILE_VARIANCE), c.read(dfb.DFB_BUF_FINAL)))
    (mu_a, m2_a, v_a, f_a), (mu_b, m2_b, v_b, f_b) = res
    assert np.array_equal(mu_a, mu_b) and np.array_equal(m2_a, m2_b) and np.array_equal(f_a, f_b)
    # the per-tile sums run over a different reduction tree (workgroup sizes differ)
    np.testing.assert_allclose(v_a, v_b, rtol=1e-6)


def test_reset_restarts_the_mean(dfb):
    f = workloads.c1()
    cfg = dfb.make_config(256, 256, 64, work=64, waves=4, flags=dfb.DFB_KEEP_FINISHED)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(upload(f.frag), f.frag.shape[0], f.layers, f.expected)
        c.composite(accumulate=True)
        c.composite(accumulate=True)
        c.reset()
        c.composite(accumulate=True)
        assert c.info().accumulation_id == 1
        assert np.array_equal(c.read(dfb.DFB_BUF_ACCUM_F32), c.read(dfb.DFB_BUF_FINISHED_F32))
        assert np.all(np.isinf(c.read(dfb.DFB_BUF_TILE_VARIANCE)))


def test_kernel_timing_leaves_results_unchanged(dfb):
    """Event timing of the frame kernel (a ring of 64 event pairs, each read
    back when its slot comes round again), of every frame or of every third:
    accumulated results are bit-identical with and without it, and the
    average time is reported only while timing is on."""
    f = workloads.brick_frame(256, 256, (4, 4, 4), 64, seed=11)
    xs = [upload(workloads.noisy_colour(f, 0.1, 6, k)) for k in range(4)]
    bufs = (dfb.DFB_BUF_ACCUM_F32, dfb.DFB_BUF_M2_F32, dfb.DFB_BUF_TILE_VARIANCE, dfb.DFB_BUF_FINAL)
    res = []
    for timing in (0, 1, 3):
        cfg = dfb.make_config(256, 256, 64, work=64, waves=2, flags=dfb.DFB_KEEP_FINISHED)
        with dfb.Compositor(cfg, stream_handle()) as c:
            assert dfb.dfb_kernel_ms(c.h) == -1.0
            dfb.dfb_set_timing(c.h, timing)
            for k in range(70):  # more frames than event pairs in the ring
                c.set_fragments(xs[k % 4], xs[0].shape[0], f.layers, f.expected)
                c.composite(accumulate=True)
            ms = dfb.dfb_kernel_ms(c.h)
            if timing:
                assert 0.0 < ms < 100.0
            else:
                assert ms == -1.0
            res.append([c.read(b) for b in bufs])
            dfb.dfb_set_timing(c.h, False)
            assert dfb.dfb_kernel_ms(c.h) == -1.0
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)


def test_side_stream_gives_same_results(dfb):
    """Every launch and copy of a handle goes to the stream it was created
    with: accumulated frames on a second (default-priority) stream equal
    those on the current one bit for bit."""
    torch = torch_dev()
    f = workloads.brick_frame(256, 256, (4, 4, 4), 64, seed=13)
    xs = [upload(workloads.noisy_colour(f, 0.1, 7, k)) for k in range(3)]
    torch.cuda.synchronize()
    bufs = (dfb.DFB_BUF_ACCUM_F32, dfb.DFB_BUF_M2_F32, dfb.DFB_BUF_TILE_VARIANCE, dfb.DFB_BUF_FINAL)
    res = []
    for stream in (torch.cuda.current_stream(), torch.cuda.Stream()):
        cfg = dfb.make_config(256, 256, 64, work=32, waves=2, flags=dfb.DFB_KEEP_FINISHED)
        with dfb.Compositor(cfg, stream.cuda_stream) as c:
            for x in xs:
                c.set_fragments(x, x.shape[0], f.layers, f.expected)
                c.composite(accumulate=True)
            res.append([c.read(b) for b in bufs])
    for a, b in zip(*res):
        assert np.array_equal(a, b)


# ------------------------------------------------------------------ errors
def test_errors_are_reported(dfb):
    f = workloads.c1()
    frag = upload(f.frag)
    cfg = dfb.make_config(256, 256, 64, work=64, waves=4, flags=dfb.DFB_VALIDATE)
    with dfb.Compositor(cfg, stream_handle()) as c:
        with pytest.raises(dfb.DfbError) as e:
            c.composite()
        assert e.value.status == dfb.DFB_ERR_STATE
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments(frag, f.frag.shape[0], f.layers[1:], f.expected)
        assert e.value.status == dfb.DFB_ERR_INCOMPLETE
        dup = f.layers.copy()
        dup[1] = (dup[0]["tile_id"], dup[0]["source_id"], dup[1]["block"])
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments(frag, f.frag.shape[0], dup)
        assert e.value.status == dfb.DFB_ERR_DUPLICATE
        bad = f.layers.copy()
        bad[3]["block"] = f.frag.shape[0]
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments(frag, f.frag.shape[0], bad)
        assert e.value.status == dfb.DFB_ERR_INVALID_ARG
        nan = f.frag.copy()
        nan[5, 4, 77] = np.nan
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments(upload(nan), f.frag.shape[0], f.layers, f.expected)
        assert e.value.status == dfb.DFB_ERR_BAD_VALUE
        with pytest.raises(dfb.DfbError) as e:
            c.accumulate()
        assert e.value.status == dfb.DFB_ERR_STATE
        # the handle still works after rejected input
        c.set_fragments(frag, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        assert c.read(dfb.DFB_BUF_FINAL).shape == (16, 4096, 4)


def test_layouts_changing_every_frame(dfb):
    """New layer layouts frame after frame with nothing synchronised between
    them (the layer tables alternate between two device sets): the running
    mean of 6 frames over three different layouts -- two arrival orders of
    one brick frame and a frame with other per-tile layer counts -- against
    the oracle's Welford of the same frames."""
    a = workloads.brick_frame(320, 256, (4, 4, 4), 64, seed=21)
    b = workloads.brick_frame(320, 256, (4, 4, 4), 64, seed=21)
    b.layers = b.layers[::-1].copy()                # same fragments, another arrival order
    c_counts = workloads.ragged_counts(a.n_tiles, 12, seed=22)
    c = workloads.generation_frame(320, 256, 64, c_counts, seed=23, depth_by_generation=False)
    frames = [a, b, c, a, c, b]
    bufs = [upload(f.frag) for f in frames]
    cfg = dfb.make_config(320, 256, 64, work=32, waves=2, flags=dfb.DFB_KEEP_FINISHED)
    mu = np.zeros((a.n_tiles, a.P, 4))
    m2 = np.zeros((a.n_tiles, a.P, 3))
    with dfb.Compositor(cfg, stream_handle()) as comp:
        for k, (f, x) in enumerate(zip(frames, bufs)):
            comp.set_fragments(x, f.frag.shape[0], f.layers, f.expected)
            comp.composite(accumulate=True)
            r = oracle.composite(f.frag, f.layers, 320, 256, 64, 64, expected=f.expected)
            oracle.accumulate(mu, m2, r["rgba"], k + 1)
        g_mu = comp.read(dfb.DFB_BUF_ACCUM_F32)
        assert comp.info().accumulation_id == 6
    assert np.all(np.abs(g_mu - mu) <= 1e-5 * (np.abs(mu) + 1.0)), float(np.abs(g_mu - mu).max())
