"""GPU parity of the other tile operations (list, average), the background
texture, dependency-tree-checked fragments and the variance-driven sample
assignment, through the C ABI, against the FP64 oracle.  Bars: colour within
1e-5 of the per-pixel magnitude sum, RGBA8 within 1 LSB, orders and integer
results bit-exact."""
import numpy as np
import pytest

import oracle
import workloads
from oracle import schedule
from gpu_helpers import assert_colour, assert_rgba8, order_as_sources, stream_handle, torch_dev, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfb():
    torch_dev()
    import paper_2305_07083_amd as m
    m.load()
    return m


def run(dfb, f, op, *, work=32, waves=2, bg=(0, 0, 0, 0), image=None, flags=None, expected=None,
        frames=1, accumulate=False):
    if flags is None:
        flags = dfb.DFB_KEEP_FINISHED | (dfb.DFB_KEEP_SORT_ORDER if op != dfb.DFB_OP_AVERAGE else 0)
    dt = dfb.DFB_F16 if f.frag.dtype == np.float16 else dfb.DFB_F32
    img = None if image is None else upload(np.ascontiguousarray(image, dtype=np.float32))
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=work, waves=waves, dtype=dt,
                          background=bg, flags=flags, op=op, background_image=img)
    frag = upload(f.frag)
    out = {}
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(frag, f.frag.shape[0], f.layers, expected)
        for _ in range(frames):
            c.composite(accumulate=accumulate)
        out["finished"] = c.read(dfb.DFB_BUF_FINISHED_F32)
        out["final"] = c.read(dfb.DFB_BUF_FINAL)
        if flags & dfb.DFB_KEEP_SORT_ORDER:
            out["order"] = c.read(dfb.DFB_BUF_SORT_ORDER)
        if accumulate:
            out["accum"] = c.read(dfb.DFB_BUF_ACCUM_F32)
            out["var"] = c.read(dfb.DFB_BUF_TILE_VARIANCE)
    return out


def ref_of(f, op, bg=(0, 0, 0, 0), image=None, order=True):
    return oracle.composite(f.frag, f.layers, f.width, f.height, f.tile_w, f.tile_h, background=bg,
                            op=op, background_image=image, want_mag=True, want_order=order)


def check_order(g, ref, f):
    counts = np.bincount(f.layers["tile_id"], minlength=f.n_tiles)
    tiles = np.arange(f.n_tiles)
    gord = order_as_sources(g["order"], f.layers, tiles, counts, f.P)
    for t in tiles:
        K = int(counts[t])
        assert np.array_equal(gord[t], ref["order"][t, :, :K]), "order differs in tile %d" % t


# ------------------------------------------------------------------ list
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("work,waves", [(32, 1), (64, 4), (16, 2), ((64, 16), 4), ((64, 4), 2)])
def test_list_parity(dfb, dtype, work, waves):
    counts = workloads.ragged_counts(20, 40, 21)              # 0..40 generations, K > 32 too
    f = workloads.generation_frame(300, 250, 64, counts, 22, depth_by_generation=False).as_dtype(dtype)
    bg = (0.1, 0.2, 0.3, 0.5)
    g = run(dfb, f, dfb.DFB_OP_LIST, work=work, waves=waves, bg=bg)
    ref = ref_of(f, "list", bg)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "list")
    assert_rgba8(g["final"], ref["rgba"], what="list")
    check_order(g, ref, f)


def test_list_equals_blend_when_rank_order_is_correct(dfb):
    f = workloads.brick_frame(512, 384, tile=64, seed=31)
    lst = workloads.as_generation_list(f, workloads.brick_generations())
    a = run(dfb, lst, dfb.DFB_OP_LIST, flags=dfb.DFB_KEEP_FINISHED)
    b = run(dfb, f, dfb.DFB_OP_ALPHA_BLEND, flags=dfb.DFB_KEEP_FINISHED)
    ref = ref_of(f, "blend", order=False)
    assert_colour(a["finished"], ref["rgba"], ref["mag"], "list vs sort")
    np.testing.assert_allclose(a["finished"], b["finished"], rtol=0, atol=2e-6)


# ------------------------------------------------------------------ average
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("work,waves", [(32, 2), (64, 1), ((64, 16), 4)])
def test_average_parity(dfb, dtype, work, waves):
    counts = workloads.ragged_counts(20, 70, 23, p_empty=0.15)
    f, _ = workloads.redundant_frame(300, 250, 64, counts, 0.2, 24)
    f = f.as_dtype(dtype)
    bg = (0.0, 0.25, 0.5, 1.0)
    g = run(dfb, f, dfb.DFB_OP_AVERAGE, work=work, waves=waves, bg=bg)
    ref = ref_of(f, "average", bg, order=False)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "average")
    assert_rgba8(g["final"], ref["rgba"], what="average")


def test_average_accumulates_like_the_oracle(dfb):
    """Three frames of averaged renders folded into the running mean and the
    per-tile variance (the oracle's Welford on the oracle's averages)."""
    counts = workloads.ragged_counts(16, 6, 25)
    frames = [workloads.redundant_frame(256, 256, 64, counts, 0.2, 30 + i)[0] for i in range(3)]
    f0 = frames[0]
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, op=dfb.DFB_OP_AVERAGE, flags=dfb.DFB_KEEP_FINISHED)
    mu = np.zeros((16 * f0.P, 4))
    m2 = np.zeros((16 * f0.P, 3))
    with dfb.Compositor(cfg, stream_handle()) as c:
        bufs = [upload(fr.frag) for fr in frames]
        for n, (fr, buf) in enumerate(zip(frames, bufs), start=1):
            c.set_fragments(buf, fr.frag.shape[0], fr.layers)
            c.composite(accumulate=True)
            x = oracle.composite(fr.frag, fr.layers, 256, 256, 64, 64, op="average")["rgba"]
            oracle.accumulate(mu, m2, x.reshape(-1, 4), n)
        acc = c.read(dfb.DFB_BUF_ACCUM_F32)
        var = c.read(dfb.DFB_BUF_TILE_VARIANCE)
    np.testing.assert_allclose(acc.reshape(-1, 4), mu, rtol=0, atol=2e-5)
    v = oracle.tile_variance(m2.reshape(16, f0.P, 3), np.arange(16), 256, 256, 64, 64, 3)
    np.testing.assert_allclose(var, v, rtol=1e-3)


# ------------------------------------------------------------------ background texture
@pytest.mark.parametrize("op", ["blend", "list", "average"])
def test_background_texture_parity(dfb, op):
    counts = workloads.ragged_counts(20, 40, 26, p_empty=0.25)
    if op == "average":
        f, _ = workloads.redundant_frame(300, 250, 64, counts, 0.2, 27)
    else:
        f = workloads.generation_frame(300, 250, 64, counts, 28, depth_by_generation=False)
    img = workloads.background_texture(f.n_tiles, f.P, 29)
    code = {"blend": dfb.DFB_OP_ALPHA_BLEND, "list": dfb.DFB_OP_LIST, "average": dfb.DFB_OP_AVERAGE}[op]
    g = run(dfb, f, code, image=img, flags=dfb.DFB_KEEP_FINISHED)
    ref = ref_of(f, op, image=img.astype(np.float64), order=False)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "texture " + op)
    assert_rgba8(g["final"], ref["rgba"], what="texture " + op)


def test_background_texture_swap_between_frames(dfb):
    counts = workloads.ragged_counts(16, 5, 40, p_empty=0.3)
    f = workloads.generation_frame(256, 256, 64, counts, 41)
    img = workloads.background_texture(16, f.P, 42)
    bg = (0.5, 0.5, 0.5, 1.0)
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, background=bg, flags=dfb.DFB_KEEP_FINISHED)
    d_img = upload(img)
    buf = upload(f.frag)  # must outlive the composites that read it
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(buf, f.frag.shape[0], f.layers)
        c.composite()
        plain = c.read(dfb.DFB_BUF_FINISHED_F32).copy()
        c.set_background_image(d_img)
        c.composite()
        textured = c.read(dfb.DFB_BUF_FINISHED_F32).copy()
        c.set_background_image(None)
        c.composite()
        again = c.read(dfb.DFB_BUF_FINISHED_F32).copy()
        with pytest.raises(dfb.DfbError):
            c.set_background_image(d_img.data_ptr() + 4)
    r0 = ref_of(f, "blend", bg, order=False)
    r1 = ref_of(f, "blend", image=img.astype(np.float64), order=False)
    assert_colour(plain, r0["rgba"], r0["mag"], "colour")
    assert_colour(textured, r1["rgba"], r1["mag"], "texture")
    np.testing.assert_array_equal(again, plain)


# ------------------------------------------------------------------ dependency trees
def tree_frame(seed, max_children=3, n_tiles=16):
    bg, tid, gen, ch = workloads.random_trees(n_tiles, seed, max_gen=3, max_children=max_children)
    L = len(tid)
    vals = workloads.uniform_frame(256, 256, 64, ranks=max(1, -(-L // n_tiles)), seed=seed)
    frag = vals.frag[:L].copy()
    layers = np.empty(L, dtype=workloads.LAYER_DTYPE)
    layers["tile_id"] = tid
    layers["source_id"] = np.arange(L, dtype=np.uint32)
    layers["block"] = np.arange(L)
    tree = np.empty(L, dtype=[("generation", "<i4"), ("children", "<i4")])
    tree["generation"] = gen
    tree["children"] = ch
    perm = np.random.Generator(np.random.PCG64(seed + 1)).permutation(L)
    f = workloads.Frame(256, 256, 64, 64, frag, layers[perm], np.bincount(tid, minlength=n_tiles).astype(np.int32),
                        np.ones((L, 64 * 64), bool), "tree")
    return f, tree[perm], bg


def test_tree_fragments_blend_like_plain_fragments(dfb):
    f, tree, bg = tree_frame(50)
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, flags=dfb.DFB_KEEP_FINISHED)
    buf = upload(f.frag)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments_tree(buf, f.frag.shape[0], f.layers, tree, bg)
        c.composite()
        a = c.read(dfb.DFB_BUF_FINISHED_F32).copy()
        c.set_fragments(buf, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        b = c.read(dfb.DFB_BUF_FINISHED_F32).copy()
    np.testing.assert_array_equal(a, b)
    ref = ref_of(f, "blend", order=False)
    assert_colour(a, ref["rgba"], ref["mag"], "tree blend")


def test_tree_list_blends_by_generation(dfb):
    f, tree, bg = tree_frame(51, max_children=1)               # every tree is a list
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, flags=dfb.DFB_KEEP_FINISHED, op=dfb.DFB_OP_LIST)
    buf = upload(f.frag)
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments_tree(buf, f.frag.shape[0], f.layers, tree, bg)
        c.composite()
        got = c.read(dfb.DFB_BUF_FINISHED_F32)
    lay = f.layers.copy()
    lay["source_id"] = tree["generation"]
    ref = oracle.composite(f.frag, lay, 256, 256, 64, 64, op="list", want_mag=True)
    assert_colour(got, ref["rgba"], ref["mag"], "tree list")


def test_tree_errors(dfb):
    f, tree, bg = tree_frame(52)
    buf = upload(f.frag)
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2)
    with dfb.Compositor(cfg, stream_handle()) as c:
        # one layer missing -> incomplete
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments_tree(buf, f.frag.shape[0], f.layers[1:], tree[1:], bg)
        assert e.value.status == dfb.DFB_ERR_INCOMPLETE
        # a tile declares one child fewer -> more tiles than declared
        bg2 = bg.copy()
        t = int(np.argmax(bg2 > 0))
        bg2[t] -= 1
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments_tree(buf, f.frag.shape[0], f.layers, tree, bg2)
        assert e.value.status == dfb.DFB_ERR_TREE
        # and the handle still works
        c.set_fragments_tree(buf, f.frag.shape[0], f.layers, tree, bg)
        c.composite()
    # LIST needs one tile per generation
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, op=dfb.DFB_OP_LIST)
    f3, tree3, bg3 = tree_frame(53, max_children=3)
    assert np.any(bg3 > 1)
    buf3 = upload(f3.frag)
    with dfb.Compositor(cfg, stream_handle()) as c:
        with pytest.raises(dfb.DfbError) as e:
            c.set_fragments_tree(buf3, f3.frag.shape[0], f3.layers, tree3, bg3)
        assert e.value.status == dfb.DFB_ERR_INVALID_ARG


# ------------------------------------------------------------------ sample assignment
def test_assign_samples_from_the_variance(dfb):
    f = workloads.c1()
    cfg = dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=0, waves=0)
    with dfb.Compositor(cfg, stream_handle()) as c:
        assert c.assign_samples(10).tolist() == schedule.assign_samples([np.inf] * f.n_tiles, 10)
        for i in range(3):
            x = workloads.noisy_colour(f, 0.2, 60, i)
            buf = upload(x)
            c.set_fragments(buf, x.shape[0], f.layers, f.expected)
            c.composite(accumulate=True)
            if i == 0:
                assert c.assign_samples(7).tolist() == schedule.assign_samples([np.inf] * f.n_tiles, 7)
        var = c.read(dfb.DFB_BUF_TILE_VARIANCE)
        for extra in (0, 1, 5, 1000, 123457):
            got = c.assign_samples(extra)
            assert got.tolist() == schedule.assign_samples(var, extra)
            assert got.sum() == extra


def test_dynamic_load_balancing_round_trip(dfb):
    """Measure the variance of averaged redundant renders, give the noisiest
    tiles extra renders, and average the larger set: the assignment equals
    the oracle's on the measured variance, the extra renders go where the
    variance is, and the larger set averages like the oracle."""
    T = 16
    base_counts = np.full(T, 2, dtype=np.int32)
    sig = np.linspace(0.02, 0.4, T).astype(np.float32)    # per-tile noise level
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, op=dfb.DFB_OP_AVERAGE, flags=dfb.DFB_KEEP_FINISHED)
    with dfb.Compositor(cfg, stream_handle()) as c:
        keep = []
        for i in range(3):
            # renders with unit noise, rescaled per tile to base + sig_t * noise
            f, base = workloads.redundant_frame(256, 256, 64, base_counts, 1.0, 70 + i)
            tid = np.zeros(f.frag.shape[0], dtype=np.int64)
            tid[f.layers["block"]] = f.layers["tile_id"]
            f.frag[:, 0:4] = base[tid] + (f.frag[:, 0:4] - base[tid]) * sig[tid, None, None]
            buf = upload(f.frag)
            keep.append(buf)
            c.set_fragments(buf, f.frag.shape[0], f.layers)
            c.composite(accumulate=True)
        var = c.read(dfb.DFB_BUF_TILE_VARIANCE)
        extra = c.assign_samples(64)
    assert extra.tolist() == schedule.assign_samples(var, 64)
    assert extra[-1] > extra[0] and extra.sum() == 64
    counts = base_counts + extra
    f, _ = workloads.redundant_frame(256, 256, 64, counts, 0.2, 80)
    g = run(dfb, f, dfb.DFB_OP_AVERAGE)
    ref = ref_of(f, "average", order=False)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "rebalanced average")


# ------------------------------------------------------------------ more layers, other widths
@pytest.mark.parametrize("dtype", [np.float32, np.float16])
def test_list_and_average_past_64_layers(dfb, dtype):
    """Tiles of up to 150 layers: the vector paths hold 64 layer offsets at a
    time, so the walk crosses two reloads."""
    counts = workloads.ragged_counts(16, 150, 90, p_empty=0.1)
    counts[3] = 150
    counts[7] = 65
    f = workloads.generation_frame(256, 256, 64, counts, 91, depth_by_generation=False).as_dtype(dtype)
    g = run(dfb, f, dfb.DFB_OP_LIST, work=32, waves=4)
    ref = ref_of(f, "list")
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "list K<=150")
    check_order(g, ref, f)
    r, _ = workloads.redundant_frame(256, 256, 64, counts, 0.2, 92)
    r = r.as_dtype(dtype)
    g = run(dfb, r, dfb.DFB_OP_AVERAGE, work=64, waves=2)
    ref = ref_of(r, "average", order=False)
    assert_colour(g["finished"], ref["rgba"], ref["mag"], "average K<=150")


@pytest.mark.parametrize("op", ["list", "average"])
def test_scalar_path_for_narrow_rows(dfb, op):
    """Tile rows of 30 pixels cannot be read 4 (fp32) or 8 (fp16) pixels at a
    time: the per-pixel path runs and gives the same results."""
    counts = workloads.ragged_counts(6, 20, 93, p_empty=0.2)
    code = dfb.DFB_OP_LIST if op == "list" else dfb.DFB_OP_AVERAGE
    for dtype in (np.float32, np.float16):
        if op == "list":
            f = workloads.generation_frame(90, 60, 30, counts, 94, depth_by_generation=False)
        else:
            f, _ = workloads.redundant_frame(90, 60, 30, counts, 0.2, 95)
        f = f.as_dtype(dtype)
        g = run(dfb, f, code, work=0, waves=0, bg=(0.2, 0.1, 0.0, 0.5))
        ref = ref_of(f, op, (0.2, 0.1, 0.0, 0.5), order=(op == "list"))
        assert_colour(g["finished"], ref["rgba"], ref["mag"], op + " narrow")
        if op == "list":
            check_order(g, ref, f)


def test_texture_with_accumulation(dfb):
    """The texture goes into the accumulated mean like any finished pixel."""
    counts = workloads.ragged_counts(16, 12, 96, p_empty=0.3)
    base = workloads.generation_frame(256, 256, 64, counts, 97)
    img = workloads.background_texture(16, base.P, 98)
    d_img = upload(img)
    cfg = dfb.make_config(256, 256, 64, work=32, waves=2, background_image=d_img)
    mu = np.zeros((16 * base.P, 4))
    m2 = np.zeros((16 * base.P, 3))
    keep = []
    with dfb.Compositor(cfg, stream_handle()) as c:
        for n in range(1, 4):
            f = workloads.generation_frame(256, 256, 64, counts, 97 + 10 * n)
            buf = upload(f.frag)
            keep.append(buf)
            c.set_fragments(buf, f.frag.shape[0], f.layers)
            c.composite(accumulate=True)
            x = ref_of(f, "blend", image=img.astype(np.float64), order=False)["rgba"]
            oracle.accumulate(mu, m2, x.reshape(-1, 4), n)
        acc = c.read(dfb.DFB_BUF_ACCUM_F32)
    np.testing.assert_allclose(acc.reshape(-1, 4), mu, rtol=0, atol=3e-5)
