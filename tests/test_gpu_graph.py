"""Frames launched from HIP graphs (the persistent, graph-captured launch per
frame) against direct dfb_composite_frame calls on the same inputs.

The per-frame state (work-queue counter slot, accumulation count) lives in
device memory and is advanced by the frame's own kernels, so one graph serves
every frame.  Both routes run the same kernels with the same launch shape on
the same bytes, so the running mean, M2, per-tile variance and RGBA8 must be
bit-identical after every frame -- and the direct route is itself checked
against the FP64 oracle by the other parity tests (and here once, at the end,
against the oracle's Welford over the same 16 frames).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_helpers import assert_rgba8, torch_dev

pytestmark = pytest.mark.gpu

BUFS = ("ACCUM_F32", "M2_F32", "TILE_VARIANCE", "FINAL")


@pytest.fixture(scope="module")
def dfb():
    torch_dev()
    import paper_2305_07083_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def scene():
    # ragged on both axes: 600 x 300 in 64 x 64 tiles (10 x 5 tiles)
    return workloads.brick_frame(600, 300, (4, 4, 4), 64, seed=5, name="600x300 bricks")


def snapshot(dfb, c):
    return {b: c.read(getattr(dfb, "DFB_BUF_" + b)).copy() for b in BUFS}


def assert_same(a, b, what):
    for k in BUFS:
        assert a[k].tobytes() == b[k].tobytes(), "%s: %s differs" % (what, k)


def make(dfb, f, stream, flags=0):
    cfg = dfb.make_config(f.width, f.height, 64, work=32, waves=2, fmt=dfb.DFB_FMT_RGBA8, flags=flags)
    return dfb.Compositor(cfg, stream)


@pytest.mark.timeout(300)
def test_replayed_frames_match_direct_calls(dfb, scene):
    """16 accumulating frames: DFB_REPLAY (the library's graph, built on the
    first frame and replayed for the other 15) against stream launches."""
    torch = torch_dev()
    f = scene
    s = torch.cuda.current_stream()
    buf = torch.empty(f.frag.shape, dtype=torch.float32, device="cuda:0")
    mu = np.zeros((f.n_tiles, f.P, 4))
    m2 = np.zeros((f.n_tiles, f.P, 3))
    with make(dfb, f, s.cuda_stream) as d, make(dfb, f, s.cuda_stream) as g:
        for k in range(16):
            x = workloads.noisy_colour(f, 0.1, 11, k)
            buf.copy_(torch.from_numpy(x))
            d.set_fragments(buf, x.shape[0], f.layers, f.expected)
            g.set_fragments(buf, x.shape[0], f.layers, f.expected)
            d.composite(accumulate=True)
            g.composite(accumulate=True, replay=True)
            assert_same(snapshot(dfb, d), snapshot(dfb, g), "frame %d" % (k + 1))
            r = oracle.composite(x, f.layers, f.width, f.height, 64, 64, expected=f.expected)
            oracle.accumulate(mu, m2, r["rgba"], k + 1)
        assert g.info().accumulation_id == 16
        assert_rgba8(g.read(dfb.DFB_BUF_FINAL), mu, what="16 replayed frames")
        # a reset between replays restarts the mean at the next frame
        g.reset()
        d.reset()
        d.composite(accumulate=True)
        g.composite(accumulate=True, replay=True)
        assert_same(snapshot(dfb, d), snapshot(dfb, g), "after reset")
        assert g.info().accumulation_id == 1
        assert np.all(np.isinf(g.read(dfb.DFB_BUF_TILE_VARIANCE)))
        # plain replayed frames leave the accumulation alone
        before = snapshot(dfb, g)
        g.composite(replay=True)
        after = snapshot(dfb, g)
        for k in ("ACCUM_F32", "M2_F32", "TILE_VARIANCE"):
            assert before[k].tobytes() == after[k].tobytes(), k
        assert g.info().accumulation_id == 1


@pytest.mark.timeout(300)
def test_caller_captured_frame_replays_per_frame(dfb, scene):
    """The caller captures one accumulating dfb_composite_frame call on the
    handle's stream into a graph of its own (torch.cuda.graph) and replays
    it for 15 further frames, the inputs rewritten in place between replays."""
    torch = torch_dev()
    f = scene
    s = torch.cuda.Stream()
    buf = torch.empty(f.frag.shape, dtype=torch.float32, device="cuda:0")
    with torch.cuda.stream(s):
        with make(dfb, f, s.cuda_stream) as d, make(dfb, f, s.cuda_stream) as g:
            x0 = workloads.noisy_colour(f, 0.1, 12, 0)
            buf.copy_(torch.from_numpy(x0))
            d.set_fragments(buf, x0.shape[0], f.layers, f.expected)
            g.set_fragments(buf, x0.shape[0], f.layers, f.expected)
            d.composite(accumulate=True)
            g.composite(accumulate=True)   # chooses the shape, allocates the accumulation
            s.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=s):
                g.composite(accumulate=True)
            for k in range(1, 16):
                x = workloads.noisy_colour(f, 0.1, 12, k)
                buf.copy_(torch.from_numpy(x))
                d.composite(accumulate=True)
                graph.replay()
                s.synchronize()
                assert_same(snapshot(dfb, d), snapshot(dfb, g), "frame %d" % (k + 1))
            assert g.info().accumulation_id == 16
            assert d.info().accumulation_id == 16


def test_accumulate_refuses_a_frame_already_accumulated(dfb, scene):
    """dfb_accumulate folds in a frame composited without DFB_ACCUMULATE, once."""
    torch = torch_dev()
    f = scene
    frag = torch.from_numpy(f.frag).to("cuda:0")
    with make(dfb, f, torch.cuda.current_stream().cuda_stream, flags=dfb.DFB_KEEP_FINISHED) as c:
        c.set_fragments(frag, f.frag.shape[0], f.layers, f.expected)
        c.composite(accumulate=True)
        with pytest.raises(dfb.DfbError) as e:
            c.accumulate()
        assert e.value.status == dfb.DFB_ERR_STATE
        c.composite()
        c.accumulate()
        with pytest.raises(dfb.DfbError) as e:
            c.accumulate()
        assert e.value.status == dfb.DFB_ERR_STATE
        assert c.info().accumulation_id == 2
        # the unfused pass continued the same mean: two equal frames give it exactly
        mu = c.read(dfb.DFB_BUF_ACCUM_F32)
        fin = c.read(dfb.DFB_BUF_FINISHED_F32)
        assert np.array_equal(mu, fin)


@pytest.mark.timeout(300)
def test_replay_of_frames_with_large_tiles(dfb):
    """Frames with tiles of more than 32 layers run two frame kernels (the
    LDS sort of the large tiles, then the register sort of the rest, which
    advances the frame state): replayed as one graph, 6 accumulating frames
    are bit-identical to direct calls."""
    torch = torch_dev()
    counts = workloads.ragged_counts(24, 150, seed=31, p_empty=0.1)
    f = workloads.generation_frame(384, 256, 64, counts, seed=32, depth_by_generation=False, name="K <= 150")
    s = torch.cuda.current_stream()
    buf = torch.empty(f.frag.shape, dtype=torch.float32, device="cuda:0")
    with make(dfb, f, s.cuda_stream) as d, make(dfb, f, s.cuda_stream) as g:
        for k in range(6):
            x = f.frag.copy()
            x[:, 0:3, :] *= np.float32(1.0 + 0.1 * k)
            buf.copy_(torch.from_numpy(x))
            d.set_fragments(buf, x.shape[0], f.layers, f.expected)
            g.set_fragments(buf, x.shape[0], f.layers, f.expected)
            d.composite(accumulate=True)
            g.composite(accumulate=True, replay=True)
            assert_same(snapshot(dfb, d), snapshot(dfb, g), "frame %d" % (k + 1))
        assert g.info().accumulation_id == 6
