"""dfb_composite_noalloc, the entry point for callers that cannot allocate,
against the existing entry point (dfb_set_fragments + dfb_composite_frame)
on the same inputs with the same launch shape: the same frame kernel runs,
so the finished tile and the display pixels must be bit-identical.  Two
calls in a row, the second with a smaller frame (the static scratch keeps
the first call's contents), then a frame through the K > 32 path."""
import numpy as np
import pytest

import workloads
from gpu_helpers import stream_handle, torch_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dfb():
    torch_dev()
    import paper_2305_07083_amd as m
    m.load()
    return m


def cfg_of(dfb, f, work, waves, dtype):
    return dfb.make_config(f.width, f.height, f.tile_w, f.tile_h, work=work, waves=waves,
                           dtype=dfb.DFB_F16 if dtype == np.float16 else dfb.DFB_F32,
                           fmt=dfb.DFB_FMT_RGBA8, background=(0.1, 0.2, 0.3, 0.4), flags=dfb.DFB_KEEP_FINISHED)


def via_handle(dfb, f, frag, cfg):
    with dfb.Compositor(cfg, stream_handle()) as c:
        c.set_fragments(frag, f.frag.shape[0], f.layers, f.expected)
        c.composite()
        return c.read(dfb.DFB_BUF_FINISHED_F32), c.read(dfb.DFB_BUF_FINAL)


def via_noalloc(dfb, f, frag, cfg):
    torch = torch_dev()
    off, lo, kmax = dfb.layer_tables(f.layers, f.n_tiles, f.P)
    off_d = torch.from_numpy(off).to("cuda:0")
    lo_d = torch.from_numpy(lo).to("cuda:0")
    final = torch.empty((f.n_tiles, f.P, 4), dtype=torch.uint8, device="cuda:0")
    finished = torch.empty((f.n_tiles, f.P, 4), dtype=torch.float32, device="cuda:0")
    torch.cuda.synchronize()
    dfb.dfb_composite_noalloc(cfg, frag, off_d, lo_d, kmax, final, finished, stream_handle())
    torch.cuda.synchronize()
    return finished.cpu().numpy(), final.cpu().numpy()


def check(dfb, f, work, waves, dtype=np.float32):
    torch = torch_dev()
    frag = torch.from_numpy(np.ascontiguousarray(f.frag.astype(dtype))).to("cuda:0")
    cfg = cfg_of(dfb, f, work, waves, dtype)
    print("noalloc: %s, %d tiles, K <= %d, work %d, waves %d" % (f.name, f.n_tiles, int(f.expected.max()),
                                                               work, waves), flush=True)
    a_fin, a_8 = via_handle(dfb, f, frag, cfg)
    b_fin, b_8 = via_noalloc(dfb, f, frag, cfg)
    assert a_fin.tobytes() == b_fin.tobytes(), f.name
    assert a_8.tobytes() == b_8.tobytes(), f.name


def test_noalloc_matches_composite_frame_on_two_calls(dfb):
    # ragged 600 x 300 brick frame, then the smaller 256 x 256 four-rank frame
    check(dfb, workloads.brick_frame(600, 300, (4, 4, 4), 64, seed=5, name="600x300 bricks"), 32, 2)
    check(dfb, workloads.c1(), 64, 4)


def test_noalloc_large_layer_counts_and_fp16(dfb):
    counts = workloads.ragged_counts(12, 96, seed=8, p_empty=0.2)
    f = workloads.generation_frame(256, 192, 64, counts, seed=9, depth_by_generation=False, name="ragged K <= 96")
    check(dfb, f, 32, 4)
    check(dfb, workloads.brick_frame(320, 192, (4, 4, 4), 64, seed=6, name="320x192 bricks fp16"), 64, 1,
          dtype=np.float16)
