"""What the trained denoiser gains over plain accumulation, measured against
the FP64 oracle's noise-free composite (the limit of the accumulation: the
composite is linear in colour for fixed alpha and order, and the noise has
zero mean).

Scenes: the 4x4x4-brick geometry at 1024x1024 with spatially correlated
alpha / colour (16 px), colour noise sigma 0.2; 16 training views (random
azimuth and elevation) and the 30/25 test view.  The plain path is first
pinned to its closed form E[MSE(n)] = sigma^2 mean_p sum_i T_i^2 / n (sum over
covered fragments), then the network, trained on the GPU by the library's
own kernels for a few hundred steps, must beat the 64-frame plain PSNR from
at most 8 frames.  The learned PSNR itself is not pinned (it is learned).
"""
import numpy as np
import pytest

import oracle
from gpu_helpers import torch_dev

pytestmark = pytest.mark.gpu


def sum_t2(f):
    """sum over covered fragments of T_i^2 per pixel, T_i from the definition."""
    out = np.zeros((f.n_tiles, f.P))
    for t in range(f.n_tiles):
        sel = f.layers[f.layers["tile_id"] == t]
        if len(sel) == 0:
            continue
        d = f.frag[sel["block"], 4, :]
        a = f.frag[sel["block"], 3, :].astype(np.float64)
        cov = f.covered[sel["block"]]
        order = np.lexsort((np.broadcast_to(sel["source_id"][:, None], d.shape), d), axis=0)
        a_s = np.take_along_axis(a, order, axis=0)
        c_s = np.take_along_axis(cov, order, axis=0)
        Tb = np.cumprod(np.vstack([np.ones((1, f.P)), 1 - a_s[:-1]]), axis=0)
        out[t] = (Tb ** 2 * c_s).sum(axis=0)
    return out


@pytest.mark.timeout(600)
def test_denoiser_beats_64_plain_frames_within_8():
    torch_dev()
    import paper_2305_07083_amd as dfb
    from paper_2305_07083_amd import denoise_train as dt
    train = dt.make_scenes(range(1, 17), size=1024)
    test = dt.make_scenes([0], size=1024, test_view=True)[0]
    dfb.load()
    pairs, vmax = dt.build_pairs(train)
    with dfb.Denoiser(1024 * 1024, seed=0) as net:
        losses, _ = dt.train(net.net, pairs, steps=800, batch=8, crop=128)
        del pairs
        ref = oracle.composite(test.frag, test.layers, 1024, 1024, 64, 64, expected=test.expected)["rgba"]
        res = dt.evaluate(net.net, test, vmax, ref)
    assert losses[-1][1] < 0.2 * losses[0][1]
    # plain accumulation against its closed form
    st2 = sum_t2(test).mean()
    for n in (1, 8, 64):
        predicted = 10 * np.log10(1.0 / (dt.SIGMA ** 2 * st2 / n))
        assert abs(res["plain"][n] - predicted) < 0.15, (n, res["plain"][n], predicted)
    # the learned part's gain
    assert res["frames_to_psnr"] is not None and res["frames_to_psnr"] <= 8, res
    assert res["denoised"][8] > res["plain"][8] + 6.0
    for n in (1, 2, 4, 8):
        assert res["denoised"][n] > res["plain"][n]
    # lower end-to-end time than 64 plain frames
    assert res["ms_denoised"][res["frames_to_psnr"]] < res["ms_plain"]
    print("denoiser:", {k: res[k] for k in ("plain", "denoised", "frames_to_psnr", "ms_plain", "ms_denoised")})
