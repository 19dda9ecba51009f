"""Pins of the oracle's other tile operations and of the background texture,
against facts the paper and the mathematics fix:

* list (the end of Sec. 4.2): when a rank order is correct, the list of
  generations gives the image of the per-pixel sort; a closed form for
  constant layers; and it does ignore depth;
* average (Sec. 4.1.1): redundant renders averaged equal a higher sampling
  rate, i.e. the running mean of the same renders taken one per frame
  (the oracle's Welford accumulation), and the plain numpy mean;
* background texture (Sec. 4.2: the background tile holds a colour or a
  texture): a constant texture is the constant colour, and the texture
  shows exactly through the remaining transmittance prod(1 - alpha).
"""
import numpy as np
import pytest

import oracle
import workloads


def _small(counts_seed=1, kmax=9, depth_by_generation=True, seed=2):
    c = workloads.ragged_counts(16, kmax, counts_seed)
    return workloads.generation_frame(256, 256, 64, c, seed, depth_by_generation)


def _run(f, **kw):
    return oracle.composite(f.frag, f.layers, f.width, f.height, f.tile_w, f.tile_h, **kw)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_list_equals_sorted_blend_when_rank_order_is_correct(seed):
    f = _small(counts_seed=seed, seed=10 + seed)
    bg = (0.1, 0.2, 0.3, 0.4)
    a = _run(f, op="list", background=bg, want_order=True)
    b = _run(f, op="blend", background=bg, want_order=True)
    np.testing.assert_allclose(a["rgba"], b["rgba"], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(a["order"], b["order"])


def test_list_ignores_depth():
    f = _small(depth_by_generation=False)
    a = _run(f, op="list")["rgba"]
    b = _run(f, op="blend")["rgba"]
    assert np.abs(a - b).max() > 1e-3
    # and the list image does not change when depths change
    g = workloads.Frame(**{**f.__dict__, "frag": f.frag.copy()})
    g.frag[:, 4, :] = np.float32(0.5)
    np.testing.assert_array_equal(_run(g, op="list")["rgba"], a)


def test_list_closed_form_constant_layers():
    """K layers of constant alpha a and colour c over background bg:
    C = c (1 - (1-a)^K) / a + (1-a)^K bg (geometric series)."""
    K, a, c = 7, 0.375, 0.25
    bg = np.array([0.5, 0.25, 0.125, 1.0])
    counts = np.full(16, K, dtype=np.int32)
    f = workloads.generation_frame(256, 256, 64, counts, 3, depth_by_generation=False)
    f.frag[:, 0:3, :] = c
    f.frag[:, 3, :] = a
    out = _run(f, op="list", background=tuple(bg))["rgba"]
    r = (1 - a) ** K
    want = np.array([c, c, c, a]) * (1 - r) / a + r * bg
    np.testing.assert_allclose(out, np.broadcast_to(want, out.shape), rtol=1e-14, atol=1e-15)


def test_list_rejects_generation_zero():
    f = _small()
    lay = f.layers.copy()
    lay["source_id"][0] = 0
    with pytest.raises(oracle.OracleError):
        oracle.composite(f.frag, lay, 256, 256, 64, 64, op="list")


def test_average_is_the_accumulated_mean_of_the_renders():
    counts = workloads.ragged_counts(16, 8, 5)
    f, _ = workloads.redundant_frame(256, 256, 64, counts, 0.3, 6)
    bg = (0.0, 0.5, 0.0, 1.0)
    out = _run(f, op="average", background=bg, want_mag=True)
    for t in range(16):
        sel = np.sort(f.layers[f.layers["tile_id"] == t], order="source_id")
        if len(sel) == 0:
            np.testing.assert_array_equal(out["rgba"][t], np.broadcast_to(bg, (f.P, 4)))
            continue
        x = f.frag[sel["block"], 0:4, :].astype(np.float64)   # [K, 4, P]
        np.testing.assert_allclose(out["rgba"][t], x.mean(axis=0).T, rtol=1e-13, atol=1e-15)
        # the same renders folded in one per frame (progressive refinement)
        mu = np.zeros((f.P, 4))
        m2 = np.zeros((f.P, 3))
        for n in range(1, len(sel) + 1):
            oracle.accumulate(mu, m2, np.ascontiguousarray(x[n - 1].T), n)
        np.testing.assert_allclose(out["rgba"][t], mu, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(out["mag"][t], np.abs(x).mean(axis=0).T, rtol=1e-13)


def test_average_rejects_order_output():
    counts = np.full(16, 2, dtype=np.int32)
    f, _ = workloads.redundant_frame(256, 256, 64, counts, 0.1, 1)
    with pytest.raises(oracle.OracleError):
        _run(f, op="average", want_order=True)


@pytest.mark.parametrize("op", ["blend", "list", "average"])
def test_constant_texture_is_the_background_colour(op):
    f = _small(counts_seed=4, seed=8)
    bg = (0.25, 0.5, 0.75, 0.5)
    img = np.broadcast_to(np.asarray(bg), (16, f.P, 4))
    a = _run(f, op=op, background=bg)["rgba"]
    b = _run(f, op=op, background_image=img)["rgba"]
    np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("op", ["blend", "list"])
def test_texture_shows_through_the_transmittance(op):
    f = _small(counts_seed=6, seed=9)
    img = workloads.background_texture(16, f.P, 11).astype(np.float64)
    with_img = _run(f, op=op, background_image=img)["rgba"]
    without = _run(f, op=op)["rgba"]
    T = np.ones((16, f.P))
    for t in range(16):
        sel = f.layers[f.layers["tile_id"] == t]
        T[t] = np.prod(1.0 - f.frag[sel["block"], 3, :].astype(np.float64), axis=0)
    np.testing.assert_allclose(with_img - without, T[..., None] * img, rtol=0, atol=1e-13)


def test_average_shows_texture_only_where_empty():
    counts = workloads.ragged_counts(16, 3, 12, p_empty=0.4)
    f, _ = workloads.redundant_frame(256, 256, 64, counts, 0.1, 13)
    img = workloads.background_texture(16, f.P, 14).astype(np.float64)
    out = _run(f, op="average", background_image=img)["rgba"]
    plain = _run(f, op="average")["rgba"]
    for t in range(16):
        if counts[t] == 0:
            np.testing.assert_array_equal(out[t], img[t])
        else:
            np.testing.assert_array_equal(out[t], plain[t])
