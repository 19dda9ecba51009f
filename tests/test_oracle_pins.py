"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here re-types the oracle's recurrences: each expectation comes from a
different formulation (exact rationals of the closed forms, the binary 'over'
operator under every bracketing, Python's sort, numpy's statistics, the
IEEE binary16 table) or from an invariant (arrival-order independence,
occlusion, no-op fragments).  The compositing definition pinned here is the
per-pixel depth sort followed by front-to-back premultiplied 'over' with the
background as the sole generation-0 tile (Usher et al., Sec. 3.1.1, Sec. 4.2,
Listing 4).
"""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))


def tiny_frame(pixels, tile_w=None, dtype=np.float32):
    """One tile; ``pixels`` is a list (per pixel) of lists (per layer) of
    (depth, source_id, r, g, b, alpha).  Layer l of every pixel comes from the
    l-th source listed for pixel 0; arrival order is the list order."""
    K = len(pixels[0])
    P = len(pixels)
    tile_w = tile_w or P
    frag = np.zeros((K, 5, P), dtype=dtype)
    layers = np.empty(K, dtype=oracle.LAYER_DTYPE)
    for l in range(K):
        layers[l] = (0, pixels[0][l][1], l)
        for p in range(P):
            d, sid, r, g, b, a = pixels[p][l]
            assert sid == pixels[0][l][1]
            frag[l, :, p] = (r, g, b, a, d)
    return frag, layers, tile_w, P // tile_w


def run(frag, layers, tw, th, bg=(0, 0, 0, 0), **kw):
    return oracle.composite(frag, layers, tw, th, tw, th, background=bg, **kw)


def exact_closed_form(frags, bg):
    """C = sum_i c_i prod_{j<i}(1-a_j) + bg prod(1-a), A likewise, in the
    order given (rationals)."""
    C = [Fraction(0)] * 3
    A = Fraction(0)
    for i, f in enumerate(frags):
        w = Fraction(1)
        for j in range(i):
            w *= 1 - Fraction(float(frags[j][5]))
        for c in range(3):
            C[c] += w * Fraction(float(f[2 + c]))
        A += w * Fraction(float(f[5]))
    Tend = Fraction(1)
    for f in frags:
        Tend *= 1 - Fraction(float(f[5]))
    return [C[c] + Tend * Fraction(float(bg[c])) for c in range(3)] + [A + Tend * Fraction(float(bg[3]))]


def over(x, y):
    """Binary premultiplied 'over' on (C, A) pairs: x in front of y."""
    (cx, ax), (cy, ay) = x, y
    return ([cx[c] + (1 - ax) * cy[c] for c in range(3)], ax + (1 - ax) * ay)


def all_bracketings(items):
    if len(items) == 1:
        yield items[0]
        return
    for k in range(1, len(items)):
        for left in all_bracketings(items[:k]):
            for right in all_bracketings(items[k:]):
                yield over(left, right)


def random_pixel(rng, K, sids=None, ties=False):
    sids = list(range(K)) if sids is None else sids
    out = []
    for l in range(K):
        a = np.float32(rng.random())
        d = np.float32(rng.choice([0.25, 0.5])) if ties else np.float32(rng.random())
        out.append((d, sids[l], np.float32(a * rng.random()), np.float32(a * rng.random()),
                    np.float32(a * rng.random()), a))
    return out


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 6])
def test_every_arrival_order_matches_exact_closed_form(K):
    rng = np.random.default_rng(100 + K)
    px = [random_pixel(rng, K, ties=(K % 2 == 0)) for _ in range(3)]
    bg = (0.125, 0.25, 0.5, 0.75)
    # expected: Python's sort on the key tuple, then the rational closed form
    expect = []
    for p in px:
        order = sorted(range(K), key=lambda i: (math.isnan(p[i][0]), p[i][0] + 0.0, p[i][1]))
        expect.append((order, exact_closed_form([p[i] for i in order], bg)))
    first = None
    for perm in itertools.permutations(range(K)):
        pp = [[p[i] for i in perm] for p in px]
        frag, layers, tw, th = tiny_frame(pp)
        r = run(frag, layers, tw, th, bg, want_order=True, want_mag=True)
        for p in range(3):
            order, ex = expect[p]
            assert list(r["order"][0, p, :K]) == [px[p][i][1] for i in order]
            for c in range(4):
                assert abs(r["rgba"][0, p, c] - float(ex[c])) <= 1e-15 * max(1.0, r["mag"][0, p, c])
        if first is None:
            first = r["rgba"].copy()
        else:
            assert np.array_equal(first, r["rgba"])  # bit-identical for every arrival order


@pytest.mark.parametrize("K", [2, 3, 4, 5])
def test_associativity_every_bracketing(K):
    """Every binary bracketing of 'over' (exact rationals) equals the oracle's
    sequential front-to-back result."""
    rng = np.random.default_rng(7 + K)
    p = random_pixel(rng, K)
    order = sorted(range(K), key=lambda i: (p[i][0], p[i][1]))
    items = [([Fraction(float(p[i][2 + c])) for c in range(3)], Fraction(float(p[i][5]))) for i in order]
    frag, layers, tw, th = tiny_frame([p])
    r = run(frag, layers, tw, th, want_mag=True)
    n = 0
    for C, A in all_bracketings(items):
        n += 1
        for c in range(3):
            assert abs(float(C[c]) - r["rgba"][0, 0, c]) <= 1e-15 * max(1.0, r["mag"][0, 0, c])
        assert abs(float(A) - r["rgba"][0, 0, 3]) <= 1e-15
    assert n == [1, 1, 2, 5, 14, 42][K - 1]  # Catalan number of bracketings


def test_split_front_back_with_background():
    """(front over back) over bg == front over (back over bg): compositing the
    back group first and using it as the background gives the same pixel."""
    rng = np.random.default_rng(3)
    p = random_pixel(rng, 6)
    p = [(np.float32(0.1 * (i + 1)),) + tuple(f[1:]) for i, f in enumerate(p)]
    bg = (0.2, 0.1, 0.3, 0.6)
    frag, layers, tw, th = tiny_frame([p])
    full = run(frag, layers, tw, th, bg)["rgba"][0, 0]
    fb, lb, _, _ = tiny_frame([p[3:]])
    back = run(fb, lb, tw, th, bg)["rgba"][0, 0]
    ff, lf, _, _ = tiny_frame([p[:3]])
    split = run(ff, lf, tw, th, tuple(back))["rgba"][0, 0]
    np.testing.assert_allclose(split, full, rtol=0, atol=1e-15)


def test_opaque_fragment_occludes_everything_behind():
    rng = np.random.default_rng(5)
    p = random_pixel(rng, 5)
    p[2] = (np.float32(0.3), p[2][1], np.float32(0.2), np.float32(0.4), np.float32(0.6), np.float32(1.0))
    bg = (0.9, 0.9, 0.9, 1.0)
    frag, layers, tw, th = tiny_frame([p])
    full = run(frag, layers, tw, th, bg)["rgba"][0, 0]
    kept = [f for f in p if f[0] <= np.float32(0.3)]
    fk, lk, _, _ = tiny_frame([kept])
    assert np.array_equal(run(fk, lk, tw, th, (0.1, 0.2, 0.3, 0.4))["rgba"][0, 0], full)


def test_transparent_empty_fragment_is_a_no_op():
    rng = np.random.default_rng(6)
    p = random_pixel(rng, 4)
    bg = (0.1, 0.2, 0.3, 0.4)
    frag, layers, tw, th = tiny_frame([p])
    base = run(frag, layers, tw, th, bg)["rgba"][0, 0]
    for depth in (np.float32(0.0), np.float32(0.5), np.float32(2.0)):
        q = p + [(depth, 99, np.float32(0), np.float32(0), np.float32(0), np.float32(0))]
        fq, lq, _, _ = tiny_frame([q])
        assert np.array_equal(run(fq, lq, tw, th, bg)["rgba"][0, 0], base)


def test_single_fragment_identity():
    f = (np.float32(0.7), 3, np.float32(0.1), np.float32(0.2), np.float32(0.3), np.float32(0.6))
    frag, layers, tw, th = tiny_frame([[f]])
    r = run(frag, layers, tw, th)["rgba"][0, 0]
    assert list(r) == [float(np.float32(0.1)), float(np.float32(0.2)), float(np.float32(0.3)), float(np.float32(0.6))]


@pytest.mark.parametrize("K", [1, 3, 8, 17])
def test_identical_fragments_closed_form(K):
    a, c = 0.375, 0.25
    p = [(np.float32(0.5), l, np.float32(c), np.float32(c), np.float32(c), np.float32(a)) for l in range(K)]
    frag, layers, tw, th = tiny_frame([p])
    r = run(frag, layers, tw, th)["rgba"][0, 0]
    assert abs(r[3] - (1 - (1 - a) ** K)) <= 1e-15
    assert abs(r[0] - c * (1 - (1 - a) ** K) / a) <= 1e-15


def test_worked_example_fixture():
    ex = json.load(open(os.path.join(HERE, "golden", "worked_example.json")))
    p = [(np.float32(f["depth"]), f["source_id"], np.float32(f["colour"]), np.float32(f["colour"]),
          np.float32(f["colour"]), np.float32(f["alpha"])) for f in ex["fragments"]]
    frag, layers, tw, th = tiny_frame([p])
    assert [int(s) for s in layers["source_id"]] == ex["arrival_order"]
    for bg in [(0, 0, 0, 0), (1, 0.5, 0.25, 1)]:
        r = run(frag, layers, tw, th, bg, want_order=True)
        assert list(r["order"][0, 0]) == ex["sorted_source_ids"]
        assert list(r["rgba"][0, 0]) == ex["final_rgba"]
        assert list(oracle.tonemap(r["rgba"][0])[0]) == ex["final_rgba8"]
    # the intermediate steps: prefixes of the sorted list
    srt = sorted(p, key=lambda f: f[0])
    for k, step in enumerate(ex["after_each_step"]):
        fk, lk, _, _ = tiny_frame([srt[:k + 1]])
        r = run(fk, lk, tw, th)["rgba"][0, 0]
        assert r[0] == step["C"] and r[3] == step["A"]
        assert 1.0 - r[3] == step["T"]


def test_key_rules_negative_zero_nan_inf():
    """-0 == +0 (tie broken by source id), NaN after every number, +-inf allowed."""
    depths = [np.float32(np.nan), np.float32(0.0), np.float32(-0.0), np.float32(np.inf),
              np.float32(-np.inf), np.float32(1e-40), np.float32(-1e-40), np.float32(np.nan)]
    sids = [5, 7, 2, 1, 9, 3, 4, 0]
    p = [(d, s, np.float32(0.1), np.float32(0.1), np.float32(0.1), np.float32(0.1)) for d, s in zip(depths, sids)]
    frag, layers, tw, th = tiny_frame([p])
    r = run(frag, layers, tw, th, want_order=True)
    # -inf, -1e-40 (subnormal), {+0,-0 by sid: 2, 7}, 1e-40, +inf, NaNs by sid (0, 5)
    assert list(r["order"][0, 0]) == [9, 4, 2, 7, 3, 1, 0, 5]


def test_sort_equals_stable_argsort_when_depths_distinct():
    rng = np.random.default_rng(11)
    K, P = 9, 16
    depth = rng.random((K, P), dtype=np.float32)
    sids = rng.permutation(1000)[:K]
    px = [[(depth[l, q], int(sids[l]), np.float32(0.1), np.float32(0.1), np.float32(0.1), np.float32(0.5))
           for l in range(K)] for q in range(P)]
    frag, layers, tw, th = tiny_frame(px, tile_w=4)
    r = run(frag, layers, tw, th, want_order=True)
    for q in range(P):
        assert list(r["order"][0, q]) == list(sids[np.argsort(depth[:, q], kind="stable")])


def test_per_pixel_not_per_rank_order():
    """Two ranks whose depth order flips between the two pixels of a tile."""
    px = [[(np.float32(0.2), 0, np.float32(0.5), 0, 0, np.float32(0.5)),
           (np.float32(0.8), 1, 0, np.float32(0.5), 0, np.float32(0.5))],
          [(np.float32(0.9), 0, np.float32(0.5), 0, 0, np.float32(0.5)),
           (np.float32(0.1), 1, 0, np.float32(0.5), 0, np.float32(0.5))]]
    frag, layers, tw, th = tiny_frame(px)
    r = run(frag, layers, tw, th)["rgba"][0]
    assert list(r[0]) == [0.5, 0.25, 0.0, 0.75]
    assert list(r[1]) == [0.25, 0.5, 0.0, 0.75]


def test_fp16_decoder_against_numpy_all_patterns():
    bits = np.arange(65536, dtype=np.uint16)
    ours = oracle.half_to_double(bits)
    ref = bits.view(np.float16).astype(np.float64)
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(ours), nan)
    assert np.array_equal(ours[~nan], ref[~nan])
    assert np.array_equal(np.signbit(ours[~nan]), np.signbit(ref[~nan]))


def test_fp16_frame_reads_the_rounded_values():
    f = workloads.c1()
    h = f.as_dtype(np.float16)
    a = oracle.composite(h.frag, h.layers, 256, 256, 64, 64, tiles=[0, 5])["rgba"]
    b = oracle.composite(h.frag.astype(np.float32), h.layers, 256, 256, 64, 64, tiles=[0, 5])["rgba"]
    assert np.array_equal(a, b)


def test_completeness_and_validation_errors():
    f = workloads.c1()
    exp = f.expected.copy()
    with pytest.raises(oracle.OracleError) as e:
        oracle.composite(f.frag, f.layers[1:], 256, 256, 64, 64, expected=exp)
    assert e.value.code == oracle.ERR_INCOMPLETE
    dup = f.layers.copy()
    dup[1] = (dup[0]["tile_id"], dup[0]["source_id"], dup[1]["block"])
    with pytest.raises(oracle.OracleError) as e:
        oracle.composite(f.frag, dup, 256, 256, 64, 64)
    assert e.value.code == oracle.ERR_DUPLICATE
    bad = f.layers.copy()
    bad[0]["tile_id"] = 16
    with pytest.raises(oracle.OracleError) as e:
        oracle.composite(f.frag, bad, 256, 256, 64, 64)
    assert e.value.code == oracle.ERR_ARG


def test_tile_with_no_layers_is_the_background():
    f = workloads.c1()
    keep = f.layers[f.layers["tile_id"] != 3]
    r = oracle.composite(f.frag, keep, 256, 256, 64, 64, background=(0.25, 0.5, 0.75, 1.0), tiles=[3])
    assert np.all(r["rgba"][0] == np.array([0.25, 0.5, 0.75, 1.0]))


# ---------------------------- accumulation --------------------------------
def test_welford_against_numpy():
    rng = np.random.default_rng(1)
    xs = rng.standard_normal((12, 50, 4))
    mu = np.zeros((50, 4))
    m2 = np.zeros((50, 3))
    for n in range(1, 13):
        oracle.accumulate(mu, m2, xs[n - 1], n)
        np.testing.assert_allclose(mu, xs[:n].mean(axis=0), rtol=0, atol=1e-12)
        if n >= 2:
            np.testing.assert_allclose(m2 / (n - 1), xs[:n, :, :3].var(axis=0, ddof=1), rtol=0, atol=1e-12)


def test_identical_frames_converge_exactly_and_restart_on_n1():
    x = np.random.default_rng(2).random((10, 4))
    mu = np.full((10, 4), 7.0)
    m2 = np.full((10, 3), 3.0)
    for n in range(1, 6):
        oracle.accumulate(mu, m2, x, n)
        assert np.array_equal(mu, x)
        assert np.all(m2 == 0.0)


def test_tile_variance_matches_numpy_and_counts_inside_pixels_only():
    rng = np.random.default_rng(4)
    W, H, tw, th, n = 5, 3, 4, 2, 6
    tiles_x, tiles_y = 2, 2
    xs = rng.standard_normal((n, tiles_x * tiles_y, tw * th, 4))
    mu = np.zeros((tiles_x * tiles_y, tw * th, 4))
    m2 = np.zeros((tiles_x * tiles_y, tw * th, 3))
    for k in range(n):
        oracle.accumulate(mu, m2, xs[k], k + 1)
    v = oracle.tile_variance(m2, np.arange(4), W, H, tw, th, n)
    for t in range(4):
        ty, tx = divmod(t, tiles_x)
        vals = []
        for p in range(tw * th):
            py, pxl = divmod(p, tw)
            if tx * tw + pxl < W and ty * th + py < H:
                vals.extend(xs[:, t, p, :3].var(axis=0, ddof=1) / n)
        assert abs(v[t] - np.mean(vals)) <= 1e-12
    assert np.all(np.isinf(oracle.tile_variance(m2, np.arange(4), W, H, tw, th, 1)))
    assert np.all(oracle.tile_variance(np.zeros_like(m2), np.arange(4), W, H, tw, th, 3) == 0.0)


def test_tonemap_table():
    x = np.array([[-1, 0, 0.5, 1], [2, np.nan, 1e-9, 0.999]], dtype=np.float64)
    assert oracle.tonemap(x).tolist() == [[0, 0, 128, 255], [255, 0, 0, 255]]
    ks = np.arange(256, dtype=np.float64)
    codes = oracle.tonemap(np.repeat((ks / 255.0)[:, None], 4, axis=1))
    assert np.array_equal(codes[:, 0], np.arange(256))
    g = 2.2
    codes = oracle.tonemap(np.repeat(((ks / 255.0) ** g)[:, None], 4, axis=1), gamma=g)
    assert np.array_equal(codes[:, 0], np.arange(256))   # gamma applied to RGB
    assert np.all(codes[1:255, 3] <= codes[1:255, 0])    # ... and not to alpha


def test_accumulated_noise_matches_closed_form_psnr():
    """E[MSE(n)] = sigma^2 * mean_p sum_i T_i^2 / n for zero-mean colour noise on
    covered fragments (the composite is linear in colour for fixed alpha and
    order).  Checks composite + accumulate together against the statistics."""
    f = workloads.brick_frame(512, 512, (4, 4, 4), 64, seed=3)
    sigma, n = 0.1, 8
    tiles = np.arange(f.n_tiles)
    ref = oracle.composite(f.frag, f.layers, 512, 512, 64, 64)["rgba"]
    mu = np.zeros_like(ref)
    m2 = np.zeros(ref.shape[:-1] + (3,))
    for k in range(n):
        x = oracle.composite(workloads.noisy_colour(f, sigma, 11, k), f.layers, 512, 512, 64, 64)["rgba"]
        oracle.accumulate(mu, m2, x, k + 1)
    # sum_i T_i^2 over covered fragments, from the definition of T (independent loop)
    sumT2 = np.zeros((f.n_tiles, f.P))
    for t in range(f.n_tiles):
        sel = f.layers[f.layers["tile_id"] == t]
        blocks = sel["block"]
        d = f.frag[blocks, 4, :]
        a = f.frag[blocks, 3, :].astype(np.float64)
        cov = f.covered[blocks]
        order = np.lexsort((np.broadcast_to(sel["source_id"][:, None], d.shape), d), axis=0)
        a_s = np.take_along_axis(a, order, axis=0)
        cov_s = np.take_along_axis(cov, order, axis=0)
        Tb = np.cumprod(np.vstack([np.ones((1, f.P)), 1 - a_s[:-1]]), axis=0)
        sumT2[t] = (Tb ** 2 * cov_s).sum(axis=0)
    predicted = 10 * np.log10(1.0 / (sigma ** 2 * sumT2.mean() / n))
    measured = oracle.psnr(mu, ref)
    assert abs(measured - predicted) < 0.1, (measured, predicted)
    v = oracle.tile_variance(m2, tiles, 512, 512, 64, 64, n)
    expect_v = sigma ** 2 * sumT2.mean(axis=1) / n
    assert abs(np.mean(v) / np.mean(expect_v) - 1) < 0.05
