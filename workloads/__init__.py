"""Seeded synthetic fragment sets shaped like the paper's sort-last workloads.

This module only *draws inputs*: it holds none of the compositing arithmetic
(no sort, no blend, no accumulation).  Both the GPU library's tests and the
oracle consume what it returns, and neither side is imported here.

Layout of one frame (the paper's generation-1 Tile, Listing 1, stored SoA):
  ``frag``     [n_blocks, 5, P] planes R, G, B, A, depth of P = tile_w*tile_h
               pixels (row-major inside the tile); colour premultiplied.
  ``layers``   one record (tile_id, source_id, block) per contributed tile, in
               a shuffled arrival order (arrival order is not fixed, Sec. 3.1.1).
  ``expected`` [n_tiles] the background tile's children count (Sec. 4.2).
  ``covered``  [n_blocks, P] bool: pixels whose camera ray hits the brick.

Every draw comes from ``numpy.random.Generator(PCG64(seed))`` in the order
written in each function; device-side draws use ``torch.Generator`` seeded the
same way.  None of the paper's datasets is used: all inputs are synthetic.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

LAYER_DTYPE = np.dtype([("tile_id", "<i4"), ("source_id", "<u4"), ("block", "<i8")])


@dataclasses.dataclass
class Frame:
    width: int
    height: int
    tile_w: int
    tile_h: int
    frag: np.ndarray          # [n_blocks, 5, P] float32 (or float16)
    layers: np.ndarray        # LAYER_DTYPE, arrival order
    expected: np.ndarray      # [n_tiles] int32
    covered: np.ndarray | None = None   # [n_blocks, P] bool
    name: str = ""

    @property
    def n_tiles(self):
        return (-(-self.width // self.tile_w)) * (-(-self.height // self.tile_h))

    @property
    def P(self):
        return self.tile_w * self.tile_h

    @property
    def n_fragments(self):
        return len(self.layers) * self.P

    def as_dtype(self, dt):
        """All five planes rounded (round-to-nearest-even) to ``dt``."""
        return dataclasses.replace(self, frag=self.frag.astype(dt))


def _shuffle_arrival(rng, layers):
    return layers[rng.permutation(len(layers))]


# --------------------------------------------------------------------------
# Uniform random layers: every rank covers every tile (the 256^2, 4-rank case)
# --------------------------------------------------------------------------
def uniform_frame(width=256, height=256, tile=64, ranks=4, seed=0, name="uniform"):
    """Every rank contributes one layer to every tile; per fragment
    alpha ~ U(0,1), colour = alpha * U(0,1) per RGB channel, depth ~ U(0,1).

    Draw order: alpha [T, R, P], then U [T, R, 3, P], then depth [T, R, P],
    then the arrival permutation.  Block of (tile t, rank r) is t*R + r.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles_x, tiles_y = -(-width // tile), -(-height // tile)
    T, P = tiles_x * tiles_y, tile * tile
    alpha = rng.random((T, ranks, P), dtype=np.float32)
    U = rng.random((T, ranks, 3, P), dtype=np.float32)
    depth = rng.random((T, ranks, P), dtype=np.float32)
    frag = np.empty((T * ranks, 5, P), dtype=np.float32)
    frag[:, 0:3, :] = (alpha[:, :, None, :] * U).reshape(T * ranks, 3, P)
    frag[:, 3, :] = alpha.reshape(T * ranks, P)
    frag[:, 4, :] = depth.reshape(T * ranks, P)
    layers = np.empty(T * ranks, dtype=LAYER_DTYPE)
    layers["tile_id"] = np.repeat(np.arange(T, dtype=np.int32), ranks)
    layers["source_id"] = np.tile(np.arange(ranks, dtype=np.uint32), T)
    layers["block"] = np.arange(T * ranks, dtype=np.int64)
    layers = _shuffle_arrival(rng, layers)
    expected = np.full(T, ranks, dtype=np.int32)
    return Frame(width, height, tile, tile, frag, layers, expected,
                 np.ones((T * ranks, P), dtype=bool), name)


# --------------------------------------------------------------------------
# Brick decomposition of the unit cube under an orthographic camera
# --------------------------------------------------------------------------
def camera_basis(azimuth_deg=30.0, elevation_deg=25.0):
    """View direction d (camera looks along d) and screen axes u, v."""
    az, el = math.radians(azimuth_deg), math.radians(elevation_deg)
    d = -np.array([math.cos(el) * math.cos(az), math.cos(el) * math.sin(az), math.sin(el)])
    u = np.cross(d, [0.0, 0.0, 1.0])
    u /= np.linalg.norm(u)
    v = np.cross(u, d)
    return d, u, v


def _hull(points):
    """Convex hull (counter-clockwise) of 2-D points, monotone chain."""
    pts = sorted(map(tuple, points))

    def cross(o, a, b):
        return (a[0] - o[0]) * (b[1] - o[1]) - (a[1] - o[1]) * (b[0] - o[0])

    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return np.array(lower[:-1] + upper[:-1])


def frame_window(d, u, v, aspect):
    """Largest rectangle of width/height = ``aspect``, centred on the vertex
    centroid of the cube's projected outline and inscribed in it.  Returns
    (cx, cy, half_w, half_h) in screen units."""
    corners = np.array([[x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)], dtype=float)
    pts = np.stack([corners @ u, corners @ v], axis=1)
    hull = _hull(pts)
    cx, cy = hull.mean(axis=0)
    best = np.inf
    for i in range(len(hull)):
        a, b = hull[i], hull[(i + 1) % len(hull)]
        e = b - a
        n = np.array([e[1], -e[0]])          # outward normal for a CCW hull
        n /= np.linalg.norm(n)
        off = n @ a - (n[0] * cx + n[1] * cy)
        best = min(best, off / (abs(n[0]) * aspect + abs(n[1])))
    return cx, cy, best * aspect, best


def brick_frame(width, height, bricks=(4, 4, 4), tile=64, seed=0, azimuth=30.0, elevation=25.0,
                name="bricks", smooth_px=None):
    """Data-parallel frame of a brick decomposition of [0,1]^3 (Sec. 4.2).

    A brick (rank = x + nx*y + nx*ny*z) contributes a layer to a tile iff at
    least one pixel-centre ray of the tile hits its box -- the exact per-tile
    rank list the paper gets by ray tracing the brick bounds.  Covered pixels
    get alpha ~ Beta(2,5) and colour = alpha * U(0,1)^3; uncovered pixels of a
    contributed tile get alpha = colour = 0 (rays clipped to the brick).
    depth = d . (brick centre - cube corner nearest the camera) + U(0, 0.01).

    ``smooth_px``: when set, alpha and U are spatially correlated fields with
    the same marginals (Gaussian copula of a Gaussian-filtered white field with
    that length scale, drawn per brick) instead of i.i.d. per pixel.

    Draw order (i.i.d. case): alpha [L, P] (Beta), U [L, 3, P], jitter [L, P],
    arrival permutation; layers enumerated by (tile, brick) ascending.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    d, u, v = camera_basis(azimuth, elevation)
    cx, cy, hw, hh = frame_window(d, u, v, width / height)
    nx, ny, nz = bricks
    tiles_x, tiles_y = -(-width // tile), -(-height // tile)
    T, P = tiles_x * tiles_y, tile * tile
    Wp, Hp = tiles_x * tile, tiles_y * tile        # padded pixel grid
    sx = 2.0 * hw / width
    sy = 2.0 * hh / height
    corner_near = min(([x, y, z] for x in (0, 1) for y in (0, 1) for z in (0, 1)),
                      key=lambda c: float(np.dot(d, c)))
    n_bricks = nx * ny * nz
    hit_tiles = []            # per brick: dict tile -> [P] bool coverage
    brick_depth = np.zeros(n_bricks)
    for b in range(n_bricks):
        bx, by, bz = b % nx, (b // nx) % ny, b // (nx * ny)
        lo = np.array([bx / nx, by / ny, bz / nz])
        hi = np.array([(bx + 1) / nx, (by + 1) / ny, (bz + 1) / nz])
        brick_depth[b] = float(np.dot(d, (lo + hi) / 2 - np.asarray(corner_near, float)))
        box = np.array([[x, y, z] for x in (lo[0], hi[0]) for y in (lo[1], hi[1]) for z in (lo[2], hi[2])])
        pu, pv = box @ u, box @ v
        i0 = max(0, int(math.floor((pu.min() - (cx - hw)) / sx - 0.5)) - 1)
        i1 = min(Wp - 1, int(math.ceil((pu.max() - (cx - hw)) / sx - 0.5)) + 1)
        j0 = max(0, int(math.floor(((cy + hh) - pv.max()) / sy - 0.5)) - 1)
        j1 = min(Hp - 1, int(math.ceil(((cy + hh) - pv.min()) / sy - 0.5)) + 1)
        tiles = {}
        if i0 <= i1 and j0 <= j1:
            ii = np.arange(i0, i1 + 1)
            jj = np.arange(j0, j1 + 1)
            X = (cx - hw) + (ii + 0.5) * sx
            Y = (cy + hh) - (jj + 0.5) * sy
            o = X[None, :, None] * u + Y[:, None, None] * v          # [nj, ni, 3]
            with np.errstate(divide="ignore", invalid="ignore"):
                t1 = (lo - o) / d
                t2 = (hi - o) / d
            tmin = np.minimum(t1, t2).max(axis=2)
            tmax = np.maximum(t1, t2).min(axis=2)
            hit = tmin < tmax
            for ty in range(j0 // tile, j1 // tile + 1):
                for tx in range(i0 // tile, i1 // tile + 1):
                    sub = np.zeros((tile, tile), dtype=bool)
                    ya, yb = max(ty * tile, j0), min((ty + 1) * tile, j1 + 1)
                    xa, xb = max(tx * tile, i0), min((tx + 1) * tile, i1 + 1)
                    sub[ya - ty * tile:yb - ty * tile, xa - tx * tile:xb - tx * tile] = \
                        hit[ya - j0:yb - j0, xa - i0:xb - i0]
                    if sub.any():
                        tiles[ty * tiles_x + tx] = sub.reshape(P)
        hit_tiles.append(tiles)
    pairs = sorted((t, b) for b in range(n_bricks) for t in hit_tiles[b])
    L = len(pairs)
    covered = np.empty((L, P), dtype=bool)
    for i, (t, b) in enumerate(pairs):
        covered[i] = hit_tiles[b][t]
    if smooth_px is None:
        alpha = rng.beta(2.0, 5.0, size=(L, P)).astype(np.float32)
        U = rng.random((L, 3, P), dtype=np.float32)
    else:
        alpha, U = _smooth_fields(rng, pairs, n_bricks, tiles_x, tile, Wp, Hp, smooth_px)
    jitter = rng.random((L, P), dtype=np.float32) * np.float32(0.01)
    frag = np.empty((L, 5, P), dtype=np.float32)
    a = np.where(covered, alpha, np.float32(0.0))
    frag[:, 0:3, :] = a[:, None, :] * U
    frag[:, 3, :] = a
    bd = np.array([brick_depth[b] for _, b in pairs], dtype=np.float32)
    frag[:, 4, :] = bd[:, None] + jitter
    layers = np.empty(L, dtype=LAYER_DTYPE)
    layers["tile_id"] = [t for t, _ in pairs]
    layers["source_id"] = [b for _, b in pairs]
    layers["block"] = np.arange(L, dtype=np.int64)
    layers = _shuffle_arrival(rng, layers)
    expected = np.zeros(T, dtype=np.int32)
    np.add.at(expected, layers["tile_id"], 1)
    return Frame(width, height, tile, tile, frag, layers, expected, covered, name)


_BETA25_U = None
_BETA25_Q = None


def _beta25_ppf(u):
    """Beta(2,5) quantile by interpolation in a dense table of its CDF
    (F(x) = 1 - (1-x)^5 (1 + 5x), closed form for integer parameters)."""
    global _BETA25_U, _BETA25_Q
    if _BETA25_U is None:
        x = np.linspace(0.0, 1.0, 1 << 16)
        _BETA25_U = 1.0 - (1.0 - x) ** 5 * (1.0 + 5.0 * x)
        _BETA25_Q = x
    return np.interp(u, _BETA25_U, _BETA25_Q)


def _smooth_fields(rng, pairs, n_bricks, tiles_x, tile, Wp, Hp, length_px):
    """Per-brick spatially correlated alpha (Beta(2,5) marginal) and U
    (uniform marginal): a Gaussian copula of white noise filtered with a
    Gaussian of standard deviation ``length_px`` pixels.  The noise is drawn
    on a grid 8x coarser than the pixels over the brick's tile bounding box,
    filtered there and interpolated bilinearly, then rescaled to unit
    variance.  Draw order: per brick (ascending), 4 coarse normal fields."""
    from scipy import ndimage, special
    P = tile * tile
    L = len(pairs)
    alpha = np.empty((L, P), dtype=np.float32)
    U = np.empty((L, 3, P), dtype=np.float32)
    by_brick = {}
    for i, (t, b) in enumerate(pairs):
        by_brick.setdefault(b, []).append((i, t))
    f = 8
    for b in range(n_bricks):
        items = by_brick.get(b)
        if not items:
            continue
        tys = [t // tiles_x for _, t in items]
        txs = [t % tiles_x for _, t in items]
        y0, y1 = min(tys) * tile, (max(tys) + 1) * tile
        x0, x1 = min(txs) * tile, (max(txs) + 1) * tile
        hc, wc = (y1 - y0) // f + 2, (x1 - x0) // f + 2
        fields = []
        for _ in range(4):
            w = rng.standard_normal((hc, wc))
            g = ndimage.gaussian_filter(w, length_px / f, mode="wrap")
            up = ndimage.zoom(g, f, order=1)[: y1 - y0, : x1 - x0]
            up = (up - up.mean()) / up.std()
            fields.append(special.ndtr(up))
        a_img = _beta25_ppf(fields[0])
        for i, t in items:
            ty, tx = divmod(t, tiles_x)
            win = (slice(ty * tile - y0, (ty + 1) * tile - y0), slice(tx * tile - x0, (tx + 1) * tile - x0))
            alpha[i] = a_img[win].reshape(P)
            for c in range(3):
                U[i, c] = fields[1 + c][win].reshape(P)
    return alpha, U


def c1(seed=0):
    """256x256 in 64x64 tiles, 4 ranks, one fragment per pixel per rank."""
    return uniform_frame(256, 256, 64, 4, seed, name="256x256 uniform, 4 ranks")


def c2(seed=0, width=2048, height=2048):
    """2048^2 frame, 4x4x4 bricks (64 ranks), camera azimuth 30, elevation 25."""
    return brick_frame(width, height, (4, 4, 4), 64, seed, name="%dx%d 4x4x4 bricks" % (width, height))


def c3(seed=0, width=4096, height=1024):
    """4096x1024 frame, 8x8x4 bricks (256 ranks)."""
    return brick_frame(width, height, (8, 8, 4), 64, seed, name="%dx%d 8x8x4 bricks" % (width, height))


def c5(seed=0, width=2048, height=2048, azimuth=30.0, elevation=25.0):
    """Denoiser scenes: the 4x4x4-brick geometry with spatially correlated
    alpha and colour fields (correlation length 16 px)."""
    return brick_frame(width, height, (4, 4, 4), 64, seed, azimuth, elevation,
                       name="%dx%d 4x4x4 bricks, smooth fields" % (width, height), smooth_px=16.0)


# --------------------------------------------------------------------------
# Progressive refinement: per-frame colour noise
# --------------------------------------------------------------------------
def noisy_colour(frame: Frame, sigma, seed, index, dtype=np.float32):
    """Frame ``index`` of a progressive sequence: colour = base + N(0, sigma)
    per covered fragment and RGB channel, i.i.d. per frame; alpha and depth
    fixed; no clamping.  Draws: standard normal [L, 3, P] from
    PCG64(seed) jumped ``index + 1`` times.  Result rounded to ``dtype``."""
    bitgen = np.random.PCG64(seed).jumped(index + 1)
    rng = np.random.Generator(bitgen)
    noise = rng.standard_normal(frame.frag[:, 0:3, :].shape, dtype=np.float32) * np.float32(sigma)
    out = frame.frag.astype(np.float32, copy=True)
    out[:, 0:3, :] += np.where(frame.covered[:, None, :], noise, np.float32(0.0))
    return out.astype(dtype)


# --------------------------------------------------------------------------
# Heavy-tailed depth complexity: truncated Zipf per 128^2 region
# --------------------------------------------------------------------------
def zipf_counts(n, s=1.2, kmax=512, rng=None):
    """K ~ Zipf(s) truncated (renormalised) to {1..kmax}, by inverse CDF."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    pmf = k ** (-s)
    cdf = np.cumsum(pmf / pmf.sum())
    u = rng.random(n)
    return np.minimum(np.searchsorted(cdf, u, side="right") + 1, kmax).astype(np.int32)


def zipf_layout(width=8192, height=8192, region=128, ranks=512, s=1.2, kmax=512, seed=0):
    """Layer list of the heavy-tailed frame: the DFB tile is a ``region``^2
    block; each tile gets K ~ truncated Zipf(s) on {1..kmax} and K distinct
    ranks drawn uniformly without replacement.

    Draw order: K [n_tiles], then per tile (ascending) a permutation of the
    ranks whose first K entries are its contributors, then the arrival
    permutation.  Fragment values are drawn on the device by ``zipf_values``.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles_x, tiles_y = -(-width // region), -(-height // region)
    T = tiles_x * tiles_y
    K = zipf_counts(T, s, kmax, rng)
    tile_ids = np.repeat(np.arange(T, dtype=np.int32), K)
    srcs = np.concatenate([rng.permutation(ranks)[:k] for k in K]).astype(np.uint32)
    L = len(tile_ids)
    layers = np.empty(L, dtype=LAYER_DTYPE)
    layers["tile_id"] = tile_ids
    layers["source_id"] = srcs
    layers["block"] = np.arange(L, dtype=np.int64)
    layers = _shuffle_arrival(rng, layers)
    return layers, K


def uniform_values_torch(n_blocks, P, seed, device, dtype=None, chunk_blocks=4096):
    """Device-drawn fragment planes for ``n_blocks`` blocks: alpha ~ U(0,1),
    colour = alpha * U(0,1), depth ~ U(0,1), float32, from a seeded
    ``torch.Generator`` on ``device`` in chunks of ``chunk_blocks`` blocks
    (draw order per chunk: alpha, U, depth)."""
    import torch
    dtype = dtype or torch.float32
    out = torch.empty((n_blocks, 5, P), dtype=dtype, device=device)
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    for b0 in range(0, n_blocks, chunk_blocks):
        b1 = min(n_blocks, b0 + chunk_blocks)
        n = b1 - b0
        a = torch.rand((n, P), generator=g, device=device, dtype=torch.float32)
        U = torch.rand((n, 3, P), generator=g, device=device, dtype=torch.float32)
        dpt = torch.rand((n, P), generator=g, device=device, dtype=torch.float32)
        out[b0:b1, 0:3] = (a[:, None, :] * U).to(dtype)
        out[b0:b1, 3] = a.to(dtype)
        out[b0:b1, 4] = dpt.to(dtype)
    return out


class DeviceNoise:
    """Progressive frames drawn on the device: colour = base + N(0, sigma) per
    covered fragment and RGB channel, i.i.d. per frame, from a seeded
    ``torch.Generator`` (one normal draw of shape [L, 3, P] per frame, in
    frame order)."""

    def __init__(self, frame: Frame, sigma, seed, device="cuda:0"):
        import torch
        self.torch = torch
        self.base = torch.from_numpy(frame.frag.astype(np.float32)).to(device)
        self.mask = torch.from_numpy(frame.covered).to(device).unsqueeze(1).to(torch.float32) * float(sigma)
        self.gen = torch.Generator(device=device)
        self.gen.manual_seed(seed)
        self.out = torch.empty_like(self.base)

    def next(self):
        torch = self.torch
        self.out.copy_(self.base)
        noise = torch.randn(self.base[:, 0:3, :].shape, generator=self.gen, device=self.base.device,
                            dtype=torch.float32)
        self.out[:, 0:3, :] += noise * self.mask
        return self.out


# --------------------------------------------------------------------------
# Inputs of the other tile operations: generation lists, redundant renders,
# multi-generation trees and background textures
# --------------------------------------------------------------------------
def ragged_counts(n_tiles, kmax, seed, p_empty=0.1):
    """Per-tile layer counts: 0 with probability p_empty, else U{1..kmax}.
    Draws: U(0,1) [n_tiles], then the integers [n_tiles]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    empty = rng.random(n_tiles) < p_empty
    k = rng.integers(1, kmax + 1, size=n_tiles)
    return np.where(empty, 0, k).astype(np.int32)


def generation_frame(width, height, tile, counts, seed, depth_by_generation=True, name="generations"):
    """Tile t holds counts[t] layers whose source ids are the generations
    1..counts[t]; alpha ~ U(0,1), colour = alpha * U(0,1).  Depth: with
    ``depth_by_generation`` generation g of K lies in the slab
    ((K - g + U) / (K + 1)), so a higher generation is nearer at every
    pixel (a rank order that is correct); else U(0,1).

    Draw order: alpha [L, P], U [L, 3, P], U_depth [L, P] (L = sum counts,
    layers tile by tile, generation ascending), then the arrival permutation.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles_x, tiles_y = -(-width // tile), -(-height // tile)
    T, P = tiles_x * tiles_y, tile * tile
    counts = np.asarray(counts, dtype=np.int64)
    assert len(counts) == T
    L = int(counts.sum())
    tile_ids = np.repeat(np.arange(T, dtype=np.int32), counts)
    gens = (np.arange(L) - np.repeat(np.cumsum(counts) - counts, counts) + 1).astype(np.int64)
    Ks = np.repeat(counts, counts).astype(np.float32)
    alpha = rng.random((L, P), dtype=np.float32)
    U = rng.random((L, 3, P), dtype=np.float32)
    ud = rng.random((L, P), dtype=np.float32)
    frag = np.empty((L, 5, P), dtype=np.float32)
    frag[:, 0:3, :] = alpha[:, None, :] * U
    frag[:, 3, :] = alpha
    if depth_by_generation:
        frag[:, 4, :] = (Ks[:, None] - gens[:, None].astype(np.float32) + ud) / (Ks[:, None] + 1)
    else:
        frag[:, 4, :] = ud
    layers = np.empty(L, dtype=LAYER_DTYPE)
    layers["tile_id"] = tile_ids
    layers["source_id"] = gens.astype(np.uint32)
    layers["block"] = np.arange(L, dtype=np.int64)
    layers = _shuffle_arrival(rng, layers)
    return Frame(width, height, tile, tile, frag, layers, counts.astype(np.int32),
                 np.ones((L, P), dtype=bool), name)


def redundant_frame(width, height, tile, counts, sigma, seed, name="redundant"):
    """Redundant renders for dynamic load balancing: tile t is rendered
    counts[t] times with different seeds; render r of a tile is a fixed
    image (alpha ~ U(0.2,1), colour = alpha * U(0,1)) plus N(0, sigma) per
    RGBA channel, depth 0.  Source ids are 0..counts[t]-1.

    Draw order: base alpha [T, P], base U [T, 3, P], then one normal
    [L, 4, P] (layers tile by tile), then the arrival permutation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tiles_x, tiles_y = -(-width // tile), -(-height // tile)
    T, P = tiles_x * tiles_y, tile * tile
    counts = np.asarray(counts, dtype=np.int64)
    assert len(counts) == T
    L = int(counts.sum())
    a = (0.2 + 0.8 * rng.random((T, P), dtype=np.float32)).astype(np.float32)
    U = rng.random((T, 3, P), dtype=np.float32)
    base = np.empty((T, 4, P), dtype=np.float32)
    base[:, 0:3] = a[:, None, :] * U
    base[:, 3] = a
    noise = rng.standard_normal((L, 4, P), dtype=np.float32) * np.float32(sigma)
    tile_ids = np.repeat(np.arange(T, dtype=np.int32), counts)
    frag = np.zeros((L, 5, P), dtype=np.float32)
    frag[:, 0:4] = base[tile_ids] + noise
    layers = np.empty(L, dtype=LAYER_DTYPE)
    layers["tile_id"] = tile_ids
    layers["source_id"] = (np.arange(L) - np.repeat(np.cumsum(counts) - counts, counts)).astype(np.uint32)
    layers["block"] = np.arange(L, dtype=np.int64)
    layers = _shuffle_arrival(rng, layers)
    return Frame(width, height, tile, tile, frag, layers, counts.astype(np.int32),
                 np.ones((L, P), dtype=bool), name), base


def background_texture(n_tiles, P, seed):
    """A background texture [n_tiles, P, 4]: alpha ~ U(0,1), colour =
    alpha * U(0,1) (premultiplied), float32.  Draws: alpha [T, P], U [T, P, 3]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = rng.random((n_tiles, P), dtype=np.float32)
    U = rng.random((n_tiles, P, 3), dtype=np.float32)
    out = np.empty((n_tiles, P, 4), dtype=np.float32)
    out[..., 0:3] = a[..., None] * U
    out[..., 3] = a
    return out


def random_trees(n_tiles, seed, max_gen=3, max_children=3):
    """One complete dependency tree per tile, built top down: the background
    tile declares c0 ~ U{0..max_children} children, each tile of generation g
    < max_gen declares U{0..max_children} (0 at max_gen), and exactly the
    declared number of tiles is made for every generation.  Returns
    (bg_children [n_tiles], per-layer tile ids, generations, children), the
    layers tile by tile, generation ascending.  Draws: the integers in that
    order, tile by tile."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bg = np.zeros(n_tiles, dtype=np.int32)
    tid, gen, ch = [], [], []
    for t in range(n_tiles):
        c0 = int(rng.integers(0, max_children + 1))
        bg[t] = c0
        want, g = c0, 1
        while want > 0:
            nxt = 0
            for _ in range(want):
                c = int(rng.integers(0, max_children + 1)) if g < max_gen else 0
                tid.append(t)
                gen.append(g)
                ch.append(c)
                nxt += c
            want, g = nxt, g + 1
    return (bg, np.asarray(tid, dtype=np.int32), np.asarray(gen, dtype=np.int32),
            np.asarray(ch, dtype=np.int32))


def brick_generations(bricks=(4, 4, 4), azimuth=30.0, elevation=25.0):
    """Generation of every brick when a frame's tiles are handed over as a
    list ordered back to front: 1 for the brick whose centre lies farthest
    along the view direction, increasing towards the camera; among equal
    centre depths the larger brick id is taken as the farther one.
    Returns uint32 [n_bricks] indexed by brick id (the frame's source id)."""
    d, _, _ = camera_basis(azimuth, elevation)
    nx, ny, nz = bricks
    n = nx * ny * nz
    depth = np.empty(n)
    for b in range(n):
        bx, by, bz = b % nx, (b // nx) % ny, b // (nx * ny)
        depth[b] = float(np.dot(d, [(bx + 0.5) / nx, (by + 0.5) / ny, (bz + 0.5) / nz]))
    back_to_front = sorted(range(n), key=lambda b: (-depth[b], -b))
    gen = np.empty(n, dtype=np.uint32)
    for i, b in enumerate(back_to_front):
        gen[b] = i + 1
    return gen


def as_generation_list(frame: Frame, generations):
    """The same frame with every layer's source id replaced by its brick's
    generation (input of the list tile operation)."""
    lay = frame.layers.copy()
    lay["source_id"] = np.asarray(generations, dtype=np.uint32)[lay["source_id"]]
    return dataclasses.replace(frame, layers=lay, name=frame.name + "-list")


def bricks_2048_list(seed=0):
    """The 2048x2048 4x4x4-brick frame handed over as a generation list
    (input of the list tile operation at full size)."""
    return as_generation_list(c2(seed), brick_generations((4, 4, 4)))


def redundant_2048(seed=0, kmax=8, sigma=0.2):
    """2048x2048, 64x64 tiles, every tile rendered U{1..kmax} times (input of
    the averaging tile operation at full size)."""
    counts = ragged_counts(32 * 32, kmax, seed, p_empty=0.0)
    f, _ = redundant_frame(2048, 2048, 64, counts, sigma, seed + 1, name="redundant-2048")
    return f
