"""FP64 CPU oracle for per-tile sort-last compositing -- test infrastructure only.

Only the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` import this package.  The product library never does, and this
package imports nothing from it: the two share no code.

The compositor itself is plain C (``dfb_oracle.c``, built with
``-O2 -ffp-contract=off``); this module only marshals numpy arrays into it.
Each wrapped function follows one step of the paper's data-parallel tile
operation (Sec. 3.1, Sec. 3.1.1, Sec. 4.2 and Listing 4 of Usher et al.); the C
file's header lists which.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dfb_oracle.c")
_LIB = os.path.join(_HERE, "libdfb_oracle.so")

# The oracle's own layer record: (tile_id int32, source_id uint32, block int64).
LAYER_DTYPE = np.dtype([("tile_id", "<i4"), ("source_id", "<u4"), ("block", "<i8")])

OK, ERR_ARG, ERR_INCOMPLETE, ERR_DUPLICATE = 0, -1, -3, -4


def build(force: bool = True) -> str:
    """Compile ``dfb_oracle.c`` into ``libdfb_oracle.so`` next to it."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-std=c11", "-fPIC", "-shared",
             "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.orc_composite.restype = ctypes.c_int
        lib.orc_composite.argtypes = [P, ctypes.c_int, ctypes.c_int64, P, ctypes.c_int32, P,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, P, ctypes.c_int32, P, P, ctypes.c_int32,
                                      P, P, P, ctypes.c_int32, ctypes.c_int32]
        lib.orc_tile_counts.restype = ctypes.c_int
        lib.orc_tile_counts.argtypes = [P, ctypes.c_int32, ctypes.c_int64, P, ctypes.c_int32, P]
        lib.orc_accumulate.restype = None
        lib.orc_accumulate.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32]
        lib.orc_tile_variance.restype = None
        lib.orc_tile_variance.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        lib.orc_tonemap.restype = None
        lib.orc_tonemap.argtypes = [P, ctypes.c_int64, ctypes.c_double, P]
        lib.orc_half_to_double.restype = ctypes.c_double
        lib.orc_half_to_double.argtypes = [ctypes.c_uint16]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle rejected the input (code %d)" % code)
        self.code = code


def _as_layers(layers):
    out = np.empty(len(layers), dtype=LAYER_DTYPE)
    for name in LAYER_DTYPE.names:
        out[name] = np.asarray(layers[name])
    return out


OPS = {"blend": 0, "list": 1, "average": 2}


def composite(frag, layers, width, height, tile_w, tile_h, *, expected=None, background=(0, 0, 0, 0),
              tiles=None, want_mag=False, want_order=False, threads=None, op="blend",
              background_image=None):
    """O1-O5: composite the listed tiles (default: all) of one frame in FP64.

    ``op``: "blend" (per-pixel depth sort + over), "list" (back to front by
    generation = source id >= 1), "average" (mean of the layers).
    ``background_image``: optional [n_tiles, P, 4] texture behind everything.

    ``frag`` is a numpy array of float32 or float16 with ``n_blocks*5*P``
    elements (block, plane R,G,B,A,depth, pixel).  Returns a dict with
    ``rgba`` [n_out, P, 4] float64, optionally ``mag`` (sum of T_i|c_i| +
    T|bg| per channel: the scale of the colour tolerance) and ``order``
    [n_out, P, kmax] uint32 source ids nearest first (unused slots 0xFFFFFFFF).
    """
    lib = _load()
    frag = np.ascontiguousarray(frag)
    if frag.dtype == np.float32:
        dtype = 0
    elif frag.dtype == np.float16:
        dtype = 1
        frag = frag.view(np.uint16)
    else:
        raise TypeError("fragments must be float32 or float16")
    P = tile_w * tile_h
    n_blocks = frag.size // (5 * P)
    lay = _as_layers(layers)
    tiles_x = -(-width // tile_w)
    tiles_y = -(-height // tile_h)
    n_tiles = tiles_x * tiles_y
    tiles = np.arange(n_tiles, dtype=np.int32) if tiles is None else np.ascontiguousarray(tiles, dtype=np.int32)
    exp = None if expected is None else np.ascontiguousarray(expected, dtype=np.int32)
    bg = np.ascontiguousarray(background, dtype=np.float64)
    bgi = None
    if background_image is not None:
        bgi = np.ascontiguousarray(background_image, dtype=np.float64)
        if bgi.shape != (n_tiles, P, 4):
            raise ValueError("background_image must be [n_tiles, P, 4]")
    rgba = np.zeros((len(tiles), P, 4), dtype=np.float64)
    mag = np.zeros((len(tiles), P, 4), dtype=np.float64) if want_mag else None
    kmax = 0
    order = None
    if want_order:
        counts = tile_counts(lay, n_blocks, n_tiles)
        kmax = int(counts[tiles].max()) if len(tiles) else 0
        order = np.full((len(tiles), P, max(kmax, 1)), 0xFFFFFFFF, dtype=np.uint32)
    if threads is None:
        threads = len(os.sched_getaffinity(0))
    rc = lib.orc_composite(_ptr(frag), dtype, n_blocks, _ptr(lay), len(lay), _ptr(exp), width,
                           height, tile_w, tile_h, _ptr(bg), OPS[op], _ptr(bgi), _ptr(tiles),
                           len(tiles), _ptr(rgba),
                           _ptr(mag), _ptr(order), max(kmax, 1), int(threads))
    if rc != OK:
        raise OracleError(rc)
    out = {"rgba": rgba, "tiles": tiles}
    if want_mag:
        out["mag"] = mag
    if want_order:
        out["order"] = order
    return out


def tile_counts(layers, n_blocks, n_tiles, expected=None):
    """O1/O2: number of layers per tile, with the same checks as ``composite``."""
    lib = _load()
    lay = _as_layers(layers)
    counts = np.zeros(n_tiles, dtype=np.int32)
    exp = None if expected is None else np.ascontiguousarray(expected, dtype=np.int32)
    rc = lib.orc_tile_counts(_ptr(lay), len(lay), int(n_blocks), _ptr(exp), n_tiles, _ptr(counts))
    if rc != OK:
        raise OracleError(rc)
    return counts


def accumulate(mu, m2, x, n):
    """O6: Welford update in place; ``mu`` [...,4], ``m2`` [...,3], ``x`` [...,4]."""
    lib = _load()
    assert mu.dtype == np.float64 and m2.dtype == np.float64 and mu.flags.c_contiguous and m2.flags.c_contiguous
    x = np.ascontiguousarray(x, dtype=np.float64)
    n_px = mu.size // 4
    assert m2.size == 3 * n_px and x.size == 4 * n_px
    lib.orc_accumulate(_ptr(mu), _ptr(m2), _ptr(x), n_px, int(n))


def tile_variance(m2, tiles, width, height, tile_w, tile_h, n):
    """O7: per-tile variance of the mean; ``m2`` is [n_out, P, 3]."""
    lib = _load()
    m2 = np.ascontiguousarray(m2, dtype=np.float64)
    tiles = np.ascontiguousarray(tiles, dtype=np.int32)
    v = np.zeros(len(tiles), dtype=np.float64)
    lib.orc_tile_variance(_ptr(m2), _ptr(tiles), len(tiles), width, height, tile_w, tile_h, int(n), _ptr(v))
    return v


def tonemap(x, gamma=1.0):
    """O8: RGBA8 codes of ``x`` [..., 4]."""
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(x.shape, dtype=np.uint8)
    lib.orc_tonemap(_ptr(x), x.size // 4, float(gamma), _ptr(out))
    return out


def half_to_double(bits):
    """The oracle's own binary16 decoder, for its pin against numpy."""
    lib = _load()
    return np.array([lib.orc_half_to_double(int(b)) for b in np.asarray(bits).ravel()])


def psnr(img, ref):
    """O9: 10 log10(1 / MSE) over pixels and RGB, linear and unclamped, peak 1."""
    img = np.asarray(img, dtype=np.float64)[..., :3]
    ref = np.asarray(ref, dtype=np.float64)[..., :3]
    mse = float(np.mean((img - ref) ** 2))
    return float("inf") if mse == 0.0 else 10.0 * np.log10(1.0 / mse)
