"""Python binding of the MI355X per-tile sort-last compositor (``include/dfb.h``).

Argument marshalling only: every step of the compositing path runs in the
HIP library ``libdfb.so`` built from ``csrc/``.  There is no fallback: if the
library is missing, :func:`load` raises.  PyTorch, when used, only provides
device memory and streams (load this module after ``import torch`` so both
share one HIP runtime).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from ._build import LIB_PATH, build  # noqa: F401

# ---------------------------------------------------------------- constants
DFB_OK = 0
DFB_ERR_INVALID_ARG = -1
DFB_ERR_STATE = -2
DFB_ERR_INCOMPLETE = -3
DFB_ERR_DUPLICATE = -4
DFB_ERR_BAD_VALUE = -5
DFB_ERR_OOM = -6
DFB_ERR_HIP = -7
DFB_ERR_UNSUPPORTED = -8
DFB_ERR_TREE = -9

DFB_OP_ALPHA_BLEND, DFB_OP_LIST, DFB_OP_AVERAGE = 0, 1, 2

DFB_F32, DFB_F16 = 0, 1
DFB_FMT_RGBA8, DFB_FMT_RGBAF32, DFB_FMT_NONE = 0, 1, 2
(DFB_BUF_FINAL, DFB_BUF_FINISHED_F32, DFB_BUF_ACCUM_F32, DFB_BUF_M2_F32,
 DFB_BUF_TILE_VARIANCE, DFB_BUF_SORT_ORDER, DFB_BUF_DENOISED_F32) = range(7)
DFB_VALIDATE, DFB_KEEP_SORT_ORDER, DFB_KEEP_FINISHED = 0x1, 0x2, 0x4
DFB_ACCUMULATE = 0x1
DFB_REPLAY = 0x2

# every symbol include/dfb.h declares
EXPORTED = (
    "dfb_create", "dfb_destroy", "dfb_set_fragments", "dfb_composite_frame", "dfb_accumulate",
    "dfb_reset_accumulation", "dfb_read_tiles", "dfb_buffer_bytes", "dfb_synchronize",
    "dfb_get_info", "dfb_set_timing", "dfb_kernel_ms", "dfb_kernel_times", "dfb_validate_layers", "dfb_last_error",
    "dfb_status_string", "dfb_set_background_image", "dfb_set_fragments_tree", "dfb_tree_create",
    "dfb_tree_destroy", "dfb_tree_new_frame", "dfb_tree_add", "dfb_tree_query",
    "dfb_assign_samples_host", "dfb_assign_samples", "dfb_composite_noalloc",
    # dfb_denoise.h
    "dfb_denoiser_param_count", "dfb_denoiser_create", "dfb_denoiser_destroy", "dfb_denoiser_set_params",
    "dfb_denoiser_get_params", "dfb_denoiser_forward", "dfb_denoiser_train_step",
    "dfb_denoiser_read_activation", "dfb_denoiser_frame_input", "dfb_denoise", "dfb_denoiser_last_error",
)


class Config(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("work_w", ctypes.c_int32), ("work_h", ctypes.c_int32),
                ("waves_per_tile", ctypes.c_int32), ("frag_dtype", ctypes.c_int32),
                ("format", ctypes.c_int32), ("background", ctypes.c_float * 4),
                ("tonemap_gamma", ctypes.c_float), ("flags", ctypes.c_uint32),
                ("tile_op", ctypes.c_int32), ("background_image", ctypes.c_void_p)]


class TreeNode(ctypes.Structure):
    _fields_ = [("generation", ctypes.c_int32), ("children", ctypes.c_int32)]


TREE_DTYPE = np.dtype([("generation", "<i4"), ("children", "<i4")])


class Layer(ctypes.Structure):
    _fields_ = [("tile_id", ctypes.c_int32), ("source_id", ctypes.c_uint32), ("block", ctypes.c_int64)]


LAYER_DTYPE = np.dtype([("tile_id", "<i4"), ("source_id", "<u4"), ("block", "<i8")])
assert LAYER_DTYPE.itemsize == ctypes.sizeof(Layer)


class Info(ctypes.Structure):
    _fields_ = [("n_tiles", ctypes.c_int32), ("tiles_x", ctypes.c_int32), ("tiles_y", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("max_layers_per_tile", ctypes.c_int32),
                ("work_w", ctypes.c_int32), ("work_h", ctypes.c_int32),
                ("waves_per_tile", ctypes.c_int32), ("accumulation_id", ctypes.c_int32),
                ("grid_size", ctypes.c_int32), ("n_fragments", ctypes.c_int64)]


class UnetConfig(ctypes.Structure):
    _fields_ = [("max_pixels", ctypes.c_int64), ("seed", ctypes.c_uint32), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float)]


class DfbError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("dfb status %d: %s" % (status, message))
        self.status = status


_lib = None


def load():
    """Load ``libdfb.so`` (built by ``build()``).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libdfb.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sig = {
        "dfb_create": ([ctypes.POINTER(Config), P, ctypes.POINTER(P)], I32),
        "dfb_destroy": ([P], I32),
        "dfb_set_fragments": ([P, P, I64, P, I32, P], I32),
        "dfb_composite_frame": ([P, U32], I32),
        "dfb_accumulate": ([P], I32),
        "dfb_reset_accumulation": ([P], I32),
        "dfb_read_tiles": ([P, I32, I32, I32, P, ctypes.c_int], I32),
        "dfb_buffer_bytes": ([P, I32, I32, I32], I64),
        "dfb_synchronize": ([P], I32),
        "dfb_get_info": ([P, ctypes.POINTER(Info)], I32),
        "dfb_set_timing": ([P, ctypes.c_int], I32),
        "dfb_kernel_ms": ([P], ctypes.c_double),
        "dfb_kernel_times": ([P, P, I32], I32),
        "dfb_validate_layers": ([ctypes.POINTER(Config), I64, P, I32, P, P], I32),
        "dfb_last_error": ([P], ctypes.c_char_p),
        "dfb_status_string": ([I32], ctypes.c_char_p),
        "dfb_set_background_image": ([P, P], I32),
        "dfb_set_fragments_tree": ([P, P, I64, P, P, I32, P], I32),
        "dfb_tree_create": ([I32, ctypes.POINTER(P)], I32),
        "dfb_tree_destroy": ([P], I32),
        "dfb_tree_new_frame": ([P], I32),
        "dfb_tree_add": ([P, I32, I32, I32, P], I32),
        "dfb_tree_query": ([P, I32, P, P, P], I32),
        "dfb_assign_samples_host": ([P, I32, I64, P], I32),
        "dfb_assign_samples": ([P, I64, P], I32),
        "dfb_composite_noalloc": ([ctypes.POINTER(Config), P, P, P, I32, P, P, P], I32),
        "dfb_denoiser_param_count": ([], I64),
        "dfb_denoiser_create": ([ctypes.POINTER(UnetConfig), P, ctypes.POINTER(P)], I32),
        "dfb_denoiser_destroy": ([P], I32),
        "dfb_denoiser_set_params": ([P, P, I64], I32),
        "dfb_denoiser_get_params": ([P, I32, P, I64], I32),
        "dfb_denoiser_forward": ([P, P, P, I32, I32, I32], I32),
        "dfb_denoiser_train_step": ([P, P, P, I32, I32, I32, ctypes.c_float, I32, P], I32),
        "dfb_denoiser_read_activation": ([P, I32, P, I64], I32),
        "dfb_denoiser_frame_input": ([P, P], I32),
        "dfb_denoise": ([P, P, ctypes.c_float], I32),
        "dfb_denoiser_last_error": ([P], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(status, handle=None, net=None):
    if status != DFB_OK:
        lib = load()
        if net is not None:
            msg = lib.dfb_denoiser_last_error(net).decode(errors="replace")
        else:
            msg = lib.dfb_last_error(handle).decode(errors="replace")
        raise DfbError(status, msg or lib.dfb_status_string(status).decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data_as(ctypes.c_void_p)
    if hasattr(a, "data_ptr"):
        return ctypes.c_void_p(a.data_ptr())
    return ctypes.c_void_p(int(a))


def make_config(width, height, tile_w=64, tile_h=None, *, work=0, waves=0, dtype=DFB_F32,
                fmt=DFB_FMT_RGBA8, background=(0.0, 0.0, 0.0, 0.0), gamma=1.0, flags=0,
                op=DFB_OP_ALPHA_BLEND, background_image=None):
    """``background_image``: a device pointer (int) or a tensor with data_ptr()."""
    tile_h = tile_w if tile_h is None else tile_h
    ww, wh = (work, work) if isinstance(work, int) else work
    bgi = None if background_image is None else _ptr(background_image).value
    return Config(width, height, tile_w, tile_h, ww, wh, waves, dtype, fmt,
                  (ctypes.c_float * 4)(*background), gamma, flags, op, bgi)


def as_layers(layers):
    """numpy record array with fields tile_id, source_id, block -> C layout
    (returned as is when it already is one)."""
    if isinstance(layers, np.ndarray) and layers.dtype == LAYER_DTYPE and layers.flags.c_contiguous:
        return layers
    out = np.empty(len(layers), dtype=LAYER_DTYPE)
    for f in LAYER_DTYPE.names:
        out[f] = np.asarray(layers[f])
    return out


# ---------------------------------------------------------- the C calls
def dfb_create(cfg: Config, stream=0):
    lib = load()
    h = ctypes.c_void_p()
    _check(lib.dfb_create(ctypes.byref(cfg), ctypes.c_void_p(int(stream)), ctypes.byref(h)))
    return h


def dfb_destroy(h):
    _check(load().dfb_destroy(h))


def dfb_set_fragments(h, frag_dev, n_blocks, layers, expected=None):
    lay = as_layers(layers)
    exp = None if expected is None else np.ascontiguousarray(expected, dtype=np.int32)
    _check(load().dfb_set_fragments(h, _ptr(frag_dev), int(n_blocks), _ptr(lay), len(lay), _ptr(exp)), h)


def dfb_composite_frame(h, frame_flags=0):
    _check(load().dfb_composite_frame(h, frame_flags), h)


def dfb_accumulate(h):
    _check(load().dfb_accumulate(h), h)


def dfb_reset_accumulation(h):
    _check(load().dfb_reset_accumulation(h), h)


def dfb_buffer_bytes(h, which, first_tile, n_tiles):
    return int(load().dfb_buffer_bytes(h, which, first_tile, n_tiles))


def dfb_read_tiles(h, which, first_tile, n_tiles, dst, dst_is_device=False):
    _check(load().dfb_read_tiles(h, which, first_tile, n_tiles, _ptr(dst), int(bool(dst_is_device))), h)


def dfb_synchronize(h):
    _check(load().dfb_synchronize(h), h)


def dfb_get_info(h) -> Info:
    info = Info()
    _check(load().dfb_get_info(h, ctypes.byref(info)), h)
    return info


def dfb_set_timing(h, every=1):
    """Time every ``every``-th composite (True: each one; False or 0: none)."""
    _check(load().dfb_set_timing(h, int(every)), h)


def dfb_kernel_ms(h) -> float:
    return float(load().dfb_kernel_ms(h))


def dfb_kernel_times(h):
    """Every per-frame timing (ms) since dfb_set_timing, in frame order."""
    lib = load()
    n = lib.dfb_kernel_times(h, None, 0)
    if n < 0:
        raise DfbError(DFB_ERR_HIP, "dfb_kernel_times")
    out = np.zeros(n, dtype=np.float32)
    if n:
        lib.dfb_kernel_times(h, out.ctypes.data, n)
    return out


def dfb_validate_layers(cfg: Config, n_blocks, layers, expected=None):
    """Host-only validation; returns per-tile counts or raises DfbError."""
    lib = load()
    lay = as_layers(layers)
    n_tiles = (-(-cfg.width // cfg.tile_w)) * (-(-cfg.height // cfg.tile_h))
    counts = np.zeros(n_tiles, dtype=np.int32)
    exp = None if expected is None else np.ascontiguousarray(expected, dtype=np.int32)
    _check(lib.dfb_validate_layers(ctypes.byref(cfg), int(n_blocks), _ptr(lay), len(lay), _ptr(exp), _ptr(counts)))
    return counts


def dfb_set_background_image(h, image_dev):
    _check(load().dfb_set_background_image(h, _ptr(image_dev)), h)


def as_tree(tree):
    """numpy record array with fields generation, children -> C layout."""
    if isinstance(tree, np.ndarray) and tree.dtype == TREE_DTYPE and tree.flags.c_contiguous:
        return tree
    out = np.empty(len(tree), dtype=TREE_DTYPE)
    for f in TREE_DTYPE.names:
        out[f] = np.asarray(tree[f])
    return out


def dfb_set_fragments_tree(h, frag_dev, n_blocks, layers, tree, bg_children):
    lay = as_layers(layers)
    tr = as_tree(tree)
    if len(tr) != len(lay):
        raise ValueError("one tree node per layer")
    bgc = np.ascontiguousarray(bg_children, dtype=np.int32)
    _check(load().dfb_set_fragments_tree(h, _ptr(frag_dev), int(n_blocks), _ptr(lay), _ptr(tr), len(lay),
                                         _ptr(bgc)), h)


def dfb_assign_samples_host(variance, extra):
    """Host-only largest-remainder assignment; returns int32[n_tiles]."""
    v = np.ascontiguousarray(variance, dtype=np.float32)
    counts = np.zeros(len(v), dtype=np.int32)
    st = load().dfb_assign_samples_host(_ptr(v), len(v), int(extra), _ptr(counts))
    if st != DFB_OK:
        raise DfbError(st, load().dfb_status_string(st).decode())
    return counts


NOALLOC_MAX_WORK = 1048576


def dfb_composite_noalloc(cfg: Config, frag_dev, tile_off_dev, layer_off_dev, max_layers, final_dev,
                          finished_dev=None, stream=0):
    """One plain frame into caller-owned device outputs, with no allocation
    (device CSR tables: tile_off int32[n_tiles + 1], layer_off int64 element
    offsets block * 5 * P, each tile's layers by ascending source id)."""
    st = load().dfb_composite_noalloc(ctypes.byref(cfg), _ptr(frag_dev), _ptr(tile_off_dev), _ptr(layer_off_dev),
                                      int(max_layers), _ptr(final_dev), _ptr(finished_dev), stream)
    _check(st)


def layer_tables(layers, n_tiles, P):
    """The per-tile layer table of a layer list, as dfb_composite_noalloc
    takes it (host arrays): tile_off int32[n_tiles + 1], layer_off int64
    (block * 5 * P, per tile by ascending source id) and the largest count."""
    lay = np.asarray(layers)
    counts = np.bincount(lay["tile_id"], minlength=n_tiles).astype(np.int64)
    off = np.zeros(n_tiles + 1, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    order = np.lexsort((lay["source_id"], lay["tile_id"]))
    layer_off = lay["block"][order].astype(np.int64) * 5 * P
    return off, layer_off, int(counts.max()) if n_tiles else 0


def dfb_assign_samples(h, extra, n_tiles):
    counts = np.zeros(n_tiles, dtype=np.int32)
    _check(load().dfb_assign_samples(h, int(extra), _ptr(counts)), h)
    return counts


class Tree:
    """Dependency-tree bookkeeping for tiles arriving one at a time (host)."""

    def __init__(self, n_tiles):
        self.lib = load()
        self.t = ctypes.c_void_p()
        st = self.lib.dfb_tree_create(int(n_tiles), ctypes.byref(self.t))
        if st != DFB_OK:
            raise DfbError(st, "dfb_tree_create")

    def close(self):
        if self.t:
            self.lib.dfb_tree_destroy(self.t)
            self.t = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def new_frame(self):
        self.lib.dfb_tree_new_frame(self.t)

    def add(self, tile_id, generation, children):
        """Returns (status, completed)."""
        done = ctypes.c_int32(0)
        st = self.lib.dfb_tree_add(self.t, int(tile_id), int(generation), int(children), ctypes.byref(done))
        return st, bool(done.value)

    def query(self, tile_id):
        """(state 1/0/-1, generation, missing)."""
        a, b, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        st = self.lib.dfb_tree_query(self.t, int(tile_id), ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        if st != DFB_OK:
            raise DfbError(st, "dfb_tree_query")
        return a.value, b.value, c.value


# ---------------------------------------------------------- convenience
class Compositor:
    """Owns a handle; reads results back into numpy arrays."""

    def __init__(self, cfg: Config, stream=0):
        self.cfg = cfg
        self.h = dfb_create(cfg, stream)
        self.P = cfg.tile_w * cfg.tile_h
        self.n_tiles = (-(-cfg.width // cfg.tile_w)) * (-(-cfg.height // cfg.tile_h))

    def close(self):
        if self.h:
            dfb_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_fragments(self, frag_dev, n_blocks, layers, expected=None):
        dfb_set_fragments(self.h, frag_dev, n_blocks, layers, expected)

    def set_fragments_tree(self, frag_dev, n_blocks, layers, tree, bg_children):
        dfb_set_fragments_tree(self.h, frag_dev, n_blocks, layers, tree, bg_children)

    def set_background_image(self, image_dev):
        dfb_set_background_image(self.h, image_dev)

    def assign_samples(self, extra):
        return dfb_assign_samples(self.h, extra, self.n_tiles)

    def composite(self, accumulate=False, replay=False):
        dfb_composite_frame(self.h, (DFB_ACCUMULATE if accumulate else 0) | (DFB_REPLAY if replay else 0))

    def accumulate(self):
        dfb_accumulate(self.h)

    def reset(self):
        dfb_reset_accumulation(self.h)

    def info(self):
        return dfb_get_info(self.h)

    def read(self, which, first_tile=0, n_tiles=None):
        n_tiles = self.n_tiles - first_tile if n_tiles is None else n_tiles
        nbytes = dfb_buffer_bytes(self.h, which, first_tile, n_tiles)
        buf = np.empty(nbytes, dtype=np.uint8)
        if nbytes:
            dfb_read_tiles(self.h, which, first_tile, n_tiles, buf)
        dfb_synchronize(self.h)
        P = self.P
        if which == DFB_BUF_FINAL:
            if self.cfg.format == DFB_FMT_RGBA8:
                return buf.reshape(n_tiles, P, 4)
            return buf.view(np.float32).reshape(n_tiles, P, 4)
        if which in (DFB_BUF_FINISHED_F32, DFB_BUF_ACCUM_F32):
            return buf.view(np.float32).reshape(n_tiles, P, 4)
        if which == DFB_BUF_M2_F32:
            return buf.view(np.float32).reshape(n_tiles, 3, P)
        if which == DFB_BUF_TILE_VARIANCE:
            return buf.view(np.float32)
        if which == DFB_BUF_SORT_ORDER:
            return buf.view(np.uint16)
        if which == DFB_BUF_DENOISED_F32:
            return buf.view(np.float32).reshape(n_tiles, P, 4)
        raise ValueError(which)


# ---------------------------------------------------------- denoiser (dfb_denoise.h)
UNET_CONV3 = [("enc1a", 6, 32, 0), ("enc1b", 32, 32, 0), ("enc2a", 32, 64, 1), ("enc2b", 64, 64, 1),
              ("enc3a", 64, 128, 2), ("enc3b", 128, 128, 2), ("up2", 128, 64, 1), ("dec2a", 128, 64, 1),
              ("dec2b", 64, 64, 1), ("up1", 64, 32, 0), ("dec1a", 64, 32, 0), ("dec1b", 32, 32, 0)]


def dfb_denoiser_param_count():
    return int(load().dfb_denoiser_param_count())


def dfb_denoiser_create(cfg: UnetConfig, stream=0):
    h = ctypes.c_void_p()
    _check(load().dfb_denoiser_create(ctypes.byref(cfg), ctypes.c_void_p(int(stream)), ctypes.byref(h)), net=None)
    return h


def dfb_denoiser_destroy(net):
    _check(load().dfb_denoiser_destroy(net), net=net)


def dfb_denoiser_set_params(net, flat):
    flat = np.ascontiguousarray(flat, dtype=np.float32)
    _check(load().dfb_denoiser_set_params(net, _ptr(flat), flat.size), net=net)


def dfb_denoiser_get_params(net, what=0):
    out = np.empty(dfb_denoiser_param_count(), dtype=np.float32)
    _check(load().dfb_denoiser_get_params(net, what, _ptr(out), out.size), net=net)
    return out


def dfb_denoiser_forward(net, in_dev, out_dev, n, h, w):
    _check(load().dfb_denoiser_forward(net, _ptr(in_dev), _ptr(out_dev), n, h, w), net=net)


def dfb_denoiser_train_step(net, in_dev, target_dev, n, h, w, lr, apply_update=True, want_loss=True):
    loss = ctypes.c_float(0.0)
    _check(load().dfb_denoiser_train_step(net, _ptr(in_dev), _ptr(target_dev), n, h, w, float(lr),
                                          int(bool(apply_update)),
                                          ctypes.byref(loss) if want_loss else None), net=net)
    return float(loss.value) if want_loss else None


def dfb_denoiser_read_activation(net, layer, n, h, w):
    lvl = UNET_CONV3[layer][3]
    co = UNET_CONV3[layer][2]
    hh, ww = h >> lvl, w >> lvl
    out = np.empty((n, hh, ww, co), dtype=np.uint16)
    _check(load().dfb_denoiser_read_activation(net, layer, _ptr(out), out.nbytes), net=net)
    return out


def dfb_denoiser_frame_input(h, in_dev):
    _check(load().dfb_denoiser_frame_input(h, _ptr(in_dev)), h)


def dfb_denoise(h, net, var_threshold):
    _check(load().dfb_denoise(h, net, float(var_threshold)), net=net)


def unet_params_to_flat(params):
    """Dict of per-layer arrays (names as UNET_CONV3 + 'out') -> flat ABI order."""
    parts = []
    for name, _, _, _ in UNET_CONV3:
        parts += [np.asarray(params[name + ".w"], np.float32).ravel(), np.asarray(params[name + ".b"], np.float32).ravel()]
    parts += [np.asarray(params["out.w"], np.float32).ravel(), np.asarray(params["out.b"], np.float32).ravel()]
    return np.concatenate(parts)


def unet_flat_to_params(flat):
    out, o = {}, 0
    for name, ci, co, _ in UNET_CONV3:
        out[name + ".w"] = flat[o:o + 9 * ci * co].reshape(3, 3, ci, co)
        o += 9 * ci * co
        out[name + ".b"] = flat[o:o + co]
        o += co
    out["out.w"] = flat[o:o + 96].reshape(32, 3)
    out["out.b"] = flat[o + 96:o + 99]
    return out


class Denoiser:
    """Owns a denoiser handle."""

    def __init__(self, max_pixels, seed=0, stream=0):
        self.net = dfb_denoiser_create(UnetConfig(int(max_pixels), seed, 0.0, 0.0, 0.0), stream)

    def close(self):
        if self.net:
            dfb_denoiser_destroy(self.net)
            self.net = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
