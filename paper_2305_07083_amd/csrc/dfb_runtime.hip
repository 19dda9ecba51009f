// Host runtime of the C ABI in include/dfb.h: handle, validation, the
// per-tile layer table (CSR), the longest-first work queue, the per-frame
// launches on the caller's stream, and the launch-shape autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/dfb.h"
#include "dfb_internal.h"
#include "dfb_tree.h"

namespace {

using dfb::FrameArgs;

std::string g_create_error;

enum class State { kEmpty, kReady, kComposited };

// A launch shape is chosen once per frame geometry, fragment type, tile
// operation and layer-count class (the register-sort capacity and the
// padded size of the largest tile's sort), so a new layer layout of the same
// class reuses it instead of autotuning again.  The caller's fixed work
// unit and wave count (0 = tuned) are part of the key: they restrict the
// candidates.
struct AutotuneKey {
  int device, width, height, tile_w, tile_h, dtype, op, kcap, lk, work_w, work_h, waves;
  bool operator<(const AutotuneKey& o) const {
    return std::tie(device, width, height, tile_w, tile_h, dtype, op, kcap, lk, work_w, work_h, waves) <
           std::tie(o.device, o.width, o.height, o.tile_w, o.tile_h, o.dtype, o.op, o.kcap, o.lk, o.work_w,
                    o.work_h, o.waves);
  }
};
struct Shape {
  int work_w, work_h, waves;
  int big_lds;  // LDS budget of the K > 32 path
};
std::map<AutotuneKey, Shape> g_autotune_cache;

}  // namespace

struct dfb_ctx {
  dfb_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 0;
  int tiles_x = 0, tiles_y = 0, n_tiles = 0, P = 0;
  State state = State::kEmpty;
  bool sticky_hip = false;
  std::string err;

  // device outputs
  float* finished = nullptr;
  float* accum = nullptr;
  float* m2 = nullptr;
  float* tile_var = nullptr;
  void* final_out = nullptr;
  uint16_t* order = nullptr;
  size_t order_cap = 0;
  float* denoised = nullptr;  // dfb_denoise result
  const float* bg_image = nullptr;  // borrowed background texture, or null
  int acc_n = 0;          // frames folded in
  bool have_finished = false;

  // per-frame layer table
  const void* frag = nullptr;
  int64_t n_blocks = 0;
  int n_layers = 0, max_k = 0;
  std::vector<int32_t> h_off;
  std::vector<dfb_layer> last_layers;
  std::vector<int32_t> last_expected;
  bool last_had_expected = false;
  // Two sets of device layer tables (per-tile offsets, layer offsets, work
  // list), used by successive layer layouts in turn, each uploaded from
  // pinned host staging: a new layout is written to the set the frames in
  // flight do not read, so its upload needs no wait for them.  A set is
  // reused two layouts later, after the event recorded when the frames
  // stopped using it.
  struct Tables {
    int32_t* off = nullptr;
    size_t off_cap = 0;
    int64_t* block = nullptr;
    size_t block_cap = 0;
    int32_t* work = nullptr;
    size_t work_cap = 0;
    int32_t* st_off = nullptr;   // pinned staging
    size_t st_off_cap = 0;
    int64_t* st_block = nullptr;
    size_t st_block_cap = 0;
    int32_t* st_work = nullptr;
    size_t st_work_cap = 0;
    hipEvent_t released = nullptr;  // the frames that read this set are done
    hipEvent_t staged[3] = {};      // uploads from st_off / st_block / st_work are done
    bool released_pending = false;
    bool staged_pending[3] = {};
  } tables[2];
  int cur_tables = 0;
  int32_t* d_off = nullptr;    // the current set's arrays
  int64_t* d_block = nullptr;
  int32_t* d_work = nullptr;
  float* d_var_partial = nullptr;
  size_t partial_cap = 0;
  uint32_t* d_flag = nullptr;
  uint32_t* d_queue_ring = nullptr;  // kQueues x kSlots counters, finish counters, FrameState
  dfb::FrameState* d_state = nullptr;  // inside d_queue_ring

  // Frame graphs for DFB_REPLAY: one per (fragment buffer, frame mode) of the
  // current layer table and launch shape; dropped when either changes.
  struct GraphEntry {
    const void* frag;
    uint32_t mode;
    hipGraph_t graph;
    hipGraphExec_t exec;
  };
  static constexpr int kMaxGraphs = 8;
  std::vector<GraphEntry> graphs;

  // launch shape
  Shape shape{0, 0, 0, 64 * 1024};
  bool shape_valid = false;
  int kcap = 8;
  int grid = 0;
  int n_work = 0;
  int subs_x = 1, subs_per_tile = 1;
  bool work_valid = false;  // d_work matches shape + layer table

  // timing: a ring of event pairs, harvested when a slot is reused; every
  // timing_every-th composite is timed (0: none)
  static constexpr int kRing = 64;
  int timing_every = 0;
  int64_t timing_seq = 0;
  hipEvent_t ev0[kRing] = {}, ev1[kRing] = {};
  bool pending[kRing] = {};
  int ring_pos = 0;
  double time_sum_ms = 0.0;
  int time_n = 0;
  std::vector<float> times_ms;  // every harvested timing since dfb_set_timing, in frame order
};

namespace {

dfb_status fail(dfb_ctx* h, dfb_status s, const std::string& msg) {
  if (h) h->err = msg;
  else g_create_error = msg;
  return s;
}

dfb_status hip_fail(dfb_ctx* h, hipError_t e, const char* what) {
  if (h) h->sticky_hip = true;
  return fail(h, DFB_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define DFB_HIP(h, call)                                    \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) return hip_fail((h), e_, #call);  \
  } while (0)

dfb_status check_config(const dfb_config* c, std::string& msg) {
  if (!c) { msg = "config is null"; return DFB_ERR_INVALID_ARG; }
  if (c->width <= 0 || c->height <= 0 || c->tile_w <= 0 || c->tile_h <= 0) {
    msg = "width, height, tile_w, tile_h must be positive";
    return DFB_ERR_INVALID_ARG;
  }
  if (static_cast<int64_t>(c->tile_w) * c->tile_h > 65536) {
    msg = "tile_w * tile_h must be <= 65536";
    return DFB_ERR_INVALID_ARG;
  }
  const int64_t tx = (c->width + c->tile_w - 1) / c->tile_w, ty = (c->height + c->tile_h - 1) / c->tile_h;
  if (tx * ty > (1 << 24) || tx * ty * c->tile_w * c->tile_h > (int64_t(1) << 31)) {
    msg = "framebuffer too large";
    return DFB_ERR_OOM;
  }
  if ((c->work_w == 0) != (c->work_h == 0)) {
    msg = "work_w and work_h must both be 0 (autotune) or both set";
    return DFB_ERR_INVALID_ARG;
  }
  if (c->work_w < 0 || c->work_h < 0 || (c->work_w && (c->tile_w % c->work_w || c->tile_h % c->work_h))) {
    msg = "work_w / work_h must divide tile_w / tile_h";
    return DFB_ERR_INVALID_ARG;
  }
  if (!(c->waves_per_tile == 0 || c->waves_per_tile == 1 || c->waves_per_tile == 2 || c->waves_per_tile == 4)) {
    msg = "waves_per_tile must be 0, 1, 2 or 4";
    return DFB_ERR_INVALID_ARG;
  }
  if (c->frag_dtype != DFB_F32 && c->frag_dtype != DFB_F16) { msg = "bad frag_dtype"; return DFB_ERR_INVALID_ARG; }
  if (c->format != DFB_FMT_RGBA8 && c->format != DFB_FMT_RGBAF32 && c->format != DFB_FMT_NONE) {
    msg = "bad format";
    return DFB_ERR_INVALID_ARG;
  }
  if (!(c->tonemap_gamma > 0.f) || !std::isfinite(c->tonemap_gamma)) { msg = "tonemap_gamma must be > 0"; return DFB_ERR_INVALID_ARG; }
  if (c->flags & ~(DFB_VALIDATE | DFB_KEEP_SORT_ORDER | DFB_KEEP_FINISHED)) { msg = "unknown flag"; return DFB_ERR_INVALID_ARG; }
  if (c->tile_op != DFB_OP_ALPHA_BLEND && c->tile_op != DFB_OP_LIST && c->tile_op != DFB_OP_AVERAGE) {
    msg = "tile_op must be DFB_OP_ALPHA_BLEND, DFB_OP_LIST or DFB_OP_AVERAGE";
    return DFB_ERR_INVALID_ARG;
  }
  if (c->tile_op == DFB_OP_AVERAGE && (c->flags & DFB_KEEP_SORT_ORDER)) {
    msg = "DFB_KEEP_SORT_ORDER has no meaning for DFB_OP_AVERAGE";
    return DFB_ERR_INVALID_ARG;
  }
  if (reinterpret_cast<uintptr_t>(c->background_image) % 16) {
    msg = "background_image must be 16-byte aligned";
    return DFB_ERR_INVALID_ARG;
  }
  return DFB_OK;
}

// Validation + per-tile counts (host, O(n_layers + n_tiles)).
dfb_status validate_layers(const dfb_config* c, int64_t n_blocks, const dfb_layer* layers, int32_t n_layers,
                           const int32_t* expected, std::vector<int32_t>& counts, std::string& msg) {
  dfb_status s = check_config(c, msg);
  if (s != DFB_OK) return s;
  const int tiles_x = (c->width + c->tile_w - 1) / c->tile_w;
  const int n_tiles = tiles_x * ((c->height + c->tile_h - 1) / c->tile_h);
  if (n_layers < 0 || n_blocks < 0 || (n_layers > 0 && !layers)) { msg = "bad layer list"; return DFB_ERR_INVALID_ARG; }
  counts.assign(n_tiles, 0);
  for (int32_t i = 0; i < n_layers; ++i) {
    const dfb_layer& L = layers[i];
    if (L.tile_id < 0 || L.tile_id >= n_tiles) {
      msg = "layer " + std::to_string(i) + ": tile_id " + std::to_string(L.tile_id) + " out of range";
      return DFB_ERR_INVALID_ARG;
    }
    if (L.block < 0 || L.block >= n_blocks) {
      msg = "layer " + std::to_string(i) + ": block " + std::to_string(L.block) + " out of range";
      return DFB_ERR_INVALID_ARG;
    }
    if (c->tile_op == DFB_OP_LIST && L.source_id == 0) {
      msg = "layer " + std::to_string(i) + ": DFB_OP_LIST takes the generation as source_id, and generation 0 "
            "is the background tile";
      return DFB_ERR_INVALID_ARG;
    }
    counts[L.tile_id]++;
  }
  for (int t = 0; t < n_tiles; ++t) {
    if (counts[t] > dfb::kMaxLayers) {
      msg = "tile " + std::to_string(t) + " has " + std::to_string(counts[t]) + " layers; at most " +
            std::to_string(dfb::kMaxLayers) + " are supported";
      return DFB_ERR_UNSUPPORTED;
    }
    if (expected && expected[t] != counts[t]) {
      msg = "tile " + std::to_string(t) + ": " + std::to_string(counts[t]) + " layers arrived, background declared " +
            std::to_string(expected[t]);
      return DFB_ERR_INCOMPLETE;
    }
  }
  return DFB_OK;
}

template <typename T>
dfb_status ensure(dfb_ctx* h, T*& ptr, size_t& cap, size_t count) {
  if (count <= cap && ptr) return DFB_OK;
  if (ptr) {
    DFB_HIP(h, hipStreamSynchronize(h->stream));
    DFB_HIP(h, hipFree(ptr));
    ptr = nullptr;
    cap = 0;
  }
  size_t n = std::max<size_t>(count, 1);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), n * sizeof(T));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    return fail(h, DFB_ERR_OOM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  cap = n;
  return DFB_OK;
}

dfb_status alloc_plain(dfb_ctx* h, void** ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 16));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *ptr = nullptr;
    return fail(h, DFB_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  return DFB_OK;
}

dfb_status check_usable(dfb_ctx* h) {
  if (!h) return DFB_ERR_INVALID_ARG;
  if (h->sticky_hip) return fail(h, DFB_ERR_HIP, "an earlier HIP error left the handle unusable: " + h->err);
  return DFB_OK;
}

int kcap_for(int max_k) { return max_k <= 8 ? 8 : (max_k <= 16 ? 16 : 32); }

// log2 of the padded sort size of a tile with max_k layers (the K > 32 path
// pads to a power of two of at least 64).
int layer_class(int max_k) {
  int lk = 0;
  while ((1 << lk) < max_k) ++lk;
  return lk;
}

// Candidate launch shapes: square work units of 16/32/64/128 that divide the
// tile (else the whole tile), and full-width strips of the same pixel count
// (a strip row is a whole tile row, so a unit's plane rows are contiguous in
// memory and fp16 rows fill whole cache lines), times 1/2/4 waves, times
// (frames with tiles of more than 128 layers) a small or a large LDS budget
// for the K > 32 path -- two workgroups per CU, or one with twice the pixels
// per sorting group.
std::vector<Shape> candidates(const dfb_config& c, int max_k) {
  std::vector<std::pair<int, int>> sizes;
  if (c.work_w) {
    sizes.push_back({c.work_w, c.work_h});
  } else {
    for (int s : {16, 32, 64, 128})
      if (c.tile_w % s == 0 && c.tile_h % s == 0) {
        sizes.push_back({s, s});
        const int h = s * s / c.tile_w;
        if (s < c.tile_w && (s * s) % c.tile_w == 0 && h >= 1 && c.tile_h % h == 0)
          sizes.push_back({c.tile_w, h});
      }
    if (sizes.empty()) sizes.push_back({c.tile_w, c.tile_h});
  }
  std::vector<int> waves;
  if (c.waves_per_tile) waves.push_back(c.waves_per_tile);
  else waves = {1, 2, 4};
  std::vector<int> ldss{dfb::big_lds_bytes(max_k)};
  if (max_k > 128 && c.tile_op == DFB_OP_ALPHA_BLEND) ldss.push_back(64 * 1024);
  std::vector<Shape> out;
  for (auto& s : sizes)
    for (int w : waves)
      for (int l : ldss) out.push_back({s.first, s.second, w, l});
  return out;
}

void drop_graphs(dfb_ctx* h);

// Device array of a table set, grown when too small.  Only called on a set
// no frame in flight reads (the other set's, or during the autotuner's
// synchronous sweep).
template <typename T>
dfb_status ensure_device_table(dfb_ctx* h, T*& ptr, size_t& cap, size_t count) {
  if (count <= cap && ptr) return DFB_OK;
  if (ptr) DFB_HIP(h, hipFree(ptr));
  ptr = nullptr;
  cap = 0;
  const size_t n = std::max<size_t>(count, 1);
  if (hipMalloc(reinterpret_cast<void**>(&ptr), n * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    return fail(h, DFB_ERR_OOM, "device allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  cap = n;
  return DFB_OK;
}

// Pinned staging buffer `which` of a set, ready to be written: waits for the
// last upload from it, grows it when too small.
template <typename T>
dfb_status stage(dfb_ctx* h, dfb_ctx::Tables& S, int which, T*& ptr, size_t& cap, size_t count) {
  if (S.staged_pending[which]) {
    DFB_HIP(h, hipEventSynchronize(S.staged[which]));
    S.staged_pending[which] = false;
  }
  if (count <= cap && ptr) return DFB_OK;
  if (ptr) DFB_HIP(h, hipHostFree(ptr));
  ptr = nullptr;
  cap = 0;
  const size_t n = std::max<size_t>(count, 1);
  if (hipHostMalloc(reinterpret_cast<void**>(&ptr), n * sizeof(T), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    ptr = nullptr;
    return fail(h, DFB_ERR_OOM, "pinned host allocation of " + std::to_string(n * sizeof(T)) + " bytes failed");
  }
  cap = n;
  return DFB_OK;
}

// Stream-ordered upload of a staged array; the staging is free again once
// the recorded event has passed.
template <typename T>
dfb_status upload(dfb_ctx* h, dfb_ctx::Tables& S, int which, T* dev, const T* staging, size_t count) {
  if (count) DFB_HIP(h, hipMemcpyAsync(dev, staging, count * sizeof(T), hipMemcpyHostToDevice, h->stream));
  if (!S.staged[which]) DFB_HIP(h, hipEventCreateWithFlags(&S.staged[which], hipEventDisableTiming));
  DFB_HIP(h, hipEventRecord(S.staged[which], h->stream));
  S.staged_pending[which] = true;
  return DFB_OK;
}

void free_tables(dfb_ctx* h) {
  for (auto& S : h->tables) {
    if (S.off) (void)hipFree(S.off);
    if (S.block) (void)hipFree(S.block);
    if (S.work) (void)hipFree(S.work);
    if (S.st_off) (void)hipHostFree(S.st_off);
    if (S.st_block) (void)hipHostFree(S.st_block);
    if (S.st_work) (void)hipHostFree(S.st_work);
    if (S.released) (void)hipEventDestroy(S.released);
    for (auto& e : S.staged)
      if (e) (void)hipEventDestroy(e);
    S = dfb_ctx::Tables{};
  }
}

// Work list for a shape: every (tile, unit) pair, tiles with more layers
// first (longest-processing-time order), ties by tile id.
dfb_status build_work(dfb_ctx* h, const Shape& s) {
  drop_graphs(h);
  const int sx = h->cfg.tile_w / s.work_w, sy = h->cfg.tile_h / s.work_h;
  h->subs_x = sx;
  h->subs_per_tile = sx * sy;
  h->n_work = h->n_tiles * h->subs_per_tile;
  std::vector<int32_t> tiles(h->n_tiles);
  for (int t = 0; t < h->n_tiles; ++t) tiles[t] = t;
  std::stable_sort(tiles.begin(), tiles.end(), [&](int a, int b) {
    return (h->h_off[a + 1] - h->h_off[a]) > (h->h_off[b + 1] - h->h_off[b]);
  });
  dfb_ctx::Tables& T = h->tables[h->cur_tables];
  const size_t n = static_cast<size_t>(h->n_work);
  dfb_status st = ensure_device_table(h, T.work, T.work_cap, n);
  if (st != DFB_OK) return st;
  st = ensure(h, h->d_var_partial, h->partial_cap, n);
  if (st != DFB_OK) return st;
  st = stage(h, T, 2, T.st_work, T.st_work_cap, n);
  if (st != DFB_OK) return st;
  size_t k = 0;
  for (int t : tiles)
    for (int u = 0; u < h->subs_per_tile; ++u) T.st_work[k++] = t * h->subs_per_tile + u;
  st = upload(h, T, 2, T.work, T.st_work, n);
  if (st != DFB_OK) return st;
  h->d_work = T.work;
  h->work_valid = true;
  return DFB_OK;
}

dfb_status ensure_accum(dfb_ctx* h) {
  if (h->accum) return DFB_OK;
  const size_t px = static_cast<size_t>(h->n_tiles) * h->P;
  dfb_status s = alloc_plain(h, reinterpret_cast<void**>(&h->accum), px * 16);
  if (s != DFB_OK) return s;
  s = alloc_plain(h, reinterpret_cast<void**>(&h->m2), px * 12);
  if (s != DFB_OK) return s;
  return DFB_OK;
}

// Launch arguments of a frame from the geometry alone: the buffers are
// filled in by the caller.
FrameArgs base_args(const dfb_config& c, int tiles_x, int n_tiles, const Shape& sh, const void* frag,
                    uint32_t mode) {
  FrameArgs a{};
  a.frag = frag;
  a.slot = a.clear_slot = 0;  // the kernel takes both from the device frame state
  a.n_queues = 1;             // set once the grid is known
  const int sx = c.tile_w / sh.work_w, sy = c.tile_h / sh.work_h;
  a.subs_x = sx;
  a.subs_per_tile = sx * sy;
  a.queue_block = a.subs_per_tile;
  a.n_work = n_tiles * a.subs_per_tile;
  a.width = c.width;
  a.height = c.height;
  a.tiles_x = tiles_x;
  a.n_tiles = n_tiles;
  a.tile_w = c.tile_w;
  a.tile_h = c.tile_h;
  a.P = c.tile_w * c.tile_h;
  a.work_w = sh.work_w;
  a.work_h = sh.work_h;
  a.work_px = sh.work_w * sh.work_h;
  a.big_lds = sh.big_lds;
  a.work_shift = -1;
  for (int k = 0; k < 16; ++k)
    if ((1 << k) == sh.work_w) a.work_shift = k;
  // 16-byte plane loads of V = 16 / sizeof(element) pixels need aligned
  // blocks (P % V == 0 follows from tile_w % V == 0) and rows of whole vectors
  const int V = c.frag_dtype == DFB_F16 ? 8 : 4;
  a.vec_ok = (reinterpret_cast<uintptr_t>(frag) % 16 == 0) && c.tile_w % V == 0 && sh.work_w % V == 0;
  for (int k = 0; k < 4; ++k) a.bg[k] = c.background[k];
  a.bg_image = c.background_image;
  a.inv_gamma = 1.f / c.tonemap_gamma;
  a.mode = mode;
  a.n_acc = 0;    // the kernel takes it from the device frame state
  a.inv_n = 1.f;
  return a;
}

FrameArgs make_args(dfb_ctx* h, uint32_t mode) {
  FrameArgs a = base_args(h->cfg, h->tiles_x, h->n_tiles, h->shape, h->frag, mode);
  a.bg_image = h->bg_image;
  a.finished = h->finished;
  a.accum = h->accum;
  a.m2 = h->m2;
  a.tile_var = h->tile_var;
  a.var_partial = h->d_var_partial;
  a.final_out = h->final_out;
  a.order = h->order;
  return a;
}

uint32_t display_mode(const dfb_config& c) {
  uint32_t m = 0;
  if (c.format == DFB_FMT_RGBA8) m |= dfb::kModeFmtRGBA8;
  if (c.format == DFB_FMT_RGBAF32) m |= dfb::kModeFmtF32;
  if (c.tonemap_gamma != 1.f) m |= dfb::kModeGamma;
  return m;
}

// Persistent grid: as many workgroups as fit on the chip at once, at most
// one per work unit.
dfb_status grid_of(dfb_ctx* h, const void* func, int threads, size_t lds, int n_work, int n_cu, int& grid) {
  int per_cu = 0;
  DFB_HIP(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, func, threads, lds));
  if (per_cu < 1) return fail(h, DFB_ERR_UNSUPPORTED, "kernel does not fit on a compute unit with this shape");
  grid = std::max(1, std::min(n_work, per_cu * n_cu));
  return DFB_OK;
}

dfb_status grid_for(dfb_ctx* h, const void* func, int threads, size_t lds, int& grid) {
  return grid_of(h, func, threads, lds, h->n_work, h->n_cu, grid);
}

dfb::VarianceArgs make_var_args(dfb_ctx* h) {
  dfb::VarianceArgs v{};
  v.var_partial = h->d_var_partial;
  v.tile_var = h->tile_var;
  v.n_tiles = h->n_tiles;
  v.subs_per_tile = h->subs_per_tile;
  v.tiles_x = h->tiles_x;
  v.width = h->cfg.width;
  v.height = h->cfg.height;
  v.tile_w = h->cfg.tile_w;
  v.tile_h = h->cfg.tile_h;
  v.state = h->d_state;
  return v;
}

// Everything one frame's launches take: one or two persistent frame
// kernels over the same work list -- the LDS-sort kernel for the tiles with
// more than kRegMax layers (alpha-blend frames that have such tiles), then
// the register-path kernel for the others, whose last workgroup advances the
// frame state -- and, for accumulating frames, the per-tile variance
// combine.  Nothing in it changes from frame to frame (the frame's counter
// slot and accumulation count live in the device frame state), so the same
// launches serve as a graph replayed every frame.
struct KernelLaunch {
  const void* func;
  int grid, threads;
  size_t lds;
  FrameArgs fa;
  const int32_t* tab_off;
  const int64_t* tab_layer;
  const int32_t* tab_work;
  void* params[4];
  void bind() {
    params[0] = &fa;
    params[1] = &tab_off;
    params[2] = &tab_layer;
    params[3] = &tab_work;
  }
};

struct FrameLaunch {
  int nk;
  KernelLaunch k[2];
  bool acc;
  dfb::VarianceArgs va;
  void* vparams[1];
  void bind() {
    for (int i = 0; i < nk; ++i) k[i].bind();
    vparams[0] = &va;
  }
};

// The frame kernels of a frame (geometry args, queue allocation, tables and
// per-kernel buffers filled in by the caller's base): fills L.k[0..nk).
dfb_status plan_kernels(dfb_ctx* h, const dfb_config& c, const FrameArgs& base, uint32_t* queue_base,
                        const Shape& sh, int max_k, int kcap, int n_work, int n_cu, const int32_t* tab_off,
                        const int64_t* tab_layer, const int32_t* tab_work, FrameLaunch& L) {
  const int threads = 64 * sh.waves;
  const bool sorting = c.tile_op == DFB_OP_ALPHA_BLEND;
  L.nk = 0;
  const bool big = sorting && max_k > dfb::kRegMax;
  for (int pass = big ? 0 : 1; pass < 2; ++pass) {
    KernelLaunch& K = L.k[L.nk++];
    const int kc = pass == 0 ? 0 : kcap;
    K.func = dfb::frame_kernel(c.frag_dtype, kc, c.tile_op);
    K.threads = threads;
    // the list and averaging operations keep nothing in LDS
    K.lds = sorting ? dfb::frame_lds_bytes(kc, threads, max_k, sh.big_lds) : 0;
    dfb_status st = grid_of(h, K.func, threads, K.lds, n_work, n_cu, K.grid);
    if (st != DFB_OK) return st;
    if (K.lds > 64 * 1024)
      DFB_HIP(h, hipFuncSetAttribute(K.func, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(K.lds)));
    K.fa = base;
    K.fa.queue = dfb::ring_of(queue_base, pass == 0 ? 1 : 0);
    K.fa.state = dfb::state_of(queue_base);
    K.fa.advance = pass == 1;
    K.fa.n_queues = std::min(dfb::kQueues, K.grid);
    K.tab_off = tab_off;
    K.tab_layer = tab_layer;
    K.tab_work = tab_work;
  }
  return DFB_OK;
}

dfb_status prepare_launch(dfb_ctx* h, uint32_t mode, FrameLaunch& L) {
  FrameArgs base = make_args(h, mode);
  dfb_status st = plan_kernels(h, h->cfg, base, h->d_queue_ring, h->shape, h->max_k, h->kcap, h->n_work, h->n_cu,
                               h->d_off, h->d_block, h->d_work, L);
  if (st != DFB_OK) return st;
  L.acc = (mode & dfb::kModeAccumulate) != 0;
  L.va = make_var_args(h);
  L.bind();
  return DFB_OK;
}

// Launch one frame with the current shape on the caller's stream.  With
// t0/t1 given, the two events bracket the frame kernels.
dfb_status launch_frame(dfb_ctx* h, uint32_t mode, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
  FrameLaunch L;
  dfb_status st = prepare_launch(h, mode, L);
  if (st != DFB_OK) return st;
  if (t0) DFB_HIP(h, hipEventRecord(t0, h->stream));
  for (int i = 0; i < L.nk; ++i)
    DFB_HIP(h, hipLaunchKernel(L.k[i].func, dim3(L.k[i].grid), dim3(L.k[i].threads), L.k[i].params, L.k[i].lds,
                               h->stream));
  if (t1) DFB_HIP(h, hipEventRecord(t1, h->stream));
  if (L.acc)
    DFB_HIP(h, hipLaunchKernel(dfb::tile_variance_kernel(), dim3((h->n_tiles + 255) / 256), dim3(256), L.vparams, 0,
                               h->stream));
  DFB_HIP(h, hipGetLastError());
  h->grid = L.k[L.nk - 1].grid;
  return DFB_OK;
}

void drop_graphs(dfb_ctx* h) {
  for (auto& g : h->graphs) {
    (void)hipGraphExecDestroy(g.exec);
    (void)hipGraphDestroy(g.graph);
  }
  h->graphs.clear();
}

// The frame graph for the current fragment buffer and mode (built on first
// use): the frame kernel node, then the variance node of an accumulating
// frame.  Built node by node, not by stream capture, so the handle's stream
// may be the null stream.
dfb_status frame_graph(dfb_ctx* h, uint32_t mode, hipGraphExec_t& exec) {
  for (auto& g : h->graphs)
    if (g.frag == h->frag && g.mode == mode) {
      exec = g.exec;
      return DFB_OK;
    }
  FrameLaunch L;
  dfb_status st = prepare_launch(h, mode, L);
  if (st != DFB_OK) return st;
  if (static_cast<int>(h->graphs.size()) >= dfb_ctx::kMaxGraphs) {
    (void)hipGraphExecDestroy(h->graphs.front().exec);
    (void)hipGraphDestroy(h->graphs.front().graph);
    h->graphs.erase(h->graphs.begin());
  }
  dfb_ctx::GraphEntry e{h->frag, mode, nullptr, nullptr};
  DFB_HIP(h, hipGraphCreate(&e.graph, 0));
  hipKernelNodeParams kp{};
  hipGraphNode_t fnode = nullptr, vnode = nullptr;
  hipError_t err = hipSuccess;
  for (int i = 0; i < L.nk && err == hipSuccess; ++i) {
    kp.func = const_cast<void*>(L.k[i].func);
    kp.gridDim = dim3(L.k[i].grid);
    kp.blockDim = dim3(L.k[i].threads);
    kp.sharedMemBytes = static_cast<unsigned>(L.k[i].lds);
    kp.kernelParams = L.k[i].params;
    kp.extra = nullptr;
    hipGraphNode_t prev = fnode;
    err = hipGraphAddKernelNode(&fnode, e.graph, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
  }
  if (err == hipSuccess && L.acc) {
    hipKernelNodeParams vp{};
    vp.func = const_cast<void*>(dfb::tile_variance_kernel());
    vp.gridDim = dim3((h->n_tiles + 255) / 256);
    vp.blockDim = dim3(256);
    vp.sharedMemBytes = 0;
    vp.kernelParams = L.vparams;
    vp.extra = nullptr;
    err = hipGraphAddKernelNode(&vnode, e.graph, &fnode, 1, &vp);
  }
  if (err == hipSuccess) err = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
  if (err != hipSuccess) {
    (void)hipGraphDestroy(e.graph);
    return hip_fail(h, err, "building the frame graph");
  }
  h->graphs.push_back(e);
  h->grid = L.k[L.nk - 1].grid;
  exec = e.exec;
  return DFB_OK;
}

// Whether the handle's stream is being captured into a graph by the caller.
bool capturing(dfb_ctx* h) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(h->stream, &cs) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return cs != hipStreamCaptureStatusNone;
}

// The device accumulation count after everything enqueued so far
// (synchronises the stream).  Graph replays of a captured accumulating frame
// advance it without the host seeing each one.
dfb_status read_acc_count(dfb_ctx* h, int32_t& n) {
  DFB_HIP(h, hipMemcpyAsync(&n, &h->d_state->n_acc, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  DFB_HIP(h, hipStreamSynchronize(h->stream));
  return DFB_OK;
}

// Stream-ordered update of the device accumulation count (value >= 0: set;
// < 0: add one).
dfb_status set_acc_count(dfb_ctx* h, int32_t value) {
  dfb::FrameState* st = h->d_state;
  void* params[] = {&st, &value};
  DFB_HIP(h, hipLaunchKernel(dfb::state_kernel(), dim3(1), dim3(64), params, 0, h->stream));
  DFB_HIP(h, hipGetLastError());
  return DFB_OK;
}

dfb_status autotune(dfb_ctx* h) {
  AutotuneKey key{h->device,      h->cfg.width,   h->cfg.height,          h->cfg.tile_w,
                  h->cfg.tile_h,  h->cfg.frag_dtype, h->cfg.tile_op,      h->kcap,
                  layer_class(h->max_k), h->cfg.work_w, h->cfg.work_h, h->cfg.waves_per_tile};
  auto cands = candidates(h->cfg, h->max_k);
  if (cands.size() == 1) {
    h->shape = cands[0];
    h->shape_valid = true;
    return build_work(h, h->shape);
  }
  auto it = g_autotune_cache.find(key);
  if (it != g_autotune_cache.end()) {
    h->shape = it->second;
    h->shape_valid = true;
    return build_work(h, h->shape);
  }
  hipEvent_t e0, e1;
  DFB_HIP(h, hipEventCreate(&e0));
  DFB_HIP(h, hipEventCreate(&e1));
  double best = 1e300;
  Shape best_s = cands[0];
  const uint32_t mode = display_mode(h->cfg);
  for (const Shape& s : cands) {
    h->shape = s;
    dfb_status st = build_work(h, s);
    if (st != DFB_OK) return st;
    std::vector<float> times;
    int warm = 5, timed = 5;  // frames longer than 5 ms: 1 warm-up, 3 timed
    for (int r = 0; r < warm + timed; ++r) {
      DFB_HIP(h, hipEventRecord(e0, h->stream));
      st = launch_frame(h, mode);
      if (st != DFB_OK) return st;
      DFB_HIP(h, hipEventRecord(e1, h->stream));
      DFB_HIP(h, hipEventSynchronize(e1));
      float ms = 0.f;
      DFB_HIP(h, hipEventElapsedTime(&ms, e0, e1));
      if (r == 0 && ms > 5.f) {
        warm = 1;
        timed = 3;
      }
      if (r >= warm) times.push_back(ms);
    }
    std::sort(times.begin(), times.end());
    const double med = times[times.size() / 2];
    if (med < best) { best = med; best_s = s; }
  }
  DFB_HIP(h, hipEventDestroy(e0));
  DFB_HIP(h, hipEventDestroy(e1));
  g_autotune_cache[key] = best_s;
  h->shape = best_s;
  h->shape_valid = true;
  return build_work(h, best_s);
}

dfb_status harvest(dfb_ctx* h, int slot) {
  float ms = 0.f;
  DFB_HIP(h, hipEventSynchronize(h->ev1[slot]));
  DFB_HIP(h, hipEventElapsedTime(&ms, h->ev0[slot], h->ev1[slot]));
  h->time_sum_ms += ms;
  h->time_n += 1;
  h->times_ms.push_back(ms);
  h->pending[slot] = false;
  return DFB_OK;
}

dfb_status prepare_shape(dfb_ctx* h) {
  if (h->shape_valid && h->work_valid) return DFB_OK;
  return autotune(h);
}

// Device NaN scan of every layer's depth plane (DFB_VALIDATE).  Uses the
// block table already on the device.
dfb_status scan_nan(dfb_ctx* h, const void* frag_dev, const int64_t* layer_table, int n_layers) {
  if (n_layers == 0) return DFB_OK;
  DFB_HIP(h, hipMemsetAsync(h->d_flag, 0, sizeof(uint32_t), h->stream));
  dfb::ValidateArgs va{frag_dev, layer_table, n_layers, h->P, h->d_flag};
  void* params[] = {&va};
  DFB_HIP(h, hipLaunchKernel(dfb::validate_kernel(h->cfg.frag_dtype), dim3(n_layers), dim3(256), params, 0,
                             h->stream));
  uint32_t bad = 0;
  DFB_HIP(h, hipMemcpyAsync(&bad, h->d_flag, sizeof(uint32_t), hipMemcpyDeviceToHost, h->stream));
  DFB_HIP(h, hipStreamSynchronize(h->stream));
  if (bad) return fail(h, DFB_ERR_BAD_VALUE, "a fragment depth is NaN");
  return DFB_OK;
}

}  // namespace

namespace dfb {
dfb_status frame_view(dfb_ctx* h, FrameView* v, bool want_denoised) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (!v) return DFB_ERR_INVALID_ARG;
  if (!h->accum || h->acc_n < 1) return fail(h, DFB_ERR_STATE, "no accumulated frame");
  if (want_denoised && !h->denoised) {
    s = alloc_plain(h, reinterpret_cast<void**>(&h->denoised), static_cast<size_t>(h->n_tiles) * h->P * 16);
    if (s != DFB_OK) return s;
  }
  v->glue.accum = h->accum;
  v->glue.tile_var = h->tile_var;
  v->glue.width = h->cfg.width;
  v->glue.height = h->cfg.height;
  v->glue.tiles_x = h->tiles_x;
  v->glue.tile_w = h->cfg.tile_w;
  v->glue.tile_h = h->cfg.tile_h;
  v->glue.P = h->P;
  v->glue.state = h->d_state;
  v->final_out = h->final_out;
  v->denoised = h->denoised;
  v->display_mode = display_mode(h->cfg);
  v->inv_gamma = 1.f / h->cfg.tonemap_gamma;
  v->stream = h->stream;
  return DFB_OK;
}
}  // namespace dfb

// Scratch of dfb_composite_noalloc (the entry point for callers that cannot
// allocate): the work queue's counters, finish counters and frame state
// (kQueueWords words), then the longest-first work list of at most
// DFB_NOALLOC_MAX_WORK units.  One copy per device, held until the process
// ends.  Host code uses it only through the device address that
// hipGetSymbolAddress returns for the current device, never by its name.
namespace {
constexpr int64_t kScratchWords = dfb::kQueueWords + DFB_NOALLOC_MAX_WORK;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices] = {};  // device address of scratch, per device
bool g_scratch_zeroed[kScratchDevices] = {};

// The current device's scratch address, looked up once per device (with
// that device current).  *first is set when this call is the device's
// first: the caller then clears the scratch, stream-ordered before use.
dfb_status scratch_of_current_device(void** out, bool* first) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kScratchDevices) return fail(nullptr, DFB_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  *first = !g_scratch_zeroed[dev];
  g_scratch_zeroed[dev] = true;
  return DFB_OK;
}
}  // namespace

extern "C" {

const char* dfb_status_string(dfb_status s) {
  switch (s) {
    case DFB_OK: return "ok";
    case DFB_ERR_INVALID_ARG: return "invalid argument";
    case DFB_ERR_STATE: return "call out of order";
    case DFB_ERR_INCOMPLETE: return "incomplete dependency tree";
    case DFB_ERR_DUPLICATE: return "duplicate (tile, source)";
    case DFB_ERR_BAD_VALUE: return "bad value (NaN depth)";
    case DFB_ERR_OOM: return "out of memory";
    case DFB_ERR_HIP: return "HIP error";
    case DFB_ERR_UNSUPPORTED: return "unsupported";
    case DFB_ERR_TREE: return "dependency tree received more tiles than declared";
  }
  return "unknown status";
}

const char* dfb_last_error(dfb_handle h) { return h ? h->err.c_str() : g_create_error.c_str(); }

dfb_status dfb_validate_layers(const dfb_config* cfg, int64_t n_blocks, const dfb_layer* layers, int32_t n_layers,
                               const int32_t* expected, int32_t* counts) {
  std::vector<int32_t> c;
  std::string msg;
  dfb_status s = validate_layers(cfg, n_blocks, layers, n_layers, expected, c, msg);
  if (s == DFB_OK) {
    // duplicates: sort (tile, source) pairs
    std::vector<std::pair<int32_t, uint32_t>> ts(n_layers);
    for (int i = 0; i < n_layers; ++i) ts[i] = {layers[i].tile_id, layers[i].source_id};
    std::sort(ts.begin(), ts.end());
    for (int i = 1; i < n_layers; ++i)
      if (ts[i] == ts[i - 1]) {
        msg = "tile " + std::to_string(ts[i].first) + ": source " + std::to_string(ts[i].second) + " appears twice";
        s = DFB_ERR_DUPLICATE;
        break;
      }
  }
  if (s == DFB_OK && counts) std::copy(c.begin(), c.end(), counts);
  g_create_error = msg;
  return s;
}

dfb_status dfb_create(const dfb_config* cfg, void* hip_stream, dfb_handle* out) {
  if (!out) return fail(nullptr, DFB_ERR_INVALID_ARG, "out is null");
  *out = nullptr;
  std::string msg;
  dfb_status s = check_config(cfg, msg);
  if (s != DFB_OK) return fail(nullptr, s, msg);
  dfb_ctx* h = new (std::nothrow) dfb_ctx();
  if (!h) return fail(nullptr, DFB_ERR_OOM, "host allocation failed");
  h->cfg = *cfg;
  h->bg_image = cfg->background_image;
  h->stream = static_cast<hipStream_t>(hip_stream);
  auto bail = [&](dfb_status st) {
    g_create_error = h->err;
    dfb_destroy(h);
    return st;
  };
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) { hip_fail(h, e, "hipGetDevice"); return bail(DFB_ERR_HIP); }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, h->device);
  if (e != hipSuccess) { hip_fail(h, e, "hipGetDeviceProperties"); return bail(DFB_ERR_HIP); }
  h->n_cu = prop.multiProcessorCount;
  h->tiles_x = (cfg->width + cfg->tile_w - 1) / cfg->tile_w;
  h->tiles_y = (cfg->height + cfg->tile_h - 1) / cfg->tile_h;
  h->n_tiles = h->tiles_x * h->tiles_y;
  h->P = cfg->tile_w * cfg->tile_h;
  const size_t px = static_cast<size_t>(h->n_tiles) * h->P;
  if (cfg->flags & DFB_KEEP_FINISHED) {
    if ((s = alloc_plain(h, reinterpret_cast<void**>(&h->finished), px * 16)) != DFB_OK) return bail(s);
  }
  if (cfg->format == DFB_FMT_RGBA8) {
    if ((s = alloc_plain(h, &h->final_out, px * 4)) != DFB_OK) return bail(s);
  } else if (cfg->format == DFB_FMT_RGBAF32) {
    if ((s = alloc_plain(h, &h->final_out, px * 16)) != DFB_OK) return bail(s);
  }
  if ((s = alloc_plain(h, reinterpret_cast<void**>(&h->tile_var), h->n_tiles * sizeof(float))) != DFB_OK) return bail(s);
  const size_t queue_bytes = sizeof(uint32_t) * dfb::kQueueWords;
  static_assert(dfb::kSlots <= dfb::kQueueStride, "a queue's slots fit in its stride");
  if ((s = alloc_plain(h, reinterpret_cast<void**>(&h->d_queue_ring), queue_bytes)) != DFB_OK) return bail(s);
  h->d_state = dfb::state_of(h->d_queue_ring);
  if ((s = alloc_plain(h, reinterpret_cast<void**>(&h->d_flag), 64)) != DFB_OK) return bail(s);
  e = hipMemsetAsync(h->d_queue_ring, 0, queue_bytes, h->stream);
  if (e == hipSuccess) e = hipMemsetAsync(h->tile_var, 0, h->n_tiles * sizeof(float), h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) { hip_fail(h, e, "initialising device state"); return bail(DFB_ERR_HIP); }
  *out = h;
  return DFB_OK;
}

dfb_status dfb_destroy(dfb_handle h) {
  if (!h) return DFB_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(h->stream);
  drop_graphs(h);
  for (int i = 0; i < dfb_ctx::kRing; ++i) {
    if (h->ev0[i]) (void)hipEventDestroy(h->ev0[i]);
    if (h->ev1[i]) (void)hipEventDestroy(h->ev1[i]);
  }
  void* bufs[] = {h->finished, h->accum, h->m2, h->tile_var, h->final_out, h->order, h->denoised,
                  h->d_var_partial, h->d_queue_ring, h->d_flag};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  free_tables(h);
  delete h;
  return DFB_OK;
}

dfb_status dfb_set_fragments(dfb_handle h, const void* frag_dev, int64_t n_blocks, const dfb_layer* layers,
                             int32_t n_layers, const int32_t* expected) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (!frag_dev && n_layers > 0) return fail(h, DFB_ERR_INVALID_ARG, "frag_dev is null");
  // Fast path: same layer list as the previous frame, only the buffer moves.
  const bool same = h->state != State::kEmpty && n_layers == h->n_layers && n_blocks == h->n_blocks &&
                    (expected != nullptr) == h->last_had_expected &&
                    (n_layers == 0 || std::memcmp(layers, h->last_layers.data(), sizeof(dfb_layer) * n_layers) == 0) &&
                    (!expected || std::memcmp(expected, h->last_expected.data(), sizeof(int32_t) * h->n_tiles) == 0);
  if (same) {
    if (h->cfg.flags & DFB_VALIDATE) {
      s = scan_nan(h, frag_dev, h->d_block, n_layers);
      if (s != DFB_OK) return s;
    }
    h->frag = frag_dev;
    h->state = State::kReady;
    return DFB_OK;
  }
  std::vector<int32_t> counts;
  std::string msg;
  s = validate_layers(&h->cfg, n_blocks, layers, n_layers, expected, counts, msg);
  if (s != DFB_OK) return fail(h, s, msg);
  // CSR: layers grouped by tile, each tile's layers by ascending source id.
  std::vector<int32_t> off(h->n_tiles + 1, 0);
  for (int t = 0; t < h->n_tiles; ++t) off[t + 1] = off[t] + counts[t];
  std::vector<int32_t> idx(n_layers);
  {
    std::vector<int32_t> fill(off.begin(), off.end() - 1);
    for (int32_t i = 0; i < n_layers; ++i) idx[fill[layers[i].tile_id]++] = i;
  }
  std::vector<int64_t> block(n_layers);
  int max_k = 0;
  for (int t = 0; t < h->n_tiles; ++t) {
    auto b = idx.begin() + off[t], e = idx.begin() + off[t + 1];
    std::sort(b, e, [&](int32_t x, int32_t y) { return layers[x].source_id < layers[y].source_id; });
    for (auto it = b; it != e; ++it) {
      if (it != b && layers[*it].source_id == layers[*(it - 1)].source_id)
        return fail(h, DFB_ERR_DUPLICATE, "tile " + std::to_string(t) + ": source " +
                                              std::to_string(layers[*it].source_id) + " appears twice");
      block[it - idx.begin()] = layers[*it].block * 5 * static_cast<int64_t>(h->P);
    }
    max_k = std::max(max_k, counts[t]);
  }
  // Upload into the table set that no frame in flight reads (no wait for
  // the frames of the current layout).
  const bool first = !h->tables[h->cur_tables].off;
  const int nxt = first ? h->cur_tables : 1 - h->cur_tables;
  dfb_ctx::Tables& T = h->tables[nxt];
  if (T.released_pending) {  // frames of the layout before last: normally long done
    DFB_HIP(h, hipEventSynchronize(T.released));
    T.released_pending = false;
  }
  if ((s = ensure_device_table(h, T.off, T.off_cap, off.size())) != DFB_OK) return s;
  if ((s = ensure_device_table(h, T.block, T.block_cap, block.size())) != DFB_OK) return s;
  if ((s = stage(h, T, 0, T.st_off, T.st_off_cap, off.size())) != DFB_OK) return s;
  if ((s = stage(h, T, 1, T.st_block, T.st_block_cap, block.size())) != DFB_OK) return s;
  std::copy(off.begin(), off.end(), T.st_off);
  std::copy(block.begin(), block.end(), T.st_block);
  if ((s = upload(h, T, 0, T.off, T.st_off, off.size())) != DFB_OK) return s;
  if ((s = upload(h, T, 1, T.block, T.st_block, block.size())) != DFB_OK) return s;
  if (h->cfg.flags & DFB_VALIDATE) {
    s = scan_nan(h, frag_dev, T.block, n_layers);
    if (s != DFB_OK) {  // the frame is refused: set_fragments must come again before a composite
      h->state = State::kEmpty;
      h->n_layers = -1;
      return s;
    }
  }
  if (h->cfg.flags & DFB_KEEP_SORT_ORDER) {
    s = ensure(h, h->order, h->order_cap, static_cast<size_t>(n_layers) * h->P);
    if (s != DFB_OK) return s;
  }
  // graph replays in flight hold the old tables and shape
  if (!h->graphs.empty()) DFB_HIP(h, hipStreamSynchronize(h->stream));
  drop_graphs(h);
  if (!first) {  // the old set is free once the frames enqueued so far are done
    dfb_ctx::Tables& O = h->tables[h->cur_tables];
    if (!O.released) DFB_HIP(h, hipEventCreateWithFlags(&O.released, hipEventDisableTiming));
    DFB_HIP(h, hipEventRecord(O.released, h->stream));
    O.released_pending = true;
  }
  h->cur_tables = nxt;
  h->d_off = T.off;
  h->d_block = T.block;
  h->d_work = T.work;
  // a new launch shape only for a new layer-count class
  if (h->state == State::kEmpty || kcap_for(max_k) != h->kcap || layer_class(max_k) != layer_class(h->max_k))
    h->shape_valid = false;
  h->h_off.swap(off);
  h->n_layers = n_layers;
  h->n_blocks = n_blocks;
  h->max_k = max_k;
  h->kcap = kcap_for(max_k);
  h->frag = frag_dev;
  h->last_layers.assign(layers, layers + n_layers);
  h->last_had_expected = expected != nullptr;
  if (expected) h->last_expected.assign(expected, expected + h->n_tiles);
  h->work_valid = false;
  if (!h->shape_valid) {
    // fixed shapes skip the autotuner
    auto c = candidates(h->cfg, max_k);
    if (c.size() == 1) { h->shape = c[0]; h->shape_valid = true; }
  }
  if (h->shape_valid) {
    s = build_work(h, h->shape);
    if (s != DFB_OK) return s;
  }
  h->state = State::kReady;
  return DFB_OK;
}

dfb_status dfb_set_fragments_tree(dfb_handle h, const void* frag_dev, int64_t n_blocks, const dfb_layer* layers,
                                  const dfb_tree_node* tree, int32_t n_layers, const int32_t* bg_children) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (n_layers < 0 || (n_layers > 0 && (!layers || !tree)) || !bg_children)
    return fail(h, DFB_ERR_INVALID_ARG, "layers, tree and bg_children are required");
  std::vector<dfb::TileTree> trees(h->n_tiles);
  for (int t = 0; t < h->n_tiles; ++t) {
    trees[t].reset();
    bool done;
    if (bg_children[t] < 0) return fail(h, DFB_ERR_INVALID_ARG, "tile " + std::to_string(t) + ": negative children");
    trees[t].add(0, bg_children[t], done);
  }
  for (int32_t i = 0; i < n_layers; ++i) {
    const dfb_layer& L = layers[i];
    const dfb_tree_node& N = tree[i];
    if (L.tile_id < 0 || L.tile_id >= h->n_tiles)
      return fail(h, DFB_ERR_INVALID_ARG, "layer " + std::to_string(i) + ": tile_id out of range");
    if (N.generation < 1 || N.generation > dfb::kMaxGeneration || N.children < 0)
      return fail(h, DFB_ERR_INVALID_ARG, "layer " + std::to_string(i) + ": generation must be in [1, " +
                                              std::to_string(dfb::kMaxGeneration) + "], children >= 0");
    bool done;
    if (!trees[L.tile_id].add(N.generation, N.children, done))
      return fail(h, DFB_ERR_TREE, "tile " + std::to_string(L.tile_id) + ": layer " + std::to_string(i) +
                                       " is more than its dependency tree declared");
  }
  for (int t = 0; t < h->n_tiles; ++t)
    if (trees[t].state() != dfb::TileTree::kComplete)
      return fail(h, DFB_ERR_INCOMPLETE, "tile " + std::to_string(t) + ": generation " +
                                             std::to_string(trees[t].generation()) + " still waits for " +
                                             std::to_string(trees[t].missing()) + " tiles");
  if (h->cfg.tile_op != DFB_OP_LIST) return dfb_set_fragments(h, frag_dev, n_blocks, layers, n_layers, nullptr);
  // a list: one tile per generation, blended by generation
  std::vector<dfb_layer> byg(layers, layers + n_layers);
  for (int32_t i = 0; i < n_layers; ++i) {
    if (trees[layers[i].tile_id].count(tree[i].generation) != 1)
      return fail(h, DFB_ERR_INVALID_ARG, "tile " + std::to_string(layers[i].tile_id) +
                                              ": DFB_OP_LIST needs one tile per generation");
    byg[i].source_id = static_cast<uint32_t>(tree[i].generation);
  }
  return dfb_set_fragments(h, frag_dev, n_blocks, byg.data(), n_layers, nullptr);
}

dfb_status dfb_set_background_image(dfb_handle h, const float* image_dev) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (reinterpret_cast<uintptr_t>(image_dev) % 16)
    return fail(h, DFB_ERR_INVALID_ARG, "background image must be 16-byte aligned");
  h->bg_image = image_dev;
  h->cfg.background_image = image_dev;
  drop_graphs(h);
  return DFB_OK;
}

dfb_status dfb_assign_samples(dfb_handle h, int64_t extra, int32_t* counts) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (!counts || extra < 0 || extra > INT32_MAX) return fail(h, DFB_ERR_INVALID_ARG, "bad extra or counts");
  std::vector<float> v(h->n_tiles, INFINITY);  // uniform before two accumulated frames
  int32_t n_acc = 0;
  s = read_acc_count(h, n_acc);
  if (s != DFB_OK) return s;
  if (n_acc >= 2) {
    DFB_HIP(h, hipMemcpyAsync(v.data(), h->tile_var, v.size() * sizeof(float), hipMemcpyDeviceToHost, h->stream));
    DFB_HIP(h, hipStreamSynchronize(h->stream));
  }
  s = dfb::assign_samples(v.data(), h->n_tiles, extra, counts);
  if (s != DFB_OK) return fail(h, s, "sample assignment failed");
  return DFB_OK;
}

dfb_status dfb_composite_frame(dfb_handle h, uint32_t frame_flags) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (h->state == State::kEmpty) return fail(h, DFB_ERR_STATE, "dfb_set_fragments must come first");
  if (frame_flags & ~(DFB_ACCUMULATE | DFB_REPLAY)) return fail(h, DFB_ERR_INVALID_ARG, "unknown frame flag");
  const bool acc = (frame_flags & DFB_ACCUMULATE) != 0;
  const bool replay = (frame_flags & DFB_REPLAY) != 0;
  // Under the caller's stream capture nothing may synchronise or allocate:
  // the launch shape and the accumulation buffers must already exist.
  const bool captured = capturing(h);
  if (captured) {
    if (!(h->shape_valid && h->work_valid))
      return fail(h, DFB_ERR_STATE, "the first frame of a new layer layout chooses the launch shape "
                                    "(synchronously): composite it before capturing");
    if (acc && !h->accum)
      return fail(h, DFB_ERR_STATE, "accumulate one frame before capturing an accumulating frame");
    if (replay) return fail(h, DFB_ERR_INVALID_ARG, "DFB_REPLAY cannot be captured");
  }
  s = prepare_shape(h);
  if (s != DFB_OK) return s;
  uint32_t mode = display_mode(h->cfg);
  if (h->cfg.flags & DFB_KEEP_FINISHED) mode |= dfb::kModeKeepFinished;
  if (h->cfg.flags & DFB_KEEP_SORT_ORDER) mode |= dfb::kModeKeepOrder;
  if (acc) {
    s = ensure_accum(h);
    if (s != DFB_OK) return s;
    mode |= dfb::kModeAccumulate;
  }
  hipGraphExec_t exec = nullptr;
  if (replay) {
    s = frame_graph(h, mode, exec);
    if (s != DFB_OK) return s;
  }
  const int slot = h->ring_pos;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  const bool timed = !captured && h->timing_every > 0 && h->timing_seq++ % h->timing_every == 0;
  if (timed) {
    if (!h->ev0[slot]) {
      DFB_HIP(h, hipEventCreate(&h->ev0[slot]));
      DFB_HIP(h, hipEventCreate(&h->ev1[slot]));
    }
    if (h->pending[slot]) {
      s = harvest(h, slot);
      if (s != DFB_OK) return s;
    }
    t0 = h->ev0[slot];
    t1 = h->ev1[slot];
  }
  if (replay) {
    // the events bracket the whole graph (frame kernel and variance combine)
    if (t0) DFB_HIP(h, hipEventRecord(t0, h->stream));
    DFB_HIP(h, hipGraphLaunch(exec, h->stream));
    if (t1) DFB_HIP(h, hipEventRecord(t1, h->stream));
  } else {
    s = launch_frame(h, mode, t0, t1);
    if (s != DFB_OK) return s;
  }
  if (timed) {
    h->pending[slot] = true;
    h->ring_pos = (slot + 1) % dfb_ctx::kRing;
  }
  if (acc) h->acc_n += 1;
  // a frame folded into the accumulation already must not be folded again
  h->have_finished = (h->cfg.flags & DFB_KEEP_FINISHED) != 0 && !acc;
  h->state = State::kComposited;
  return DFB_OK;
}

dfb_status dfb_accumulate(dfb_handle h) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (h->state != State::kComposited || !h->have_finished)
    return fail(h, DFB_ERR_STATE, "dfb_accumulate needs a frame composited with DFB_KEEP_FINISHED and without "
                                  "DFB_ACCUMULATE, not accumulated yet");
  if (capturing(h) && !h->accum)
    return fail(h, DFB_ERR_STATE, "accumulate one frame before capturing dfb_accumulate");
  s = ensure_accum(h);
  if (s != DFB_OK) return s;
  dfb::AccumArgs a{};
  a.finished = h->finished;
  a.accum = h->accum;
  a.m2 = h->m2;
  a.tile_var = h->tile_var;
  a.final_out = h->final_out;
  a.width = h->cfg.width;
  a.height = h->cfg.height;
  a.tiles_x = h->tiles_x;
  a.n_tiles = h->n_tiles;
  a.tile_w = h->cfg.tile_w;
  a.tile_h = h->cfg.tile_h;
  a.P = h->P;
  a.inv_gamma = 1.f / h->cfg.tonemap_gamma;
  a.mode = display_mode(h->cfg);
  a.state = h->d_state;
  void* params[] = {&a};
  DFB_HIP(h, hipLaunchKernel(dfb::accumulate_kernel(), dim3(h->n_tiles), dim3(256), params, 0, h->stream));
  DFB_HIP(h, hipGetLastError());
  s = set_acc_count(h, -1);
  if (s != DFB_OK) return s;
  h->acc_n += 1;
  h->have_finished = false;  // one accumulation per finished frame
  return DFB_OK;
}

dfb_status dfb_reset_accumulation(dfb_handle h) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  s = set_acc_count(h, 0);
  if (s != DFB_OK) return s;
  h->acc_n = 0;
  return DFB_OK;
}

int64_t dfb_buffer_bytes(dfb_handle h, dfb_buffer which, int32_t first, int32_t n) {
  if (!h || first < 0 || n < 0 || first + n > h->n_tiles) return 0;
  const int64_t P = h->P;
  switch (which) {
    case DFB_BUF_FINAL:
      if (!h->final_out) return 0;
      return n * P * (h->cfg.format == DFB_FMT_RGBA8 ? 4 : 16);
    case DFB_BUF_FINISHED_F32: return h->finished ? n * P * 16 : 0;
    case DFB_BUF_ACCUM_F32: return h->accum ? n * P * 16 : 0;
    case DFB_BUF_M2_F32: return h->m2 ? n * P * 12 : 0;
    case DFB_BUF_TILE_VARIANCE: return n * 4;
    case DFB_BUF_SORT_ORDER:
      if (!h->order || h->h_off.empty()) return 0;
      return (static_cast<int64_t>(h->h_off[first + n]) - h->h_off[first]) * P * 2;
    case DFB_BUF_DENOISED_F32: return h->denoised ? n * P * 16 : 0;
  }
  return 0;
}

dfb_status dfb_read_tiles(dfb_handle h, dfb_buffer which, int32_t first, int32_t n, void* dst, int dst_is_device) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  if (!dst || first < 0 || n < 0 || first + n > h->n_tiles) return fail(h, DFB_ERR_INVALID_ARG, "bad tile range or dst");
  if (h->state != State::kComposited) return fail(h, DFB_ERR_STATE, "no composited frame to read");
  const int64_t bytes = dfb_buffer_bytes(h, which, first, n);
  if (bytes == 0 && n > 0) return fail(h, DFB_ERR_STATE, "buffer not available (flag or format not enabled)");
  const int64_t P = h->P;
  const char* src = nullptr;
  switch (which) {
    case DFB_BUF_FINAL: src = static_cast<const char*>(h->final_out) + first * P * (h->cfg.format == DFB_FMT_RGBA8 ? 4 : 16); break;
    case DFB_BUF_FINISHED_F32: src = reinterpret_cast<const char*>(h->finished) + first * P * 16; break;
    case DFB_BUF_ACCUM_F32: src = reinterpret_cast<const char*>(h->accum) + first * P * 16; break;
    case DFB_BUF_M2_F32: src = reinterpret_cast<const char*>(h->m2) + first * P * 12; break;
    case DFB_BUF_TILE_VARIANCE: src = reinterpret_cast<const char*>(h->tile_var) + first * 4; break;
    case DFB_BUF_SORT_ORDER: src = reinterpret_cast<const char*>(h->order) + static_cast<int64_t>(h->h_off[first]) * P * 2; break;
    case DFB_BUF_DENOISED_F32: src = reinterpret_cast<const char*>(h->denoised) + first * P * 16; break;
    default: return fail(h, DFB_ERR_INVALID_ARG, "unknown buffer");
  }
  if (bytes > 0)
    DFB_HIP(h, hipMemcpyAsync(dst, src, static_cast<size_t>(bytes),
                              dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream));
  return DFB_OK;
}

dfb_status dfb_synchronize(dfb_handle h) {
  dfb_status s = check_usable(h);
  if (s != DFB_OK) return s;
  DFB_HIP(h, hipStreamSynchronize(h->stream));
  return DFB_OK;
}

dfb_status dfb_get_info(dfb_handle h, dfb_info* out) {
  if (!h || !out) return DFB_ERR_INVALID_ARG;
  int32_t n_acc = h->acc_n;
  if (!h->sticky_hip) {
    dfb_status s = read_acc_count(h, n_acc);
    if (s != DFB_OK) return s;
  }
  out->n_tiles = h->n_tiles;
  out->tiles_x = h->tiles_x;
  out->tiles_y = h->tiles_y;
  out->n_layers = h->n_layers < 0 ? 0 : h->n_layers;
  out->max_layers_per_tile = h->max_k;
  out->work_w = h->shape.work_w;
  out->work_h = h->shape.work_h;
  out->waves_per_tile = h->shape.waves;
  out->accumulation_id = n_acc;
  out->grid_size = h->grid;
  out->n_fragments = static_cast<int64_t>(out->n_layers) * h->P;
  return DFB_OK;
}

dfb_status dfb_set_timing(dfb_handle h, int every) {
  if (!h) return DFB_ERR_INVALID_ARG;
  h->timing_every = every > 0 ? every : 0;
  h->timing_seq = 0;
  h->time_sum_ms = 0.0;
  h->time_n = 0;
  h->times_ms.clear();
  for (int i = 0; i < dfb_ctx::kRing; ++i) h->pending[i] = false;
  return DFB_OK;
}

// Harvest the pending timings oldest first (the ring is filled in order
// from ring_pos), so times_ms stays in frame order.
dfb_status harvest_all(dfb_ctx* h) {
  for (int k = 0; k < dfb_ctx::kRing; ++k) {
    const int i = (h->ring_pos + k) % dfb_ctx::kRing;
    if (h->pending[i]) {
      dfb_status s = harvest(h, i);
      if (s != DFB_OK) return s;
    }
  }
  return DFB_OK;
}

double dfb_kernel_ms(dfb_handle h) {
  if (!h) return -1.0;
  if (harvest_all(h) != DFB_OK) return -1.0;
  return h->time_n ? h->time_sum_ms / h->time_n : -1.0;
}

int32_t dfb_kernel_times(dfb_handle h, float* ms, int32_t cap) {
  if (!h || cap < 0 || (cap > 0 && !ms)) return -1;
  if (harvest_all(h) != DFB_OK) return -1;
  const int32_t n = static_cast<int32_t>(std::min<size_t>(h->times_ms.size(), static_cast<size_t>(cap)));
  std::copy(h->times_ms.begin(), h->times_ms.begin() + n, ms);
  return static_cast<int32_t>(h->times_ms.size());
}

dfb_status dfb_composite_noalloc(const dfb_config* cfg, const void* frag_dev, const int32_t* tile_off_dev,
                                 const int64_t* layer_off_dev, int32_t max_layers, void* final_dev,
                                 float* finished_dev, void* hip_stream) {
  std::string msg;
  dfb_status s = check_config(cfg, msg);
  if (s != DFB_OK) return fail(nullptr, s, msg);
  if (!cfg->work_w || !cfg->waves_per_tile)
    return fail(nullptr, DFB_ERR_INVALID_ARG, "set work_w, work_h and waves_per_tile: the autotuner needs buffers");
  if (cfg->flags & (DFB_VALIDATE | DFB_KEEP_SORT_ORDER))
    return fail(nullptr, DFB_ERR_UNSUPPORTED, "DFB_VALIDATE and DFB_KEEP_SORT_ORDER need buffers of their own");
  if (max_layers < 0 || max_layers > dfb::kMaxLayers)
    return fail(nullptr, DFB_ERR_INVALID_ARG, "max_layers must be in [0, 4096]");
  if (!tile_off_dev || (max_layers > 0 && (!frag_dev || !layer_off_dev)))
    return fail(nullptr, DFB_ERR_INVALID_ARG, "null fragment buffer or layer table");
  if (cfg->format != DFB_FMT_NONE && !final_dev) return fail(nullptr, DFB_ERR_INVALID_ARG, "final_dev is null");
  if ((cfg->flags & DFB_KEEP_FINISHED) && !finished_dev)
    return fail(nullptr, DFB_ERR_INVALID_ARG, "DFB_KEEP_FINISHED needs finished_dev");
  const int tiles_x = (cfg->width + cfg->tile_w - 1) / cfg->tile_w;
  const int n_tiles = tiles_x * ((cfg->height + cfg->tile_h - 1) / cfg->tile_h);
  const int64_t n_work = static_cast<int64_t>(n_tiles) * (cfg->tile_w / cfg->work_w) * (cfg->tile_h / cfg->work_h);
  if (n_work > DFB_NOALLOC_MAX_WORK)
    return fail(nullptr, DFB_ERR_UNSUPPORTED, "the frame has " + std::to_string(n_work) +
                                                  " work units; the static scratch holds at most " +
                                                  std::to_string(DFB_NOALLOC_MAX_WORK) + " (use larger work units)");
  void* base = nullptr;
  bool first = false;
  if ((s = scratch_of_current_device(&base, &first)) != DFB_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  uint32_t* queue = static_cast<uint32_t*>(base);
  int32_t* work = reinterpret_cast<int32_t*>(queue + dfb::kQueueWords);
  if (first) {  // counters and frame state start at zero; a fill kernel, no memset node
    int64_t words = kScratchWords;
    uint32_t zero = 0;
    void* fp[] = {&queue, &zero, &words};
    DFB_HIP(nullptr, hipLaunchKernel(dfb::fill_u32_kernel(), dim3(1024), dim3(256), fp, 0, st));
  }
  Shape sh{cfg->work_w, cfg->work_h, cfg->waves_per_tile, dfb::big_lds_bytes(max_layers)};
  uint32_t mode = display_mode(*cfg);
  if (cfg->flags & DFB_KEEP_FINISHED) mode |= dfb::kModeKeepFinished;
  FrameArgs a = base_args(*cfg, tiles_x, n_tiles, sh, frag_dev, mode);
  a.finished = finished_dev;
  a.final_out = final_dev;
  int dev = 0, n_cu = 0;
  DFB_HIP(nullptr, hipGetDevice(&dev));
  DFB_HIP(nullptr, hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev));
  FrameLaunch L;
  if ((s = plan_kernels(nullptr, *cfg, a, queue, sh, max_layers, kcap_for(max_layers), a.n_work, n_cu, tile_off_dev,
                        layer_off_dev, work, L)) != DFB_OK)
    return s;
  L.bind();
  int32_t nt = n_tiles, subs = a.subs_per_tile;
  void* lp[] = {&tile_off_dev, &nt, &subs, &work};
  DFB_HIP(nullptr, hipLaunchKernel(dfb::lpt_work_kernel(), dim3(1), dim3(dfb::kLptThreads), lp, 0, st));
  for (int i = 0; i < L.nk; ++i)
    DFB_HIP(nullptr, hipLaunchKernel(L.k[i].func, dim3(L.k[i].grid), dim3(L.k[i].threads), L.k[i].params,
                                     L.k[i].lds, st));
  DFB_HIP(nullptr, hipGetLastError());
  return DFB_OK;
}

}  // extern "C"
