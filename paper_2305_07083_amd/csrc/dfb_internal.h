// Internal interface between the host runtime (dfb_runtime.hip) and the
// gfx950 kernels (dfb_kernels.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dfb.h"

namespace dfb {

// Layers per tile handled by the register sort; above it, the workgroup-wide
// LDS sort takes over.
constexpr int kRegMax = 32;
// Largest layer count per tile the LDS sort supports (keys + weights of one
// pixel must fit the LDS budget below).
// Work queue: the work list is dealt round-robin to kQueues counters, each
// in its own 4 KB page, served first by the workgroups with the same index
// mod kQueues, so same-address atomics do not serialise the whole chip.
// Each counter has kSlots per-frame slots used as a ring: frame f counts in
// slot f mod kSlots and clears slot (f + kSlots/2) mod kSlots, which no
// frame in flight uses, so nothing is reset between frames.  A ring is the
// kQueues counter pages and one page of per-slot "workgroups finished"
// counters.  A frame with tiles of more than kRegMax layers runs two
// launches over the same work list -- the K > kRegMax tiles, then the rest
// -- each with a ring of its own; after the two rings comes one page
// holding the FrameState below.
constexpr int kQueues = 16;
constexpr int kQueueStride = 1024;  // 4-byte counters between queues
constexpr int kSlots = 64;
constexpr int kRingWords = (kQueues + 1) * kQueueStride;
constexpr int kQueueWords = 2 * kRingWords + kQueueStride;  // the whole allocation, in u32

// Per-handle frame state in device memory.  Kernels read it at their start
// and the last workgroup of a frame advances it, so a launch carries no
// per-frame value in its arguments and one captured frame can be replayed
// as every later frame.
struct FrameState {
  uint32_t seq;    // frames so far: selects the counter slot
  int32_t n_acc;   // frames folded into the running mean since the reset
};
// Ring r (0: the register-path launch, 1: the K > kRegMax launch) and the
// frame state inside a queue allocation.
inline uint32_t* ring_of(uint32_t* queue_base, int r) { return queue_base + r * kRingWords; }
inline FrameState* state_of(uint32_t* queue_base) {
  return reinterpret_cast<FrameState*>(queue_base + 2 * kRingWords);
}
constexpr int kMaxLayers = 4096;
// Largest LDS budget of the large-K path for keys (u64) and weights (f32);
// the host passes 64, 96 or 112 KB depending on the frame's largest tile.
constexpr int kBigLdsBytes = 112 * 1024;

enum ModeBits : uint32_t {
  kModeAccumulate = 1u,     // fold into the running mean + per-tile variance
  kModeKeepFinished = 2u,   // store the finished f32 tile
  kModeKeepOrder = 4u,      // store the per-pixel sorted order (debug)
  kModeFmtRGBA8 = 8u,       // display: RGBA8
  kModeFmtF32 = 16u,        // display: RGBA f32
  kModeGamma = 32u,         // colour ^ (1/gamma) before quantising
};

// Everything one frame launch needs besides the three read-only tables,
// which are separate __restrict__ kernel arguments so that their uniform
// reads become scalar loads:
//   tile_off   [n_tiles + 1] CSR offsets into layer_off
//   layer_off  [n_layers] element offset of each layer's block (block*5*P);
//              per tile ordered by source id
//   work_list  [n_work] work-unit ids, longest tile first
// Passed by value; nothing in it changes from frame to frame while the layer
// table, the fragment buffer and the launch shape stay the same.
struct FrameArgs {
  const void* frag;            // fragment blocks (caller's buffer)
  uint32_t* queue;             // this launch's ring: kQueues x kSlots counters, queues
                               // kQueueStride apart, then the kSlots finish counters
  FrameState* state;           // the frame state (shared by the frame's launches)
  int32_t advance;             // 1: the last workgroup advances the state (the frame's last launch)
  int32_t slot, clear_slot;    // set by the kernel from FrameState::seq
  int32_t n_queues;            // counters in use: min(kQueues, grid)
  int32_t queue_block;         // consecutive work-list positions per counter block (units per tile)
  int32_t n_work;
  int32_t width, height, tiles_x, n_tiles;
  int32_t tile_w, tile_h, P;
  int32_t work_w, work_h, subs_x, subs_per_tile, work_px;
  int32_t work_shift;          // log2(work_w) if a power of two, else -1
  int32_t big_lds;             // LDS bytes for keys + weights of the K > 32 path
  int32_t vec_ok;              // 16-byte plane loads possible (alignment, work_w, tile_w)
  float bg[4];
  const float* bg_image;       // [n_tiles][P][4] per-pixel background, or null
  float inv_gamma;
  uint32_t mode;
  int32_t n_acc;               // set by the kernel: accumulation id after this frame
  float inv_n;                 // set by the kernel: 1 / n_acc
  float* finished;             // [n_tiles][P][4]
  float* accum;                // [n_tiles][P][4]
  float* m2;                   // [n_tiles][3][P]
  float* tile_var;             // [n_tiles]
  float* var_partial;          // [n_work] M2 sum of each unit (accumulating frames)
  void* final_out;             // RGBA8 uint32[n_tiles][P] or float4[n_tiles][P]
  uint16_t* order;             // [n_layers][P]
};

struct AccumArgs {
  const float* finished;
  float* accum;
  float* m2;
  float* tile_var;
  void* final_out;
  int32_t width, height, tiles_x, n_tiles, tile_w, tile_h, P;
  float inv_gamma;
  uint32_t mode;
  const FrameState* state;     // n = state->n_acc + 1 (advanced by a separate launch)
};

struct VarianceArgs {
  const float* var_partial;    // [n_tiles * subs_per_tile]
  float* tile_var;             // [n_tiles]
  int32_t n_tiles, subs_per_tile, tiles_x, width, height, tile_w, tile_h;
  const FrameState* state;     // n = state->n_acc (already advanced by the frame kernel)
};

struct ValidateArgs {
  const void* frag;
  const int64_t* layer_off;
  int32_t n_layers, P;
  uint32_t* bad;   // set to 1 if a NaN depth is seen
};

// What the denoiser needs from a compositor handle: its accumulation.
struct FrameGlue {
  const float* accum;      // [T][P][4] running mean
  const float* tile_var;   // [T]
  const FrameState* state; // n = state->n_acc
  int width, height, tiles_x, tile_w, tile_h, P;
};
struct FrameView {
  FrameGlue glue;
  void* final_out;         // display buffer (or null for NONE)
  float* denoised;         // [T][P][4] (allocated on request)
  uint32_t display_mode;   // kModeFmt* | kModeGamma
  float inv_gamma;
  hipStream_t stream;
};
// Fails with DFB_ERR_STATE unless at least one frame has been accumulated.
dfb_status frame_view(dfb_ctx* h, FrameView* out, bool want_denoised);

// The persistent frame kernel for a fragment dtype, register-sort capacity
// and tile operation (dfb_tile_op).  dtype: 0 f32, 1 f16.  kcap 8, 16 or 32:
// the per-pixel sort of tiles with at most kcap layers in registers (tiles
// with more are left to the kcap 0 kernel); kcap 0 (ALPHA_BLEND only): the
// workgroup-wide LDS sort of the tiles with more than kRegMax layers, others
// left alone.
const void* frame_kernel(int dtype, int kcap, int op);
// Largest-remainder assignment of extra samples (host; dfb_assign_samples_host).
dfb_status assign_samples(const float* variance, int32_t n_tiles, int64_t extra, int32_t* counts);
const void* accumulate_kernel();
const void* tile_variance_kernel();
// One thread: state->n_acc = value (value >= 0), or += 1 (value < 0).
const void* state_kernel();
// (uint32_t* p, uint32_t v, int64_t n): p[0..n) = v, any grid.
const void* fill_u32_kernel();
// (const int32_t* tile_off, int32_t n_tiles, int32_t subs, int32_t* work):
// the longest-first work list, one workgroup of kLptThreads lanes.
const void* lpt_work_kernel();
constexpr int kLptThreads = 1024;
const void* validate_kernel(int dtype);

// LDS budget of the K > 32 path for a frame whose largest tile has
// max_layers layers, and the dynamic LDS bytes a frame launch needs (kcap as
// for frame_kernel).
int big_lds_bytes(int max_layers);
size_t frame_lds_bytes(int kcap, int threads, int max_layers, int big_lds);

}  // namespace dfb
