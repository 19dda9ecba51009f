// gfx950 kernels of the denoiser: BF16 MFMA implicit-GEMM conv3x3 forward,
// data gradient and weight gradient (FP32 accumulation), and the small
// elementwise / reduction kernels around them.  Every reduction has a fixed
// order (partials per chunk, then a sequential sum), so results are
// deterministic.
//
// The three convolutions are one GEMM shape, D[M][N] += A[M][K] B[K][N],
// read from LDS in K slices:
//   forward  M = c_out,  N = pixels, K = (tap, c_in)   A = W, B = x[p + tap]
//   dgrad    M = pixels, N = c_in,  K = (tap, c_out)  A = dy[p - tap], B = W^T
//   wgrad    M = c_in,   N = c_out, K = pixels (per tap, split over chunks)
// All three use v_mfma_f32_32x32x16_bf16.  Operand layout (checked on the
// device): lane l holds k = (l/32)*8 .. +7 of row/column l%32; the result
// element r of lane l is row 8*(r/4) + 4*(l/32) + r%4, column l%32.  In
// dgrad and wgrad a workgroup is 4 waves over a 64-row tile and every
// 32-column block of N: wave w takes 32x32 blocks w, w + 4, ...; with only
// two blocks (N = 32) two waves share a block, each taking half of the K
// steps, and their sums are added in a fixed order.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dfb_internal.h"
#include "unet_internal.h"

namespace dfb {
namespace unet {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int BM = 64;    // rows per workgroup tile
constexpr int LDK = 40;   // LDS row length in bf16 (32 + 8 padding)

__device__ __forceinline__ uint16_t to_bf16(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

__device__ __forceinline__ bf16x8 lds_frag(const uint16_t* p) {
  const uint4 v = *reinterpret_cast<const uint4*>(p);
  return __builtin_bit_cast(bf16x8, v);
}

struct Pix {
  int n, r, c;
  bool ok;
};
__device__ __forceinline__ Pix pixel_of(long long p, const Shape& s) {
  Pix q;
  q.ok = p < s.pixels();
  const long long hw = static_cast<long long>(s.h) * s.w;
  q.n = q.ok ? static_cast<int>(p / hw) : 0;
  const int rem = q.ok ? static_cast<int>(p - q.n * hw) : 0;
  q.r = rem / s.w;
  q.c = rem - q.r * s.w;
  return q;
}
__device__ __forceinline__ long long shifted(const Pix& q, int dr, int dc, const Shape& s, bool& in) {
  const int rr = q.r + dr, cc = q.c + dc;
  in = q.ok && rr >= 0 && rr < s.h && cc >= 0 && cc < s.w;
  return (static_cast<long long>(q.n) * s.h + rr) * s.w + cc;
}

// ------------------------------------------------------------- forward
// Persistent implicit-GEMM conv3x3 forward.  A workgroup computes a
// contiguous range of the TH x 32-pixel output tiles (each XCD one band of
// them) for all BN output channels; a tile is CP/32 steps, one per
// 32-input-channel slice.  A step stages the slice's input halo ((TH+2) x 34
// pixels, zero outside the image; with UP the (TH/2+2) x 18 source pixels the
// up-sampled halo reads) and, unless all slices' weights stay resident, the
// slice's weights of all nine taps in LDS, then runs the nine taps' MFMAs
// with no barrier between them.  The next step's halo and weights are loaded
// into registers while this step's MFMAs run, so a workgroup hides its own
// load latency.
//
// The MFMA is v_mfma_f32_32x32x16_bf16 (measured on the device: about 2.0
// PFLOP/s, against about 1.15 for v_mfma_f32_16x16x32_bf16 with the same
// number of independent accumulators).  It takes the weights as its row
// operand (32 output channels) and a 32-pixel tile row as its column
// operand; lane l holds pixel l % 32 and, in accumulator element r, channel
// 8 (r / 4) + 4 (l / 32) + r % 4.  A workgroup is CS * TH/2 waves; each
// owns two tile rows and BN / CS output channels (CS = 2 for 128 channels,
// else 1), so a taller tile spreads a staged weight slice over more waves at
// the same registers per wave.  The accumulators start from the bias;
// the epilogue (ReLU, v_cvt_pk_bf16_f32, optionally the 2x2 average pool, or
// instead of the stores the network's output conv written into a
// compositor frame) goes through a staging tile in LDS so that the stores
// are coalesced.
//
// LDS rows hold 32 bf16 channels (4 16-byte chunks).  gfx950 serves a
// ds_read_b128 16 lanes per cycle (per half-wave, the lanes whose bits 2-4
// have even parity, then odd), and a fragment read is 32 consecutive rows
// at one chunk per half-wave.  Halo pixels are 5 chunks apart (an odd pitch
// puts each 16-lane set on distinct banks wherever the 32 pixels start);
// weight rows are 4 chunks apart with the chunk index XOR-ed with
// (row >> 2) & 3, which does the same for 32 rows starting at a multiple of
// 32 (measured on the device: conflicting patterns take 2x the cycles).
// Every address of the tap loop is a per-lane register plus an immediate,
// so the loop issues no vector ALU work.
constexpr int kTW = 32;  // tile width (pixels)
constexpr int kXcds = 8;  // XCDs (each with its own L2) the workgroups of a launch are dealt to in turn
constexpr int kKC = 32;  // input channels per step
// Output-tile heights (rows of 32 pixels, 8 or 16) of the layers with
// (output, input) channels (32, 32), (32, 64), (64, 32), (64, 64), (64, 128)
// and (128, *).  16 rows (8 waves) for the 64-channel layers: a staged
// weight slice serves twice the pixels (2048^2 enc2b / dec2b 107 / 98 -> 94 /
// 87 us, dec2a 181 -> 169 us); and for the 32 -> 32 layers (4 waves per
// SIMD instead of 3: enc1b 131 -> 126 us).  The 32 -> 64 and 64 -> 32
// layers were slower with 16 rows (dec1a 186 -> 199, enc2a 53 -> 56 us) and
// the 128-channel ones would spill.
#ifndef DFB_TH_32_32
#define DFB_TH_32_32 16
#endif
#ifndef DFB_TH_32_64
#define DFB_TH_32_64 8
#endif
#ifndef DFB_TH_64_32
#define DFB_TH_64_32 8
#endif
#ifndef DFB_TH_64_64
#define DFB_TH_64_64 16
#endif
#ifndef DFB_TH_64_128
#define DFB_TH_64_128 16
#endif
#ifndef DFB_TH_128
#define DFB_TH_128 8
#endif
// the same for the up-sampled layers (32, 64) and (64, 128)
#ifndef DFB_THU_32_64
#define DFB_THU_32_64 8
#endif
#ifndef DFB_THU_64_128
#define DFB_THU_64_128 16
#endif

// Waves that share a tile's 128 output channels (each takes 128 / DFB_CS_128
// of them): 2 halves the accumulators per wave, so the 128-channel layers
// run 2 waves per SIMD instead of 1 at the same LDS.
#ifndef DFB_CS_128
#define DFB_CS_128 2
#endif
// LDS bytes up to which a layer keeps every input slice's weights resident
// (the 16-row 64 -> 64 layers need 123 KB: one 8-wave workgroup per CU)
#ifndef DFB_RESW_KB
#define DFB_RESW_KB 124
#endif
template <int BN, int TH, int NCH, bool UP>
struct ConvCfg {
  // With UP the halo is staged at the source resolution: (TH/2 + 2) x 18
  // pixels, each read by the up to four output-halo pixels it is
  // up-sampled to (the fragment reads index it through the same
  // nearest-neighbour map).
  static constexpr int SHH = UP ? TH / 2 + 2 : TH + 2, SHW = UP ? kTW / 2 + 2 : kTW + 2;  // staged rows, columns
  static constexpr int HPITCH = 5;             // 16-byte chunks per halo pixel (4 used)
  static constexpr int HALO_CH = SHH * SHW * HPITCH;  // 16-byte chunks of a step's halo
  static constexpr int HALO_EL = SHH * SHW * 4;       // chunks loaded per step
  static constexpr int W_CH = 9 * BN * 4;      // 16-byte chunks of a step's weights
  static constexpr int CS = BN >= 128 ? DFB_CS_128 : 1;  // waves sharing a tile row pair's channels
  static constexpr int NT = 32 * TH * CS;      // threads: CS waves per two tile rows
  static constexpr int HIT = (HALO_EL + NT - 1) / NT, WIT = (W_CH + NT - 1) / NT;
  // The epilogue's staging tile (TH x 32 pixels of BN bf16 + 8 padding)
  // overlays the halo region, and the weights when a step re-stages them;
  // it is written in two passes of TH/2 rows when it does not fit.  The
  // small halo of an up-sampled layer is given room for at least one pass
  // (counting the weights' region when even the halo alone leaves no room
  // for all weight slices).
  static constexpr int STG1 = TH * kTW * (BN + 8) * 2;  // bytes of the whole staging tile
  static constexpr int WEXTRA = NCH > 1 && (HALO_CH + NCH * W_CH) * 16 + BN * 4 > DFB_RESW_KB * 1024 ? W_CH : 0;
  static constexpr int REGION_CH = UP && (HALO_CH + WEXTRA) * 16 < STG1 / 2 ? STG1 / 32 - WEXTRA : HALO_CH;
  // weight slices held in LDS: all of them when the layer's LDS stays
  // within DFB_RESW_KB (no weight traffic per step), else the step's slice,
  // re-staged every step
  static constexpr int WS = (REGION_CH + NCH * W_CH) * 16 + BN * 4 <= DFB_RESW_KB * 1024 ? NCH : 1;
  static constexpr int STG_ROOM = (WS == 1 && NCH > 1 ? REGION_CH + W_CH : REGION_CH) * 16;
  static constexpr int NPASS = STG1 <= STG_ROOM ? 1 : 2;
  static constexpr size_t BYTES = static_cast<size_t>(REGION_CH + WS * W_CH) * 16 + BN * 4;  // + the bias
  // waves per SIMD the register allocation is held to: those of the
  // workgroups that fit a compute unit's 160 KB of LDS, at most 4
  static constexpr int LDS_WG = static_cast<int>((160 * 1024) / BYTES);
  // ... and at most 2 where a step re-stages 64 or more channels' weights:
  // their prefetch registers and accumulators need more than 168 VGPRs
  static constexpr int REG_WAVES = WS == 1 && NCH > 1 && BN >= 64 ? 2 : 4;
  static constexpr int WAVES_LDS = LDS_WG * NT / 256 < 1 ? 1 : (LDS_WG * NT / 256 > 4 ? 4 : LDS_WG * NT / 256);
  static constexpr int WAVES = WAVES_LDS < REG_WAVES ? WAVES_LDS : REG_WAVES;
};
// Raw buffer accesses with a 2 GB range from a per-step base: an offset of
// kOOB is out of range, so the load returns zeros or the store is dropped.
// Every lane issues every access, so the number of outstanding memory
// operations is known at compile time and waiting for the prefetched loads
// never waits for the stores issued after them.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x3 __attribute__((ext_vector_type(3)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int kOOB = static_cast<int>(0x80000000u);
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7FFFFFFF, 0x00020000);
}
__device__ __forceinline__ uint4 buf_load16(__amdgpu_buffer_rsrc_t r, int byte_off) {
  const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
  return uint4{v[0], v[1], v[2], v[3]};
}
// Cache policy of a store: kNT marks it non-temporal (streamed past the
// caches).  The first layer and the 32 -> 64 and 64 -> 128 layers store
// their activations that way (2048^2: enc1a 64 -> 55, dec1a 184 -> 176,
// dec2a 170 -> 165 us); the 32 -> 32 layers were slower with it (enc1b 125
// -> 130, dec1b 105 -> 113 us) and the others unchanged.
constexpr int kNT = 2;
template <int POLICY = 0>
__device__ __forceinline__ void buf_store16(__amdgpu_buffer_rsrc_t r, int byte_off, uint4 v) {
  const u32x4 w = {v.x, v.y, v.z, v.w};
  __builtin_amdgcn_raw_buffer_store_b128(w, r, byte_off, 0, POLICY);
}
__device__ __forceinline__ void buf_store8(__amdgpu_buffer_rsrc_t r, int byte_off, uint32_t lo, uint32_t hi) {
  const u32x2 v = {lo, hi};
  __builtin_amdgcn_raw_buffer_store_b64(v, r, byte_off, 0, 0);
}
// LDS chunk of (row p, chunk q) of the swizzled weights
__device__ __forceinline__ int swz(int p, int q) { return p * 4 + (q ^ ((p >> 2) & 3)); }

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
// two floats to bf16 (round to nearest even), packed low | high << 16
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
  const f32x2 v = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
}
__device__ __forceinline__ float bf16_lo(uint32_t u) { return __uint_as_float(u << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t u) { return __uint_as_float(u & 0xFFFF0000u); }


// Epilogue kinds: plain, plus the 2x2 average pool, or instead of storing
// y the network's 1x1 output conv and residual written straight into a
// compositor frame (inference, 32 channels).
enum Epi { kEpiPlain = 0, kEpiPool = 1, kEpiFrame = 2 };
struct OutConv {     // out[p][c] = mean[p][c] + b[c] + sum_i y[p][i] w[i][c], c < 3
  const float* w;    // [32][3]
  const float* b;    // [3]
  // the frame's running mean (tile-major) and tile variances: pixel e of the
  // frame becomes den[e] = (out[p], mean alpha), or the mean itself where
  // the tile falls back (n >= 2 and its variance above tau)
  FrameGlue glue;
  float tau;
  float* den;        // [T][P][4]
};

template <int BN, int CP, int TH, bool UP, int EPI>
__global__ void __launch_bounds__((ConvCfg<BN, TH, CP / kKC, UP>::NT))
__attribute__((amdgpu_waves_per_eu(ConvCfg<BN, TH, CP / kKC, UP>::WAVES)))
conv_fwd_k(Map x, Map x2, const uint16_t* __restrict__ w, const float* __restrict__ bias, Map y, Map pool, OutConv oc,
           Shape s) {
  using C = ConvCfg<BN, TH, CP / kKC, UP>;
  constexpr bool POOL = EPI == kEpiPool, OUT = EPI == kEpiFrame;
  constexpr int STORE_POLICY = (BN == 32 && CP == 64) || (BN == 64 && CP == 128) ? kNT : 0;
  static_assert(!OUT || BN == 32, "the output conv takes 32 channels, one pixel per thread");
  constexpr int NT = C::NT;  // threads (CS waves per two tile rows)
  constexpr int NCH = CP / kKC, MB = 2, NB = BN / 32 / C::CS;  // tile rows and 32-channel blocks per wave
  static_assert(NB >= 1 && NB * 32 * C::CS == BN, "channel split");
  constexpr int SHH = C::SHH, SHW = C::SHW, HALO_EL = C::HALO_EL, HIT = C::HIT, WIT = C::WIT;
  static_assert(!POOL || MB % 2 == 0, "the pool pairs rows inside a wave");
  extern __shared__ __align__(16) uint4 lds4[];
  uint4* halo = lds4;                // [SHH * SHW][5], and the epilogue's staging tile
  uint4* wts = lds4 + C::REGION_CH;  // [WS][9 * BN][4]
  float* lbias = reinterpret_cast<float*>(wts + C::WS * C::W_CH);  // [BN]: read per tile through LDS, so
  // starting a tile waits on no global load issued after the prefetch
  float* lout = lbias + BN;  // [32 * 3 + 3] output-conv weights and bias (kEpiFrame)
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l32 = lane & 31, lh = lane >> 5;
  // wave = (channel group) * TH/2 + (row pair): rows 2 rw, 2 rw + 1 and the
  // channel blocks cb0 / 32 .. + NB - 1
  const int rw = C::CS > 1 ? wave % (TH / 2) : wave, cb0 = C::CS > 1 ? (wave / (TH / 2)) * NB * 32 : 0;
  const int tiles_x = (s.w + kTW - 1) / kTW, tiles_y = (s.h + TH - 1) / TH;
  const long long tiles = static_cast<long long>(s.n) * tiles_x * tiles_y;
  // workgroup b walks the tiles [b T / G, (b + 1) T / G) in row order (the
  // host launches G <= T workgroups, so each has at least one), sharing the
  // halo columns of consecutive tiles through its L2.  b is the workgroup's
  // rank on its XCD (the hardware deals workgroups to the 8 XCDs in turn)
  // after those of the XCDs before it, so each XCD walks one contiguous
  // band of tiles and the workgroups working on vertically adjacent tiles
  // at the same time share their halo rows through the same L2.
  const long long G = gridDim.x;
  const int xcd = static_cast<int>(blockIdx.x % kXcds), xr = static_cast<int>(blockIdx.x / kXcds);
  const long long b0 = xcd * (G / kXcds) + (xcd < G % kXcds ? xcd : G % kXcds) + xr;
  const long long t_begin = b0 * tiles / G, t_end = (b0 + 1) * tiles / G;
  const int nsteps = static_cast<int>(t_end - t_begin) * NCH;
  const int hi = UP ? s.h / 2 : s.h, wi = UP ? s.w / 2 : s.w;  // the map x is read from
  // The input is the channel concatenation of x and x2 (x2.c may be 0; else
  // x.c is a multiple of 32 and x2.ld == x.ld): slices below x.c read x, the
  // others x2.
  const int cin = x.c + x2.c;
  const bool full = cin == CP;  // else channels cin .. CP-1 are staged as zeros
  struct Tile {
    int n, ty, tx;
  };
  auto decode = [&](long long t) {
    Tile u;
    const long long per_img = static_cast<long long>(tiles_x) * tiles_y;
    u.n = static_cast<int>(t / per_img);
    const int r = static_cast<int>(t - u.n * per_img);
    u.ty = r / tiles_x;
    u.tx = r - u.ty * tiles_x;
    return u;
  };
  auto advance = [&](Tile& u) {
    if (++u.tx == tiles_x) {
      u.tx = 0;
      if (++u.ty == tiles_y) {
        u.ty = 0;
        ++u.n;
      }
    }
  };

  // this thread's halo elements e = tid + NT k: halo pixel e / 4 (row, column),
  // chunk e % 4; byte offset from the step's source origin (the halo's
  // top-left pixel, or the pixel it is up-sampled from); LDS chunk
  // hlds + 64 * HPITCH * k
  int hrel[HIT];
#pragma unroll
  for (int k = 0; k < HIT; ++k) {
    const int e = tid + NT * k, hp = e >> 2, cc = e & 3, hr = hp / SHW, hc = hp - hr * SHW;
    hrel[k] = e < HALO_EL ? ((hr * wi + hc) * x.ld + cc * 8) * 2 : kOOB;
  }
  const int hlds = (tid >> 2) * C::HPITCH + (tid & 3);
  // fragment reads of 16-channel half kh: weights of (tap, j) at
  // wts[(tap * BN + j * 32) * 4 + boff[kh]], halo of (m, tap) at
  // halo[aoff[dc] + hrow(m + dr) * SHW * HPITCH + 2 kh], where output-halo
  // row r of the wave is staged row r (or (r + 1) / 2 with UP) and
  // aoff[dc] holds the lane's column: l32 + dc (or (l32 + dc + 1) / 2)
  const int boff[2] = {l32 * 4 + ((0 + lh) ^ ((l32 >> 2) & 3)), l32 * 4 + ((2 + lh) ^ ((l32 >> 2) & 3))};
  const int wrow0 = UP ? rw * MB / 2 : rw * MB;  // the wave's first staged row (MB is even with UP)
  int aoff[UP ? 3 : 1];
#pragma unroll
  for (int dc = 0; dc < (UP ? 3 : 1); ++dc)
    aoff[dc] = (wrow0 * SHW + (UP ? (l32 + dc + 1) >> 1 : l32)) * C::HPITCH + lh;

  // Halo of slice ck of tile u into hreg; every load is issued (with
  // `none`, all out of range).
  auto load_halo = [&](const Tile& u, int ck, bool none, uint4* hreg) {
    const int oy0 = u.ty * TH, ox0 = u.tx * kTW;
    const bool second = ck * kKC >= x.c;
    const Map& xm = second ? x2 : x;
    const int cb = second ? ck * kKC - x.c : ck * kKC;  // first channel of the slice in xm
    const uint16_t* img = xm.p + xm.off + cb + static_cast<long long>(u.n) * hi * wi * xm.ld;
    // the staged halo's top-left pixel in the map read (hi x wi)
    const int sy0 = UP ? oy0 / 2 - 1 : oy0 - 1, sx0 = UP ? ox0 / 2 - 1 : ox0 - 1;
    const bool inner = full && sy0 >= 0 && sy0 + SHH <= hi && sx0 >= 0 && sx0 + SHW <= wi;
    const __amdgpu_buffer_rsrc_t src = buf_rsrc(img + (static_cast<long long>(sy0) * wi + sx0) * x.ld);
    int off[HIT];
    if (inner && !none) {
#pragma unroll
      for (int k = 0; k < HIT; ++k) off[k] = hrel[k];
    } else {  // zeros outside the image and past xm.c
#pragma unroll
      for (int k = 0; k < HIT; ++k) {
        const int e = tid + NT * k, hp = e >> 2, cc = e & 3, hr = hp / SHW, hc = hp - hr * SHW;
        const int r = sy0 + hr, c = sx0 + hc;
        const int ok = (static_cast<unsigned>(r) < static_cast<unsigned>(hi)) &
                       (static_cast<unsigned>(c) < static_cast<unsigned>(wi)) & (cb + cc * 8 < xm.c) & !none;
        off[k] = ok ? hrel[k] : kOOB;
      }
    }
#pragma unroll
    for (int k = 0; k < HIT; ++k) hreg[k] = buf_load16(src, off[k]);
  };
  // weights [tap][co][cin]: a step's slice is 64 bytes of each (tap, co) row
  const __amdgpu_buffer_rsrc_t wsrc = buf_rsrc(w);
  int wrel[WIT];  // byte offset of this thread's chunks in slice 0
#pragma unroll
  for (int k = 0; k < WIT; ++k) {
    const int e = tid + NT * k;
    wrel[k] = e < C::W_CH ? ((e >> 2) * cin + (e & 3) * 8) * 2 : kOOB;
  }
  auto load_w = [&](int ck, bool none, uint4* wreg) {
    int off[WIT];
    if (full && !none) {
#pragma unroll
      for (int k = 0; k < WIT; ++k) off[k] = wrel[k] + ck * kKC * 2;  // kOOB stays out of range
    } else {
#pragma unroll
      for (int k = 0; k < WIT; ++k) {
        const int cc = (tid + NT * k) & 3;
        off[k] = !none && ck * kKC + cc * 8 < cin ? wrel[k] + ck * kKC * 2 : kOOB;
      }
    }
#pragma unroll
    for (int k = 0; k < WIT; ++k) wreg[k] = buf_load16(wsrc, off[k]);
  };
  auto store_w = [&](const uint4* wreg, int slot) {
#pragma unroll
    for (int k = 0; k < WIT; ++k) {
      const int e = tid + NT * k;
      if (e < C::W_CH) wts[slot * C::W_CH + swz(e >> 2, e & 3)] = wreg[k];
    }
  };
  f32x16 acc[MB][NB];
  // Epilogue of tile u: ReLU and bf16 into a staging tile in LDS (over the
  // halo, and over the weights when a step re-stages them), then 16-byte
  // stores with consecutive lanes on consecutive addresses, and the 2x2
  // pool from the staging tile.  Output channels j*32 + 8q + 4*lh .. +3 of
  // pixel l32 are accumulator elements 4q .. 4q+3.  When the staging tile
  // does not fit it is written and stored in two passes of TH/2 rows.  With
  // `dummy` only the global stores are issued, all out of range: the
  // prologue issues the same stores as a loop iteration, so the loop entry
  // and its back edge leave the same memory operations behind the prefetch
  // and the wait for it is exact on both.
  constexpr int LDO = BN + 8;  // staging row (one pixel) in bf16
  constexpr int OCH = BN / 8;  // 16-byte chunks per output pixel
  constexpr int NPASS = C::NPASS;
  constexpr int RP = TH / NPASS;  // tile rows per pass
  static_assert(RP * kTW * LDO * 2 <= C::STG_ROOM, "staging tile too large");
  static_assert((RP * kTW * OCH) % NT == 0 && RP % 2 == 0 && RP % MB == 0, "pass shape");
  static_assert(!OUT || NPASS == 1, "the output conv reads every staged row of the tile");
  constexpr int NOUT = OUT ? 0 : RP * kTW * OCH / NT;                             // stores per thread and pass
  constexpr int NPOOL = POOL ? ((RP / 2) * (kTW / 2) * OCH + NT - 1) / NT : 0;  // pool stores per thread and pass
  uint16_t* stg = reinterpret_cast<uint16_t*>(lds4);
  // kEpiFrame: the mean RGBA and tile variance of this thread's pixel of the
  // tile being computed, and its frame index
  float bcur[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  int ecur = 0;
  const int n_acc = OUT ? oc.glue.state->n_acc : 0;
  auto epilogue = [&](const Tile& u, bool dummy) {
    const int n = u.n, oy0 = u.ty * TH, ox0 = u.tx * kTW;
    const bool out_full = oy0 + TH <= s.h && ox0 + kTW <= s.w;
    const __amdgpu_buffer_rsrc_t yb = buf_rsrc(y.p + y.off + ((static_cast<long long>(n) * s.h + oy0) * s.w + ox0) * y.ld);
    const int ph = s.h / 2, pw = s.w / 2;
    const __amdgpu_buffer_rsrc_t pb =
        buf_rsrc(POOL ? pool.p + pool.off + ((static_cast<long long>(n) * ph + oy0 / 2) * pw + ox0 / 2) * pool.ld : y.p);
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
      if (!dummy) {
        __syncthreads();  // every wave is done with the halo / weights (or the previous pass)
        if (rw * MB / RP == pass) {
#pragma unroll
          for (int m = 0; m < MB; ++m)
#pragma unroll
            for (int j = 0; j < NB; ++j)
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const f32x16& v = acc[m][j];
                const int lrow = rw * MB + m - pass * RP;
                *reinterpret_cast<uint2*>(stg + (lrow * kTW + l32) * LDO + cb0 + j * 32 + 8 * q + 4 * lh) =
                    uint2{pack_bf16(fmaxf(v[4 * q], 0.f), fmaxf(v[4 * q + 1], 0.f)),
                          pack_bf16(fmaxf(v[4 * q + 2], 0.f), fmaxf(v[4 * q + 3], 0.f))};
              }
        }
        __syncthreads();
      }
#pragma unroll
      for (int k = 0; k < NOUT; ++k) {
        const int e = tid + NT * k, px = e / OCH, c = e % OCH, lrow = px / kTW, col = px % kTW;
        const int row = pass * RP + lrow;
        const int ok = !dummy & (out_full | ((oy0 + row < s.h) & (ox0 + col < s.w)));
        const uint4 v = dummy ? uint4{0u, 0u, 0u, 0u} : *reinterpret_cast<const uint4*>(stg + (lrow * kTW + col) * LDO + c * 8);
        // (distinct out-of-range offsets: identical ones would let the compiler drop all but the last)
        buf_store16<STORE_POLICY>(yb, ok ? ((row * s.w + col) * y.ld + c * 8) * 2 : kOOB + (pass * NOUT + k) * 16, v);
      }
#pragma unroll
      for (int k = 0; k < NPOOL; ++k) {
        // pooled pixel (qr, qc) of this pass: ((a + b) + c) + d of the staged
        // bf16 values, a b over c d
        const int e = tid + NT * k, qi = e / OCH, c = e % OCH, qr = qi / (kTW / 2), qc = qi % (kTW / 2);
        const int prow = pass * RP / 2 + qr;
        const int ok = !dummy & (e < (RP / 2) * (kTW / 2) * OCH) &
                       (out_full | ((oy0 / 2 + prow < ph) & (ox0 / 2 + qc < pw)));
        uint4 o = {0u, 0u, 0u, 0u};
        if (!dummy && e < (RP / 2) * (kTW / 2) * OCH) {
          const uint16_t* t00 = stg + ((2 * qr) * kTW + 2 * qc) * LDO + c * 8;
          const uint4 a4 = *reinterpret_cast<const uint4*>(t00);
          const uint4 b4 = *reinterpret_cast<const uint4*>(t00 + LDO);
          const uint4 c4 = *reinterpret_cast<const uint4*>(t00 + kTW * LDO);
          const uint4 d4 = *reinterpret_cast<const uint4*>(t00 + (kTW + 1) * LDO);
          const uint32_t A[4] = {a4.x, a4.y, a4.z, a4.w}, B[4] = {b4.x, b4.y, b4.z, b4.w},
                         Cc[4] = {c4.x, c4.y, c4.z, c4.w}, D[4] = {d4.x, d4.y, d4.z, d4.w};
          uint32_t r4[4];
#pragma unroll
          for (int h = 0; h < 4; ++h) {
            const float lo = ((bf16_lo(A[h]) + bf16_lo(B[h])) + bf16_lo(Cc[h])) + bf16_lo(D[h]);
            const float hi2 = ((bf16_hi(A[h]) + bf16_hi(B[h])) + bf16_hi(Cc[h])) + bf16_hi(D[h]);
            r4[h] = pack_bf16(0.25f * lo, 0.25f * hi2);
          }
          o = uint4{r4[0], r4[1], r4[2], r4[3]};
        }
        buf_store16(pb, ok ? ((prow * pw + qc) * pool.ld + c * 8) * 2 : kOOB + (NPASS * NOUT + pass * NPOOL + k) * 16, o);
      }
      if (OUT) {
        // pixel tid of the tile: the 1x1 conv over its 32 staged bf16
        // channels, in channel order, then (mean + b) + sum
        const int lrow = tid / kTW, col = tid % kTW, row = pass * RP + lrow;
        const int ok = !dummy & (out_full | ((oy0 + row < s.h) & (ox0 + col < s.w)));
        float o3[3] = {0.f, 0.f, 0.f};
        if (!dummy) {
          float a3[3] = {0.f, 0.f, 0.f};
#pragma unroll
          for (int c8 = 0; c8 < 4; ++c8) {
            const uint4 v = *reinterpret_cast<const uint4*>(stg + (lrow * kTW + col) * LDO + c8 * 8);
            const uint32_t wv[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int i = c8 * 8 + k;
              const float xi = (k & 1) ? bf16_hi(wv[k >> 1]) : bf16_lo(wv[k >> 1]);
#pragma unroll
              for (int c = 0; c < 3; ++c) a3[c] = fmaf(xi, lout[i * 3 + c], a3[c]);
            }
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) o3[c] = (bcur[c] + lout[96 + c]) + a3[c];
        }
        const bool fb = n_acc >= 2 && bcur[4] > oc.tau;
        const u32x4 dv = {__float_as_uint(fb ? bcur[0] : o3[0]), __float_as_uint(fb ? bcur[1] : o3[1]),
                          __float_as_uint(fb ? bcur[2] : o3[2]), __float_as_uint(bcur[3])};
        __builtin_amdgcn_raw_buffer_store_b128(dv, buf_rsrc(oc.den), ok ? ecur * 16 : kOOB + pass * 16, 0, 0);
      }
    }
  };

  uint4 hreg[HIT], wreg[WIT];
  float breg[5] = {0.f, 0.f, 0.f, 0.f, 0.f};  // bcur and ecur of the tile being prefetched
  int ereg = 0;
  auto load_base = [&](const Tile& u, bool none) {
    if (!OUT) return;
    const int oy0 = u.ty * TH, ox0 = u.tx * kTW, row = tid / kTW, col = tid % kTW;
    const FrameGlue& g = oc.glue;
    const int r = oy0 + row, c = ox0 + col, ty = r / g.tile_h, tx = c / g.tile_w, t = ty * g.tiles_x + tx;
    const int ok = !none & (r < s.h) & (c < s.w);
    ereg = t * g.P + (r - ty * g.tile_h) * g.tile_w + (c - tx * g.tile_w);
    const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(buf_rsrc(g.accum), ok ? ereg * 16 : kOOB, 0, 0);
    const uint32_t var = __builtin_amdgcn_raw_buffer_load_b32(buf_rsrc(g.tile_var), ok ? t * 4 : kOOB, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) breg[i] = __uint_as_float(v[i]);
    breg[4] = __uint_as_float(var);
  };
  if (tid < BN) lbias[tid] = bias[tid];
  if (OUT && tid < 99) lout[tid] = tid < 96 ? oc.w[tid] : oc.b[tid - 96];
  Tile cur = decode(t_begin), nxt = cur;  // the tile computed, the tile prefetched
  constexpr bool RESW = C::WS == NCH;  // every slice's weights stay in LDS for every tile
  if (RESW) {
#pragma unroll
    for (int ck = 0; ck < NCH; ++ck) {
      load_w(ck, false, wreg);
      store_w(wreg, ck);
    }
  }
  load_halo(nxt, 0, false, hreg);
  if (!RESW) load_w(0, false, wreg);
  load_base(nxt, false);
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int j = 0; j < NB; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[m][j][r] = 0.f;
  epilogue(cur, true);
  const int my_tiles = nsteps / NCH;
  for (int it = 0; it < my_tiles; ++it) {
#pragma unroll
    for (int ck = 0; ck < NCH; ++ck) {
      __syncthreads();  // the previous step's fragment reads are done
#pragma unroll
      for (int k = 0; k < HIT; ++k)
        if (tid + NT * k < HALO_EL) halo[hlds + (NT / 4) * C::HPITCH * k] = hreg[k];
      if (!RESW) store_w(wreg, 0);
      if (OUT && ck == 0) {
#pragma unroll
        for (int i = 0; i < 5; ++i) bcur[i] = breg[i];
        ecur = ereg;
      }
      __syncthreads();
      // prefetch the next step: the next slice, or slice 0 of the next tile
      const bool none = ck == NCH - 1 && it + 1 == my_tiles;
      if (ck == NCH - 1 && !none) advance(nxt);
      load_halo(nxt, (ck + 1) % NCH, none, hreg);
      if (!RESW) load_w((ck + 1) % NCH, none, wreg);
      if (ck == NCH - 1) load_base(nxt, none);
      // keep the prefetch ahead of the taps: the scheduler would otherwise
      // sink the loads below the MFMAs and expose their latency
      __builtin_amdgcn_sched_barrier(0);
      if (ck == 0) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const f32x4 b4 = *reinterpret_cast<const f32x4*>(lbias + cb0 + j * 32 + 8 * q + 4 * lh);
#pragma unroll
            for (int m = 0; m < MB; ++m)
#pragma unroll
              for (int r = 0; r < 4; ++r) acc[m][j][4 * q + r] = b4[r];
          }
      }
      // 18 (tap, 16-channel half) steps; the fragments of step i + 1 are
      // read while step i's MFMAs run
      bf16x8 wf[2][NB], hf[2][MB];
      auto frag = [&](int i, int bsel) {
        const int tap = i >> 1, kh = i & 1, dr = tap / 3, dc = tap - (tap / 3) * 3;
#pragma unroll
        for (int j = 0; j < NB; ++j)
          wf[bsel][j] = __builtin_bit_cast(bf16x8, wts[(RESW ? ck : 0) * C::W_CH + (tap * BN + cb0 + j * 32) * 4 + boff[kh]]);
#pragma unroll
        for (int m = 0; m < MB; ++m)
          hf[bsel][m] = __builtin_bit_cast(
              bf16x8, halo[aoff[UP ? dc : 0] + ((UP ? (m + dr + 1) >> 1 : m + dr) * SHW + (UP ? 0 : dc)) * C::HPITCH + 2 * kh]);
      };
      frag(0, 0);
#pragma unroll
      for (int i = 0; i < 18; ++i) {
        if (i + 1 < 18) frag(i + 1, (i + 1) & 1);
        __builtin_amdgcn_sched_barrier(0);  // the reads stay ahead of this step's MFMAs
#pragma unroll
        for (int m = 0; m < MB; ++m)
#pragma unroll
          for (int j = 0; j < NB; ++j)
            acc[m][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wf[i & 1][j], hf[i & 1][m], acc[m][j], 0, 0, 0);
      }
    }
    epilogue(cur, false);
    cur = nxt;
  }
}

// ------------------------------------------------------------- first layer
// The first conv (8 input channels, the last two zero) as a 72-deep
// contraction: two taps' 8 channels per 16-wide K slice, so a 32 x 32
// output block takes 5 v_mfma_f32_32x32x16_bf16 (the tenth tap slot has
// zero weights) where the general kernel takes 18 with K padded to 32.  One
// 8 x 32-pixel tile per workgroup; a halo pixel is one 16-byte LDS chunk
// (an odd pitch: fragment reads are free of bank conflicts), a weight row
// 11 chunks (10 tap slots and one of padding).
constexpr int kInTH = 8, kInHW = kTW + 2, kInHH = kInTH + 2, kInHalo = kInHH * kInHW, kInWP = 11;
// FRAME false reads the packed bf16 input x; true builds the input from a
// compositor frame's running mean and tile variance as it loads the halo
// (the values the frame glue writes: mean RGBA, log variance or 0 before two
// frames, 1/n, rounded to bf16 as the input packing does).
template <bool FRAME>
__global__ void __launch_bounds__(256) conv_in_k(Map x, FrameGlue fg,
                                                 const uint16_t* __restrict__ w, const float* __restrict__ bias, Map y,
                                                 Shape s) {
  constexpr int LDO = 40;  // staging row (one pixel) in bf16
  __shared__ __align__(16) uint4 halo[kInHalo];
  __shared__ __align__(16) uint4 wl[32 * kInWP];
  __shared__ __align__(16) uint16_t stg[kInTH * kTW * LDO];
  __shared__ __align__(16) float lb[32];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l32 = lane & 31, lh = lane >> 5;
  const int tiles_x = (s.w + kTW - 1) / kTW, tiles_y = (s.h + kInTH - 1) / kInTH;
  const int t = static_cast<int>(blockIdx.x), n = t / (tiles_x * tiles_y), rr = t - n * tiles_x * tiles_y;
  const int oy0 = (rr / tiles_x) * kInTH, ox0 = (rr % tiles_x) * kTW;
  // halo pixels tid and tid + 256 (of kInHalo), image row oy0 - 1 + hr, column ox0 - 1 + hc
  uint4 hv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + 256 * k, hr = e / kInHW, hc = e - hr * kInHW, r = oy0 - 1 + hr, c = ox0 - 1 + hc;
    const int ok = (e < kInHalo) & (static_cast<unsigned>(r) < static_cast<unsigned>(s.h)) &
                   (static_cast<unsigned>(c) < static_cast<unsigned>(s.w));
    const int pix = r * s.w + c;  // within image n
    if (FRAME) {  // one image
      float4 mu = make_float4(0.f, 0.f, 0.f, 0.f);
      float lv = 0.f, inv_n = 0.f;
      if (ok) {
        const int ty = r / fg.tile_h, tx = c / fg.tile_w, t = ty * fg.tiles_x + tx;
        mu = reinterpret_cast<const float4*>(fg.accum)[static_cast<size_t>(t) * fg.P + (r - ty * fg.tile_h) * fg.tile_w +
                                                      (c - tx * fg.tile_w)];
        const float v = fg.tile_var[t];
        const int n_acc = fg.state->n_acc;
        lv = n_acc >= 2 ? logf(v > 1e-12f ? v : 1e-12f) : 0.f;
        inv_n = 1.f / static_cast<float>(n_acc);
      }
      hv[k] = uint4{pack_bf16(mu.x, mu.y), pack_bf16(mu.z, mu.w), pack_bf16(lv, inv_n), 0u};
    } else {
      const __amdgpu_buffer_rsrc_t src = buf_rsrc(x.p + x.off + static_cast<long long>(n) * s.h * s.w * x.ld);
      hv[k] = buf_load16(src, ok ? pix * x.ld * 2 : kOOB);
    }
  }
  // weights [tap][co][8] -> wl[co][tap] (tap slot 9 zero)
  const __amdgpu_buffer_rsrc_t wsrc = buf_rsrc(w);
  uint4 wv[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + 256 * k, co = e / 10, tap = e - co * 10;
    wv[k] = buf_load16(wsrc, e < 320 && tap < 9 ? (tap * 32 + co) * 16 : kOOB);
  }
  if (tid < 32) lb[tid] = bias[tid];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const int e = tid + 256 * k;
    if (e < kInHalo) halo[e] = hv[k];
    if (e < 320) wl[(e / 10) * kInWP + e % 10] = wv[k];
  }
  __syncthreads();
  // wave w: tile rows 2w, 2w + 1; slice i holds taps 2i (lanes 0-31) and 2i + 1 (lanes 32-63)
  f32x16 acc[2];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f32x4 b4 = *reinterpret_cast<const f32x4*>(lb + 8 * q + 4 * lh);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[m][4 * q + r] = b4[r];
  }
#pragma unroll
  for (int i = 0; i < 5; ++i) {
    const int tap = 2 * i + lh < 9 ? 2 * i + lh : 8, dr = tap / 3, dc = tap - (tap / 3) * 3;
    const bf16x8 a = __builtin_bit_cast(bf16x8, wl[l32 * kInWP + 2 * i + lh]);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const bf16x8 b = __builtin_bit_cast(bf16x8, halo[(2 * wave + m + dr) * kInHW + l32 + dc]);
      acc[m] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[m], 0, 0, 0);
    }
  }
#pragma unroll
  for (int m = 0; m < 2; ++m)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *reinterpret_cast<uint2*>(stg + ((2 * wave + m) * kTW + l32) * LDO + 8 * q + 4 * lh) =
          uint2{pack_bf16(fmaxf(acc[m][4 * q], 0.f), fmaxf(acc[m][4 * q + 1], 0.f)),
                pack_bf16(fmaxf(acc[m][4 * q + 2], 0.f), fmaxf(acc[m][4 * q + 3], 0.f))};
  __syncthreads();
  const __amdgpu_buffer_rsrc_t yb = buf_rsrc(y.p + y.off + ((static_cast<long long>(n) * s.h + oy0) * s.w + ox0) * y.ld);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = tid + 256 * k, px = e / 4, c = e % 4, row = px / kTW, col = px % kTW;
    const int ok = (oy0 + row < s.h) & (ox0 + col < s.w);
    buf_store16<kNT>(yb, ok ? ((row * s.w + col) * y.ld + c * 8) * 2 : kOOB,
                     *reinterpret_cast<const uint4*>(stg + px * LDO + c * 8));
  }
}

// ------------------------------------------------------------- dgrad
// A[p][(tap, co)] = g[p - tap][co], g = bf16(dy * (y > 0)) (gate_k); B =
// W[tap][ci][co].  K runs over (tap, 32-wide c_out slice) in stages of
// kDgradKS slices (one barrier pair per stage; slots past the last slice
// stage zeros); the next stage's A chunks and weights are loaded into
// registers while this stage's MFMAs run.  The MFMA is
// v_mfma_f32_32x32x16_bf16 on 32-pixel x 32-c_in blocks, split over the
// waves as in the weight gradient below (the K steps of a slice are split
// between two waves per block when there are only two blocks).
constexpr int kDgradKS = 4;
constexpr int LDD = 32 * kDgradKS + 8;  // LDS row: the stage's K + 8 padding

template <int BN>
__global__ void __launch_bounds__(256) conv_dgrad_k(Map g, const uint16_t* __restrict__ w, MapF dx, Shape s) {
  __shared__ __align__(16) uint16_t As[BM * LDD];
  __shared__ __align__(16) uint16_t Bs[BN * LDD];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l32 = lane & 31, lh = lane >> 5;
  const long long m0 = static_cast<long long>(blockIdx.x) * BM;
  const int ap = tid >> 2, ach = (tid & 3) * 8;
  const Pix q = pixel_of(m0 + ap, s);
  const int co_n = g.c;
  constexpr int NBLK = 2 * (BN / 32);                      // 32 x 32 output blocks
  constexpr int KSPLIT = NBLK >= 4 ? 1 : 4 / NBLK;         // waves per block
  constexpr int BPW = NBLK >= 4 ? NBLK / 4 : 1;            // blocks per wave
  const int kpart = wave / (4 / KSPLIT);                   // which 16-wide K step of a slice
  f32x16 acc[BPW];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
  const int nk = (co_n + 31) / 32, n_it = 9 * nk;
  constexpr int WPT = (BN * 4 + 255) / 256;  // 16-byte weight chunks per thread and slice
  uint4 av[kDgradKS], wv[kDgradKS][WPT];
  auto load = [&](int it0) {
#pragma unroll
    for (int sl = 0; sl < kDgradKS; ++sl) {
      const int it = it0 + sl;
      const int tap = it / nk, kc = it - (it / nk) * nk;
      av[sl] = uint4{0u, 0u, 0u, 0u};
#pragma unroll
      for (int i = 0; i < WPT; ++i) wv[sl][i] = uint4{0u, 0u, 0u, 0u};
      if (it < n_it) {
        bool in;
        const long long src = shifted(q, 1 - tap / 3, 1 - tap % 3, s, in);
        const int c0 = kc * 32 + ach;
        if (in && c0 < co_n) av[sl] = *reinterpret_cast<const uint4*>(g.p + src * g.ld + g.off + c0);
#pragma unroll
        for (int i = 0; i < WPT; ++i) {
          const int e = tid + i * 256;
          const int ci = e >> 2, k0 = kc * 32 + (e & 3) * 8;
          if (e < BN * 4 && k0 < co_n)
            wv[sl][i] = *reinterpret_cast<const uint4*>(w + (static_cast<size_t>(tap) * BN + ci) * co_n + k0);
        }
      }
    }
  };
  load(0);
  for (int it0 = 0; it0 < n_it; it0 += kDgradKS) {
#pragma unroll
    for (int sl = 0; sl < kDgradKS; ++sl) {
      *reinterpret_cast<uint4*>(As + ap * LDD + sl * 32 + ach) = av[sl];
#pragma unroll
      for (int i = 0; i < WPT; ++i) {
        const int e = tid + i * 256;
        if (e < BN * 4) *reinterpret_cast<uint4*>(Bs + (e >> 2) * LDD + sl * 32 + (e & 3) * 8) = wv[sl][i];
      }
    }
    __syncthreads();
    if (it0 + kDgradKS < n_it) load(it0 + kDgradKS);
#pragma unroll
    for (int sl = 0; sl < kDgradKS; ++sl) {
      if (it0 + sl < n_it) {  // uniform
#pragma unroll
        for (int kk = 0; kk < 2 / KSPLIT; ++kk) {
          const int k = sl * 32 + (KSPLIT > 1 ? kpart : kk) * 16 + lh * 8;
#pragma unroll
          for (int b = 0; b < BPW; ++b) {
            const int blk = KSPLIT > 1 ? wave % NBLK : wave + 4 * b, mb = blk & 1, nb = blk >> 1;
            const bf16x8 a = lds_frag(As + (mb * 32 + l32) * LDD + k);
            const bf16x8 bv = lds_frag(Bs + (nb * 32 + l32) * LDD + k);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  if constexpr (KSPLIT > 1) {  // part 0 + part 1 (the stage loop ended on a barrier: As is free)
    static_assert(KSPLIT == 2 && NBLK * 64 * 16 * 4 <= BM * LDD * 2, "reduction fits As");
    float* red = reinterpret_cast<float*>(As);
    const int blk = wave % NBLK;
    if (kpart == 1) {
#pragma unroll
      for (int r = 0; r < 16; ++r) red[(blk * 16 + r) * 64 + lane] = acc[0][r];
    }
    __syncthreads();
    if (kpart == 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[0][r] += red[(blk * 16 + r) * 64 + lane];
    }
  }
  const long long P = s.pixels();
  if (kpart == 0) {
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      const int blk = KSPLIT > 1 ? wave % NBLK : wave + 4 * b, mb = blk & 1, nb = blk >> 1;
      const int col = nb * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const long long p = m0 + mb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (p < P) dx.p[p * dx.ld + dx.off + col] = acc[b][r];
      }
    }
  }
}

// ------------------------------------------------------------- gate
// g[p][c] = bf16(dy[p][c] * (y[p][c] > 0)), the ReLU-gated output gradient
// that the data and weight gradients read (8 channels per thread); and the
// bias-gradient partial of the workgroup's pixels, partial[block][c] = the
// sum over its pixels, in pixel order, of dy * (y > 0) in f32.
__global__ void __launch_bounds__(256) gate_k(MapF dy, Map y, Map g, float* __restrict__ partial, Shape s) {
  __shared__ float red[256 * 9];  // [thread][8], one pad slot
  const int t = threadIdx.x, cb = dy.c / 8;
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + t;
  float gf[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) gf[i] = 0.f;
  if (e < s.pixels() * cb) {
    const long long p = e / cb;
    const int c0 = static_cast<int>(e - p * cb) * 8;
    const float4 g0 = *reinterpret_cast<const float4*>(dy.p + p * dy.ld + dy.off + c0);
    const float4 g1 = *reinterpret_cast<const float4*>(dy.p + p * dy.ld + dy.off + c0 + 4);
    const uint4 mk = *reinterpret_cast<const uint4*>(y.p + p * y.ld + y.off + c0);
    const float gv[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
    const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
    uint32_t h[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const uint16_t yh = static_cast<uint16_t>(mw[i >> 1] >> ((i & 1) * 16));
      gf[i] = from_bf16(yh) > 0.f ? gv[i] : 0.f;
      h[i] = to_bf16(gf[i]);
    }
    *reinterpret_cast<uint4*>(g.p + p * g.ld + g.off + c0) =
        uint4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) red[t * 9 + i] = gf[i];
  __syncthreads();
  if (t < dy.c) {  // channel t: thread (pixel k, chunk t/8) of the block holds it at slot t%8
    float sum = 0.f;
    for (int k = 0; k < 256 / cb; ++k) sum += red[(k * cb + t / 8) * 9 + (t & 7)];
    partial[static_cast<size_t>(blockIdx.x) * dy.c + t] = sum;
  }
}

// ------------------------------------------------------------- wgrad
// Per tap and 64-wide c_in tile, over one chunk of pixels:
// partial[chunk][tap][ci][co] = sum_p x[p + tap][ci] * g[p][co], g = bf16(dy * (y > 0)).
constexpr int kWgradChunk = 1024;

// A stage is KS slices of 32 pixels (one barrier pair per stage); the
// next stage's x and g are loaded into registers while this stage's MFMAs
// run.  Slices past the image end stage zeros.
constexpr int kWgradKS = 4;
constexpr int LDW = 32 * kWgradKS + 8;  // LDS row: the stage's pixels + 8 padding

// The MFMA is v_mfma_f32_32x32x16_bf16 on 32 c_in x 32 c_out blocks (row
// and column operands read as 32 consecutive LDS rows at one 16-byte chunk;
// the 136-element row pitch is an odd number of chunks, so the reads are free
// of bank conflicts).  Wave w takes blocks w, w + 4, ... of the MBLK * BN / 32
// blocks (MBLK = 1 when the input has at most 32 channels: the c_in tile's
// upper half is zero and is not multiplied); with fewer blocks than waves the
// stage's pixels are split between 4 / blocks waves per block and their sums
// added in a fixed order.
template <int BN, bool HALF>
__global__ void __launch_bounds__(256) conv_wgrad_k(Map x, Map g, float* __restrict__ partial, Shape s) {
  __shared__ __align__(16) uint16_t As[BM * LDW];   // [ci][px]
  __shared__ __align__(16) uint16_t Bs[BN * LDW];   // [co][px]
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, l32 = lane & 31, lh = lane >> 5;
  const int chunk = blockIdx.x, tap = blockIdx.y, ci0 = blockIdx.z * BM;
  const int dr = tap / 3 - 1, dc = tap % 3 - 1;
  const long long P = s.pixels();
  const long long p_begin = static_cast<long long>(chunk) * kWgradChunk;
  constexpr int MBLK = HALF ? 1 : 2;                       // 32-row c_in blocks multiplied
  constexpr int NBLK = MBLK * (BN / 32);                   // 32 x 32 output blocks
  constexpr int KSPLIT = NBLK >= 4 ? 1 : 4 / NBLK;         // waves per block
  constexpr int BPW = NBLK >= 4 ? NBLK / 4 : 1;            // blocks per wave
  constexpr int KSUB = 32 * kWgradKS / 16 / KSPLIT;        // 16-pixel MFMA steps per wave and stage
  const int kpart = wave / (4 / KSPLIT);                   // which part of the stage's pixels
  f32x16 acc[BPW];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[b][r] = 0.f;
  // thread (q, cg) stages the 4 consecutive pixels 4q..4q+3 of the stage
  // (q < 32) for channel group cg: 4 loads of x and of g, then one 8-byte
  // LDS store per channel (4 pixels of one channel, transposed in registers)
  const int q4 = (tid >> 3) * 4;
  const int a8 = (tid & 7) * 8;            // 8 c_in values
  constexpr int BPER = BN / 8;             // c_out values per thread
  const int b0 = (tid & 7) * BPER;
  uint4 v[4];
  uint32_t gw[4][BPER / 2];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const long long p = p_begin + k0 + q4 + i;
      const Pix q = pixel_of(p, s);
      bool in;
      const long long src = shifted(q, dr, dc, s, in);
      v[i] = uint4{0u, 0u, 0u, 0u};
      if (in && ci0 + a8 < x.c) v[i] = *reinterpret_cast<const uint4*>(x.p + src * x.ld + x.off + ci0 + a8);
#pragma unroll
      for (int k = 0; k < BPER / 2; ++k) gw[i][k] = 0u;
      if (q.ok) {  // 8-byte loads (g's row stride and offset are multiples of 4)
        const uint16_t* gp = g.p + p * g.ld + g.off + b0;
#pragma unroll
        for (int k = 0; k < BPER / 4; ++k) {
          const uint2 t = *reinterpret_cast<const uint2*>(gp + 4 * k);
          gw[i][2 * k] = t.x;
          gw[i][2 * k + 1] = t.y;
        }
      }
    }
  };
  // channel c of 4 pixels' packed words w[i] (2 channels per word) as 4 bf16
  auto column = [](const uint32_t (&w)[4], int c) {
    const int sh = (c & 1) * 16;
    const uint32_t e0 = (w[0] >> sh) & 0xFFFFu, e1 = (w[1] >> sh) & 0xFFFFu, e2 = (w[2] >> sh) & 0xFFFFu,
                   e3 = (w[3] >> sh) & 0xFFFFu;
    return uint2{e0 | (e1 << 16), e2 | (e3 << 16)};
  };
  load(0);
  for (int k0 = 0; k0 < kWgradChunk; k0 += 32 * kWgradKS) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int wi = c >> 1;
      const uint32_t w[4] = {wi == 0 ? v[0].x : wi == 1 ? v[0].y : wi == 2 ? v[0].z : v[0].w,
                             wi == 0 ? v[1].x : wi == 1 ? v[1].y : wi == 2 ? v[1].z : v[1].w,
                             wi == 0 ? v[2].x : wi == 1 ? v[2].y : wi == 2 ? v[2].z : v[2].w,
                             wi == 0 ? v[3].x : wi == 1 ? v[3].y : wi == 2 ? v[3].z : v[3].w};
      *reinterpret_cast<uint2*>(As + (a8 + c) * LDW + q4) = column(w, c);
    }
#pragma unroll
    for (int c = 0; c < BPER; ++c) {
      const uint32_t w[4] = {gw[0][c >> 1], gw[1][c >> 1], gw[2][c >> 1], gw[3][c >> 1]};
      *reinterpret_cast<uint2*>(Bs + (b0 + c) * LDW + q4) = column(w, c);
    }
    __syncthreads();
    const int k1 = k0 + 32 * kWgradKS;
    const bool more = k1 < kWgradChunk && p_begin + k1 < P;
    if (more) load(k1);
#pragma unroll
    for (int kk = 0; kk < KSUB; ++kk) {
      const int px = (kpart * KSUB + kk) * 16 + lh * 8;
#pragma unroll
      for (int b = 0; b < BPW; ++b) {
        const int blk = KSPLIT > 1 ? wave % NBLK : wave + 4 * b, mb = blk % MBLK, nb = blk / MBLK;
        const bf16x8 a = lds_frag(As + (mb * 32 + l32) * LDW + px);
        const bf16x8 bv = lds_frag(Bs + (nb * 32 + l32) * LDW + px);
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bv, acc[b], 0, 0, 0);
      }
    }
    __syncthreads();
    if (!more) break;
  }
  if constexpr (KSPLIT > 1) {  // part 0 + part 1 + ... (the stage loop ended on a barrier: As is free)
    static_assert((KSPLIT - 1) * NBLK * 64 * 16 * 4 <= BM * LDW * 2, "reduction fits As");
    float* red = reinterpret_cast<float*>(As);
    const int blk = wave % NBLK;
    if (kpart > 0) {
#pragma unroll
      for (int r = 0; r < 16; ++r) red[(((kpart - 1) * NBLK + blk) * 16 + r) * 64 + lane] = acc[0][r];
    }
    __syncthreads();
    if (kpart == 0) {
#pragma unroll
      for (int k = 1; k < KSPLIT; ++k)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[0][r] += red[(((k - 1) * NBLK + blk) * 16 + r) * 64 + lane];
    }
  }
  const int ci_n = x.c;
  if (kpart == 0) {
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      const int blk = KSPLIT > 1 ? wave % NBLK : wave + 4 * b, mb = blk % MBLK, nb = blk / MBLK;
      const int co = nb * 32 + l32;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int ci = ci0 + mb * 32 + 8 * (r / 4) + 4 * lh + (r % 4);
        if (ci < ci_n) partial[((static_cast<size_t>(chunk) * 9 + tap) * ci_n + ci) * BN + co] = acc[b][r];
      }
    }
  }
}

// dw[tap][ci][co] (ci < ci_out) = sum over chunks: a workgroup takes 64
// outputs; wave g sums chunks g, g + 4, g + 8, ... in order, then the four
// wave sums are added in wave order (deterministic).
__global__ void __launch_bounds__(256) wgrad_reduce_k(const float* __restrict__ partial, float* __restrict__ dw,
                                                      int chunks, int ci_n, int ci_out, int co_n) {
  __shared__ float red[4][64];
  const int t = threadIdx.x & 63, g = threadIdx.x >> 6;
  const long long e = static_cast<long long>(blockIdx.x) * 64 + t;
  const long long total = 9LL * ci_out * co_n;
  float sum = 0.f;
  if (e < total) {
    const int co = static_cast<int>(e % co_n);
    const int ci = static_cast<int>((e / co_n) % ci_out);
    const int tap = static_cast<int>(e / (static_cast<long long>(co_n) * ci_out));
    for (int c = g; c < chunks; c += 4) sum += partial[((static_cast<size_t>(c) * 9 + tap) * ci_n + ci) * co_n + co];
  }
  red[g][t] = sum;
  __syncthreads();
  if (g == 0 && e < total) dw[e] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// out[i] = sum over chunks of partial[chunk][i]: a strided sum per thread, then a
// fixed tree (one workgroup per output): deterministic.
__global__ void __launch_bounds__(256) chunk_reduce_k(const float* __restrict__ partial, float* __restrict__ out,
                                                      int chunks, int n) {
  __shared__ float red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  float sum = 0.f;
  for (int c = t; c < chunks; c += 256) sum += partial[static_cast<size_t>(c) * n + i];
  red[t] = sum;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) out[i] = red[0];
}

// ------------------------------------------------------------- glue kernels
__global__ void avgpool2_k(Map x, Map y, Shape so) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long total = so.pixels() * x.c;
  if (e >= total) return;
  const int ch = static_cast<int>(e % x.c);
  const long long p = e / x.c;
  const Pix q = pixel_of(p, so);
  const int wi = so.w * 2, hi = so.h * 2;
  const long long b = (static_cast<long long>(q.n) * hi + 2 * q.r) * wi + 2 * q.c;
  const float v = from_bf16(x.p[b * x.ld + x.off + ch]) + from_bf16(x.p[(b + 1) * x.ld + x.off + ch]) +
                  from_bf16(x.p[(b + wi) * x.ld + x.off + ch]) + from_bf16(x.p[(b + wi + 1) * x.ld + x.off + ch]);
  y.p[p * y.ld + y.off + ch] = to_bf16(0.25f * v);
}

__global__ void avgpool2_bwd_add_k(MapF dy, MapF dx, Shape si) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long total = si.pixels() * dx.c;
  if (e >= total) return;
  const int ch = static_cast<int>(e % dx.c);
  const long long p = e / dx.c;
  const Pix q = pixel_of(p, si);
  const long long po = (static_cast<long long>(q.n) * (si.h / 2) + q.r / 2) * (si.w / 2) + q.c / 2;
  dx.p[p * dx.ld + dx.off + ch] += 0.25f * dy.p[po * dy.ld + dy.off + ch];
}

__global__ void upsample2_k(Map x, Map y, Shape si) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  Shape so{si.n, si.h * 2, si.w * 2};
  const long long total = so.pixels() * x.c;
  if (e >= total) return;
  const int ch = static_cast<int>(e % x.c);
  const long long p = e / x.c;
  const Pix q = pixel_of(p, so);
  const long long pi = (static_cast<long long>(q.n) * si.h + q.r / 2) * si.w + q.c / 2;
  y.p[p * y.ld + y.off + ch] = x.p[pi * x.ld + x.off + ch];
}

__global__ void upsample2_bwd_k(MapF dy, MapF dx, Shape si) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long total = si.pixels() * dx.c;
  if (e >= total) return;
  const int ch = static_cast<int>(e % dx.c);
  const long long p = e / dx.c;
  const Pix q = pixel_of(p, si);
  const int wo = si.w * 2;
  const long long b = (static_cast<long long>(q.n) * si.h * 2 + 2 * q.r) * wo + 2 * q.c;
  float v = dy.p[b * dy.ld + dy.off + ch];
  v += dy.p[(b + 1) * dy.ld + dy.off + ch];
  v += dy.p[(b + wo) * dy.ld + dy.off + ch];
  v += dy.p[(b + wo + 1) * dy.ld + dy.off + ch];
  dx.p[p * dx.ld + dx.off + ch] = v;
}

__global__ void add_into_k(MapF src, MapF dst, Shape s) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long total = s.pixels() * dst.c;
  if (e >= total) return;
  const int ch = static_cast<int>(e % dst.c);
  const long long p = e / dst.c;
  dst.p[p * dst.ld + dst.off + ch] += src.p[p * src.ld + src.off + ch];
}

__global__ void out_fwd_k(Map x, const float* __restrict__ w, const float* __restrict__ b,
                          const float* __restrict__ base, int base_ld, float* __restrict__ out, Shape s) {
  const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= s.pixels()) return;
  float o0 = base[p * base_ld] + b[0], o1 = base[p * base_ld + 1] + b[1], o2 = base[p * base_ld + 2] + b[2];
  float a0 = 0.f, a1 = 0.f, a2 = 0.f;
  const uint16_t* row = x.p + p * x.ld + x.off;
  for (int i0 = 0; i0 < x.c; i0 += 8) {  // x.c, ld and off are multiples of 8
    const uint4 v = *reinterpret_cast<const uint4*>(row + i0);
    const uint32_t vw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int i = i0 + k;
      const float xi = from_bf16(static_cast<uint16_t>(vw[k >> 1] >> ((k & 1) * 16)));
      a0 = fmaf(xi, w[i * 3 + 0], a0);
      a1 = fmaf(xi, w[i * 3 + 1], a1);
      a2 = fmaf(xi, w[i * 3 + 2], a2);
    }
  }
  out[p * 3 + 0] = o0 + a0;
  out[p * 3 + 1] = o1 + a1;
  out[p * 3 + 2] = o2 + a2;
}

// Per pixel: dout = 2 (out - t) / count; dx = dout w^T.  Per chunk of
// kOutChunk pixels: partial[chunk] = {dw[ci][3], db[3], sum (out - t)^2}.
// Thread (g, i) of G = 256 / ci groups handles channel i of the chunk's
// pixels g, g + G, ... in order; the groups are added in group order.
constexpr int kOutChunk = 256;
__global__ void __launch_bounds__(256) out_bwd_k(Map x, const float* __restrict__ out, const float* __restrict__ tgt,
                                                 const float* __restrict__ w, MapF dx, float* __restrict__ partial,
                                                 Shape s, float scale) {
  __shared__ float red[7][256];
  const int chunk = blockIdx.x, t = threadIdx.x;
  const int ci = x.c, G = 256 / ci, i = t % ci, g = t / ci;
  const long long P = s.pixels();
  const long long p0 = static_cast<long long>(chunk) * kOutChunk;
  const long long p1 = p0 + kOutChunk < P ? p0 + kOutChunk : P;
  float dw0 = 0.f, dw1 = 0.f, dw2 = 0.f, db0 = 0.f, db1 = 0.f, db2 = 0.f, ls = 0.f;
  if (g < G) {
    const float w0 = w[i * 3], w1 = w[i * 3 + 1], w2 = w[i * 3 + 2];
    for (long long p = p0 + g; p < p1; p += G) {
      const float e0 = out[p * 3] - tgt[p * 3], e1 = out[p * 3 + 1] - tgt[p * 3 + 1], e2 = out[p * 3 + 2] - tgt[p * 3 + 2];
      const float g0 = scale * e0, g1 = scale * e1, g2 = scale * e2;
      const float xi = from_bf16(x.p[p * x.ld + x.off + i]);
      dw0 = fmaf(xi, g0, dw0);
      dw1 = fmaf(xi, g1, dw1);
      dw2 = fmaf(xi, g2, dw2);
      dx.p[p * dx.ld + dx.off + i] = g0 * w0 + g1 * w1 + g2 * w2;
      db0 += g0;
      db1 += g1;
      db2 += g2;
      ls = fmaf(e0, e0, ls);
      ls = fmaf(e1, e1, ls);
      ls = fmaf(e2, e2, ls);
    }
  }
  const float v[7] = {dw0, dw1, dw2, db0, db1, db2, ls};
#pragma unroll
  for (int k = 0; k < 7; ++k) red[k][t] = v[k];
  __syncthreads();
  const int n = ci * 3 + 4;
  float* q = partial + static_cast<size_t>(chunk) * n;
  if (t < ci) {  // dw[t][*]: this channel's groups in order
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float a = 0.f;
      for (int gg = 0; gg < G; ++gg) a += red[k][gg * ci + t];
      q[t * 3 + k] = a;
    }
  } else if (t < ci + 4) {  // db and the loss: every (group, channel) thread, in thread order
    const int k = 3 + (t - ci);
    float a = 0.f;
    for (int u = 0; u < G * ci; u += ci)  // one value per group: the threads of channel 0
      a += red[k][u];
    q[ci * 3 + (t - ci)] = a;
  }
}

// one thread per pixel: 6 f32 in, one 16-byte store of 8 bf16 (channels 6, 7 zero)
__global__ void pack_input_k(const float* __restrict__ in, int in_ld, uint16_t* __restrict__ x, long long P) {
  const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const float* q = in + p * in_ld;
  uint32_t h[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) h[c] = to_bf16(q[c]);
  *reinterpret_cast<uint4*>(x + p * 8) = uint4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), 0u};
}

__global__ void adam_k(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// master [9][ci][co] -> fwd [9][co][ci_pad] and dgrad [9][ci_pad][co] (bf16,
// channels ci..ci_pad-1 zero)
__global__ void refresh_k(const float* __restrict__ wm, uint16_t* __restrict__ wf, uint16_t* __restrict__ wd,
                          int ci, int ci_pad, int co) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 9 * ci_pad * co) return;
  const int o = e % co, i = (e / co) % ci_pad, t = e / (co * ci_pad);
  const uint16_t h = i < ci ? to_bf16(wm[(static_cast<size_t>(t) * ci + i) * co + o]) : static_cast<uint16_t>(0);
  wd[(static_cast<size_t>(t) * ci_pad + i) * co + o] = h;
  wf[(static_cast<size_t>(t) * co + o) * ci_pad + i] = h;
}

// ------------------------------------------------------------- frame glue
__global__ void frame_to_input_k(FrameGlue g, float* __restrict__ in6) {
  const long long p = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const long long P = static_cast<long long>(g.width) * g.height;
  if (p >= P) return;
  const int y = static_cast<int>(p / g.width), x = static_cast<int>(p - static_cast<long long>(y) * g.width);
  const int t = (y / g.tile_h) * g.tiles_x + x / g.tile_w;
  const int q = (y % g.tile_h) * g.tile_w + x % g.tile_w;
  const float4 mu = reinterpret_cast<const float4*>(g.accum)[static_cast<size_t>(t) * g.P + q];
  const float v = g.tile_var[t];
  float* o = in6 + p * 6;
  o[0] = mu.x;
  o[1] = mu.y;
  o[2] = mu.z;
  o[3] = mu.w;
  const int n_acc = g.state->n_acc;
  o[4] = n_acc >= 2 ? logf(v > 1e-12f ? v : 1e-12f) : 0.f;
  o[5] = 1.f / static_cast<float>(n_acc);
}

// display quantisation of one channel to 8 bits (optional gamma)
__device__ __forceinline__ uint32_t q8(float x, bool gamma, float inv_gamma) {
  float y = x > 0.f ? x : 0.f;
  y = y < 1.f ? y : 1.f;
  if (gamma) y = powf(y, inv_gamma);
  return static_cast<uint32_t>(floorf(fmaf(255.f, y, 0.5f)));
}

// The frame's display buffer from its denoised pixels; the padding pixels of
// ragged edge tiles, which the network does not see, take the running mean
// (in den too).
__global__ void frame_display_k(FrameGlue g, float* __restrict__ den, void* final_out, uint32_t mode,
                                float inv_gamma) {
  const long long e = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int T = g.tiles_x * ((g.height + g.tile_h - 1) / g.tile_h);
  if (e >= static_cast<long long>(T) * g.P) return;
  const int t = static_cast<int>(e / g.P), q = static_cast<int>(e - static_cast<long long>(t) * g.P);
  const int x = (t % g.tiles_x) * g.tile_w + q % g.tile_w;
  const int y = (t / g.tiles_x) * g.tile_h + q / g.tile_w;
  float4 v;
  if (x < g.width && y < g.height) {
    v = reinterpret_cast<const float4*>(den)[e];
  } else {
    v = reinterpret_cast<const float4*>(g.accum)[e];
    reinterpret_cast<float4*>(den)[e] = v;
  }
  if (mode & kModeFmtRGBA8) {
    const bool gm = (mode & kModeGamma) != 0;
    static_cast<uint32_t*>(final_out)[e] = q8(v.x, gm, inv_gamma) | (q8(v.y, gm, inv_gamma) << 8) |
                                           (q8(v.z, gm, inv_gamma) << 16) | (q8(v.w, false, 1.f) << 24);
  } else if (mode & kModeFmtF32) {
    static_cast<float4*>(final_out)[e] = v;
  }
}

inline unsigned blocks(long long n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

}  // namespace

template <int BN, int CP, int TH, bool UP, int EPI>
hipError_t launch_conv(const Map& x, const Map& x2, const uint16_t* w, const float* bias, const Map& y, const Map& pool,
                       const OutConv& oc, const Shape& s, hipStream_t st) {
  using C = ConvCfg<BN, TH, CP / kKC, UP>;
  const void* f = reinterpret_cast<const void*>(&conv_fwd_k<BN, CP, TH, UP, EPI>);
  const size_t lds = C::BYTES + (EPI == kEpiFrame ? 99 * 4 : 0);
  const long long tiles = static_cast<long long>(s.n) * ((s.h + TH - 1) / TH) * ((s.w + kTW - 1) / kTW);
  if (tiles == 0) return hipSuccess;
  if (tiles > (1LL << 30)) return hipErrorInvalidValue;
  // resident workgroups per compute unit, per device
  static int per_cu[64] = {0};
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (lds > 64 * 1024) {
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  if (per_cu[dev] == 0) {
    int nb = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, C::NT, lds);
    if (e != hipSuccess) return e;
    per_cu[dev] = nb > 0 ? nb : 1;
  }
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const long long grid = tiles < static_cast<long long>(cus) * per_cu[dev] ? tiles : static_cast<long long>(cus) * per_cu[dev];
  conv_fwd_k<BN, CP, TH, UP, EPI><<<static_cast<unsigned>(grid), C::NT, lds, st>>>(x, x2, w, bias, y, pool, oc, s);
  return hipGetLastError();
}

template <int BN, int CP, int TH, bool UP>
hipError_t launch_tile(const Map& x, const Map& x2, const uint16_t* w, const float* bias, const Map& y,
                       const Map& pool, const Shape& s, hipStream_t st) {
  const OutConv none{nullptr, nullptr, FrameGlue{}, 0.f, nullptr};
  if (pool.p) {
    if constexpr ((TH / 4) % 2 == 0) return launch_conv<BN, CP, TH, UP, kEpiPool>(x, x2, w, bias, y, pool, none, s, st);
    return hipErrorInvalidValue;
  }
  return launch_conv<BN, CP, TH, UP, kEpiPlain>(x, x2, w, bias, y, pool, none, s, st);
}

template <bool UP>
hipError_t conv_tile(const Map& x, const Map& x2, const uint16_t* w, const float* bias, const Map& y,
                     const Map& pool, const Shape& s, hipStream_t st) {
  const int cp = (x.c + x2.c + 31) / 32 * 32;
#define DFB_CONV(BN_, CP_, TH_, THU_) \
  if (y.c == BN_ && cp == CP_) return launch_tile<BN_, CP_, UP ? THU_ : TH_, UP>(x, x2, w, bias, y, pool, s, st);
  DFB_CONV(32, 32, DFB_TH_32_32, DFB_TH_32_32)
  DFB_CONV(32, 64, DFB_TH_32_64, DFB_THU_32_64)
  DFB_CONV(64, 32, DFB_TH_64_32, DFB_TH_64_32)
  DFB_CONV(64, 64, DFB_TH_64_64, DFB_TH_64_64)
  DFB_CONV(64, 128, DFB_TH_64_128, DFB_THU_64_128)
  DFB_CONV(128, 64, DFB_TH_128, DFB_TH_128)
  DFB_CONV(128, 128, DFB_TH_128, DFB_TH_128)
#undef DFB_CONV
  return hipErrorInvalidValue;
}

hipError_t conv3x3_fwd(const Map& x, const uint16_t* w_fwd, const float* bias, const Map& y, const Shape& s,
                       hipStream_t st, bool up, const Map* pool, const Map* x2) {
  const Map none{nullptr, 0, 0, 0};
  const Map& xb = x2 ? *x2 : none;
  if (x.c % 8 || x.ld % 8 || x.off % 8 || y.ld % 8 || y.off % 8) return hipErrorInvalidValue;
  if (x2 && (x.c % 32 || xb.c % 8 || xb.ld != x.ld || xb.off % 8)) return hipErrorInvalidValue;
  if ((up || pool) && (s.h % 2 || s.w % 2)) return hipErrorInvalidValue;
  // per-image element offsets are 32-bit
  const long long img = static_cast<long long>(up ? s.h / 2 : s.h) * (up ? s.w / 2 : s.w) * x.ld;
  if (img >= (1LL << 30) || static_cast<long long>(s.h) * s.w * y.ld >= (1LL << 30)) return hipErrorInvalidValue;
  const Map& pl = pool ? *pool : none;
  if (pool && (pl.ld % 8 || pl.off % 8 || pl.c != y.c)) return hipErrorInvalidValue;
  return up ? conv_tile<true>(x, xb, w_fwd, bias, y, pl, s, st) : conv_tile<false>(x, xb, w_fwd, bias, y, pl, s, st);
}

hipError_t conv3x3_gate(const MapF& dy, const Map& y, const Map& g, float* db, float* partial, const Shape& s,
                        hipStream_t st) {
  if (dy.c % 8 || dy.ld % 4 || dy.off % 4 || y.ld % 8 || y.off % 8 || g.ld % 8 || g.off % 8 || g.c != dy.c ||
      256 % (dy.c / 8))
    return hipErrorInvalidValue;
  const unsigned nb = blocks(s.pixels() * (dy.c / 8), 256);
  gate_k<<<nb, 256, 0, st>>>(dy, y, g, partial, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  chunk_reduce_k<<<dy.c, 256, 0, st>>>(partial, db, static_cast<int>(nb), dy.c);
  return hipGetLastError();
}

hipError_t conv3x3_dgrad(const Map& g, const uint16_t* w_dgrad, const MapF& dx, const Shape& s, hipStream_t st) {
  const unsigned nb = blocks(s.pixels(), BM);
  if (g.c % 8 || g.ld % 8 || g.off % 8) return hipErrorInvalidValue;
  switch (dx.c) {
    case 32: conv_dgrad_k<32><<<nb, 256, 0, st>>>(g, w_dgrad, dx, s); break;
    case 64: conv_dgrad_k<64><<<nb, 256, 0, st>>>(g, w_dgrad, dx, s); break;
    case 128: conv_dgrad_k<128><<<nb, 256, 0, st>>>(g, w_dgrad, dx, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t conv3x3_wgrad_scratch(int ci, int co, const Shape& s) {
  const long long chunks = (s.pixels() + kWgradChunk - 1) / kWgradChunk;
  const long long bchunks = (s.pixels() * (co / 8) + 255) / 256;  // gate_k's blocks
  const size_t wsum = static_cast<size_t>(chunks) * 9 * ci * co, bsum = static_cast<size_t>(bchunks) * co;
  return wsum > bsum ? wsum : bsum;
}

hipError_t conv3x3_wgrad(const Map& x, const Map& g, float* dw, float* partial, const Shape& s, hipStream_t st,
                         int ci_out) {
  const int chunks = static_cast<int>((s.pixels() + kWgradChunk - 1) / kWgradChunk);
  if (x.c % 8 || x.ld % 8 || x.off % 8) return hipErrorInvalidValue;
  if (g.ld % 4 || g.off % 4) return hipErrorInvalidValue;
  dim3 grid(chunks, 9, (x.c + BM - 1) / BM);
  const bool half = x.c <= 32;  // one 32-row c_in block carries every input channel
  switch (g.c) {
    case 32:
      if (half) conv_wgrad_k<32, true><<<grid, 256, 0, st>>>(x, g, partial, s);
      else conv_wgrad_k<32, false><<<grid, 256, 0, st>>>(x, g, partial, s);
      break;
    case 64:
      if (half) conv_wgrad_k<64, true><<<grid, 256, 0, st>>>(x, g, partial, s);
      else conv_wgrad_k<64, false><<<grid, 256, 0, st>>>(x, g, partial, s);
      break;
    case 128:
      if (half) conv_wgrad_k<128, true><<<grid, 256, 0, st>>>(x, g, partial, s);
      else conv_wgrad_k<128, false><<<grid, 256, 0, st>>>(x, g, partial, s);
      break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  wgrad_reduce_k<<<blocks(9LL * ci_out * g.c, 64), 256, 0, st>>>(partial, dw, chunks, x.c, ci_out, g.c);
  return hipGetLastError();
}

hipError_t avgpool2(const Map& x, const Map& y, const Shape& s_in, hipStream_t st) {
  Shape so{s_in.n, s_in.h / 2, s_in.w / 2};
  avgpool2_k<<<blocks(so.pixels() * x.c, 256), 256, 0, st>>>(x, y, so);
  return hipGetLastError();
}
hipError_t avgpool2_backward_add(const MapF& dy, const MapF& dx, const Shape& s_in, hipStream_t st) {
  avgpool2_bwd_add_k<<<blocks(s_in.pixels() * dx.c, 256), 256, 0, st>>>(dy, dx, s_in);
  return hipGetLastError();
}
hipError_t upsample2(const Map& x, const Map& y, const Shape& s_in, hipStream_t st) {
  upsample2_k<<<blocks(s_in.pixels() * 4 * x.c, 256), 256, 0, st>>>(x, y, s_in);
  return hipGetLastError();
}
hipError_t upsample2_backward(const MapF& dy, const MapF& dx, const Shape& s_in, hipStream_t st) {
  upsample2_bwd_k<<<blocks(s_in.pixels() * dx.c, 256), 256, 0, st>>>(dy, dx, s_in);
  return hipGetLastError();
}
hipError_t add_into(const MapF& src, const MapF& dst, const Shape& s, hipStream_t st) {
  add_into_k<<<blocks(s.pixels() * dst.c, 256), 256, 0, st>>>(src, dst, s);
  return hipGetLastError();
}

hipError_t conv3x3_in_fwd(const Map& x, const uint16_t* w_fwd, const float* bias, const Map& y, const Shape& s,
                          hipStream_t st) {
  if (y.c != 32 || y.ld % 8 || y.off % 8) return hipErrorInvalidValue;
  if (x.c != 8 || x.ld % 8 || x.off % 8) return hipErrorInvalidValue;
  const long long img = static_cast<long long>(s.h) * s.w;
  if (img * x.ld * 2 >= (1LL << 31) || img * y.ld >= (1LL << 30)) return hipErrorInvalidValue;
  const long long tiles = static_cast<long long>(s.n) * ((s.h + kInTH - 1) / kInTH) * ((s.w + kTW - 1) / kTW);
  if (tiles == 0) return hipSuccess;
  if (tiles > (1LL << 30)) return hipErrorInvalidValue;
  conv_in_k<false><<<static_cast<unsigned>(tiles), 256, 0, st>>>(x, FrameGlue{}, w_fwd, bias, y, s);
  return hipGetLastError();
}

hipError_t conv3x3_in_frame(const FrameGlue& g, const uint16_t* w_fwd, const float* bias, const Map& y,
                            const Shape& s, hipStream_t st) {
  if (y.c != 32 || y.ld % 8 || y.off % 8 || s.n != 1 || s.h != g.height || s.w != g.width) return hipErrorInvalidValue;
  if (static_cast<long long>(s.h) * s.w * y.ld >= (1LL << 30)) return hipErrorInvalidValue;
  const long long tiles = static_cast<long long>((s.h + kInTH - 1) / kInTH) * ((s.w + kTW - 1) / kTW);
  if (tiles == 0) return hipSuccess;
  const Map none{nullptr, 0, 0, 0};
  conv_in_k<true><<<static_cast<unsigned>(tiles), 256, 0, st>>>(none, g, w_fwd, bias, y, s);
  return hipGetLastError();
}

hipError_t conv3x3_out_frame(const Map& x, const uint16_t* w_fwd, const float* bias, const float* ow, const float* ob,
                             const FrameGlue& g, float tau, float* den, void* final_out, uint32_t mode,
                             float inv_gamma, const Shape& s, hipStream_t st) {
  if (x.c != 32 || x.ld % 8 || x.off % 8 || !den || s.n != 1 || s.h != g.height || s.w != g.width)
    return hipErrorInvalidValue;
  if ((mode & (kModeFmtRGBA8 | kModeFmtF32)) && !final_out) return hipErrorInvalidValue;
  const long long T = static_cast<long long>(g.tiles_x) * ((g.height + g.tile_h - 1) / g.tile_h);
  if (T * g.P * 16 >= (1LL << 31) || static_cast<long long>(s.h) * s.w * x.ld >= (1LL << 30))
    return hipErrorInvalidValue;
  const Map none{nullptr, 0, 0, 0};
  const OutConv oc{ow, ob, g, tau, den};
  const Map y{nullptr, 32, 0, 32};
  hipError_t e = launch_conv<32, 32, DFB_TH_32_32, false, kEpiFrame>(x, none, w_fwd, bias, y, none, oc, s, st);
  if (e != hipSuccess) return e;
  frame_display_k<<<blocks(T * g.P, 256), 256, 0, st>>>(g, den, final_out, mode, inv_gamma);
  return hipGetLastError();
}

hipError_t out_conv_fwd(const Map& x, const float* w, const float* b, const float* base, int base_ld, float* out,
                        const Shape& s, hipStream_t st) {
  out_fwd_k<<<blocks(s.pixels(), 256), 256, 0, st>>>(x, w, b, base, base_ld, out, s);
  return hipGetLastError();
}

size_t out_conv_scratch(const Shape& s) {  // per-chunk partials + their sum
  const long long chunks = (s.pixels() + kOutChunk - 1) / kOutChunk;
  return static_cast<size_t>(chunks + 1) * (32 * 3 + 4);
}

hipError_t out_conv_backward(const Map& x, const float* out, const float* target, const float* w, const MapF& dx,
                             float* dw, float* db, float* loss, float* partial, const Shape& s, hipStream_t st) {
  if (x.c > 64) return hipErrorInvalidValue;
  const int chunks = static_cast<int>((s.pixels() + kOutChunk - 1) / kOutChunk);
  const float scale = 2.f / static_cast<float>(s.pixels() * 3);
  out_bwd_k<<<chunks, 256, 0, st>>>(x, out, target, w, dx, partial, s, scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = x.c * 3 + 4;
  // dw (ci*3), db (3) and the loss sum are consecutive in each partial row
  chunk_reduce_k<<<n, 256, 0, st>>>(partial, partial + static_cast<size_t>(chunks) * n, chunks, n);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const float* red = partial + static_cast<size_t>(chunks) * n;
  e = hipMemcpyAsync(dw, red, sizeof(float) * x.c * 3, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(db, red + x.c * 3, sizeof(float) * 3, hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(loss, red + x.c * 3 + 3, sizeof(float), hipMemcpyDeviceToDevice, st);
}

hipError_t pack_input(const float* in, int in_ld, uint16_t* x, const Shape& s, hipStream_t st) {
  if (reinterpret_cast<uintptr_t>(x) % 16) return hipErrorInvalidValue;
  pack_input_k<<<blocks(s.pixels(), 256), 256, 0, st>>>(in, in_ld, x, s.pixels());
  return hipGetLastError();
}

hipError_t adam_update(float* w, const float* g, float* m, float* v, long long n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2, hipStream_t st) {
  adam_k<<<blocks(n, 256), 256, 0, st>>>(w, g, m, v, n, lr, beta1, beta2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t refresh_bf16(const float* w_master, uint16_t* w_fwd, uint16_t* w_dgrad, int ci, int co, hipStream_t st) {
  const int ci_pad = (ci + 7) / 8 * 8;
  refresh_k<<<blocks(9LL * ci_pad * co, 256), 256, 0, st>>>(w_master, w_fwd, w_dgrad, ci, ci_pad, co);
  return hipGetLastError();
}

hipError_t frame_to_input(const FrameGlue& g, float* in6, hipStream_t st) {
  frame_to_input_k<<<blocks(static_cast<long long>(g.width) * g.height, 256), 256, 0, st>>>(g, in6);
  return hipGetLastError();
}


}  // namespace unet
}  // namespace dfb
