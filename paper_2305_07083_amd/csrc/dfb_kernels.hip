// gfx950 kernels of the per-tile sort-last compositor.
//
// One persistent launch per frame.  Each workgroup (64 * waves_per_tile lanes)
// repeatedly takes a work unit -- a work_w x work_h rectangle of one DFB tile
// -- from a device queue ordered longest tile first, and for every pixel of it
//   1. builds the key (ordered depth bits << 32 | layer index) of each of the
//      tile's K layers from coalesced SoA depth loads, staging alpha in LDS,
//   2. sorts the keys (registers for K <= 32, an LDS bitonic sort shared by
//      the workgroup for larger K),
//   3. walks the sorted keys front to back computing the transmittance T in
//      front of each layer ("over", Sec. 4.2 of the paper) and writes it back
//      into the layer's LDS slot,
//   4. sums T_l * colour_l in layer order with coalesced colour loads and puts
//      the background behind (the generation-0 tile),
//   5. optionally stores the finished f32 pixel, folds it into the running
//      mean and M2 (Welford) and tonemaps the displayed value to RGBA8.
// Per-tile variance: a wave/LDS reduction of M2 over the unit; units of one
// tile combine their partial sums in a fixed order (deterministic).
// Every fragment byte is read from HBM exactly once.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "dfb_internal.h"
#include "sortnet.h"

namespace dfb {
namespace {

// Fragment planes are read exactly once per frame: streaming (non-temporal)
// loads keep them from displacing the outputs in L2.
#ifndef DFB_NT_LOADS
#define DFB_NT_LOADS 1
#endif
// Minimum waves per SIMD requested from the register allocator, per
// register-sort capacity (0 = no request).
#ifndef DFB_WAVES_K8
#define DFB_WAVES_K8 0
#endif
#ifndef DFB_WAVES_K16
#define DFB_WAVES_K16 0
#endif
#ifndef DFB_WAVES_K32
#define DFB_WAVES_K32 0
#endif
// Largest register-sort bucket that loads all five planes up front (larger
// buckets load depth and alpha first and the colours after the walk);
// 0 = chosen per kernel capacity (upfront_max).
#ifndef DFB_UPFRONT_MAX
#define DFB_UPFRONT_MAX 0
#endif
// Streaming (non-temporal) loads in the K > 32 path too (1), or ordinary
// loads (0, the default): those leave a line in L2 for the pixel group that
// reads its other half (a group of 16 or fewer fp32 pixels covers half a
// 128-byte line or less); on the 8192^2 heavy-tailed frame 36.5 against
// 38.6 ms.
#ifndef DFB_BIGK_NT
#define DFB_BIGK_NT 0
#endif
// Layers whose plane loads the list and averaging operations keep in flight
// per lane.
#ifndef DFB_OP_CHUNK
#define DFB_OP_CHUNK 4
#endif

// Plane loads: `base` is uniform across the wave (a layer's block start) and
// `i` a 32-bit element offset inside the block, so each load is one
// instruction with a scalar base address.
template <typename FT>
__device__ __forceinline__ float ldf(const FT* __restrict__ base, uint32_t i);
template <>
__device__ __forceinline__ float ldf<float>(const float* __restrict__ base, uint32_t i) {
#if DFB_NT_LOADS
  return __builtin_nontemporal_load(base + i);
#else
  return base[i];
#endif
}
template <>
__device__ __forceinline__ float ldf<_Float16>(const _Float16* __restrict__ base, uint32_t i) {
#if DFB_NT_LOADS
  return static_cast<float>(__builtin_nontemporal_load(base + i));
#else
  return static_cast<float>(base[i]);
#endif
}

// Workgroup barrier for LDS traffic only.  Threads of a workgroup share
// nothing through global memory inside these kernels, so a barrier need not
// wait for the wave's global stores to complete (which __syncthreads does:
// that wait costs a memory round trip at every unit boundary).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Order-preserving map of a depth to 32 bits: NaN above everything, -0 == +0.
__device__ __forceinline__ uint32_t depth_bits(float d) {
  uint32_t b = __float_as_uint(d);
  if (d != d) return 0xFFFFFFFFu;
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// Order-preserving map of a binary16 depth to 16 bits, same rules.
__device__ __forceinline__ uint32_t half_depth_bits(uint16_t h) {
  if ((h & 0x7C00u) == 0x7C00u && (h & 0x03FFu)) return 0xFFFFu;
  if (h == 0x8000u) h = 0;
  return (h & 0x8000u) ? (~static_cast<uint32_t>(h) & 0xFFFFu) : (static_cast<uint32_t>(h) | 0x8000u);
}

// Keys of fp32 depths.  The sort order (ordered depth bits, then layer
// index) is that of the 44-bit integer x = depth_bits << 12 | l (l < 4096).  Held as
// the double 2^52 + x (bit pattern 0x433 << 52 | x), every key is a normal
// double whose value orders like x, so a comparator is one v_min_f64 and one
// v_max_f64 instead of two 64-bit integer compares and four selects.  The
// layer index is the low 12 bits of the pattern.
constexpr uint64_t kKeyBias = 0x4330000000000000ull;
constexpr uint64_t kKeyPad = kKeyBias | 0x00000FFFFFFFFFFFull;  // not below any real key
__device__ __forceinline__ uint64_t big_key(uint32_t dbits, int l) {
  return kKeyBias | (static_cast<uint64_t>(dbits) << 12) | static_cast<uint32_t>(l);
}
__device__ __forceinline__ int key_layer(uint64_t k) { return static_cast<int>(k & 0xFFFu); }
struct KeyMinMax {
  __device__ __forceinline__ void operator()(uint64_t& a, uint64_t& b) const {
    const double x = __builtin_bit_cast(double, a), y = __builtin_bit_cast(double, b);
    double lo, hi;
    asm("v_min_f64 %0, %1, %2" : "=v"(lo) : "v"(x), "v"(y));
    asm("v_max_f64 %0, %1, %2" : "=v"(hi) : "v"(x), "v"(y));
    a = __builtin_bit_cast(uint64_t, lo);
    b = __builtin_bit_cast(uint64_t, hi);
  }
};

// Sort keys of the register path: (ordered depth bits, layer index), as one
// number so that one comparison orders by depth and breaks ties by index (the
// layers of a tile are in source-id order).  fp32 depths take the 64-bit
// double-encoded key above; fp16 depths and an index below 65536 fit 32 bits
// (v_min_u32 / v_max_u32), which also halves the registers.
template <typename FT>
struct SortKey;
template <>
struct SortKey<float> {
  using K = uint64_t;
  using CE = KeyMinMax;
  static constexpr K kPad = kKeyPad;
  __device__ static __forceinline__ K make(const float* __restrict__ b, uint32_t i, int l) {
    return big_key(depth_bits(ldf<float>(b, i)), l);
  }
  __device__ static __forceinline__ int index(K k) { return key_layer(k); }
};
template <>
struct SortKey<_Float16> {
  using K = uint32_t;
  using CE = CompareExchange<uint32_t>;
  static constexpr K kPad = ~0u;
  __device__ static __forceinline__ K make(const _Float16* __restrict__ b, uint32_t i, int l) {
#if DFB_NT_LOADS
    const _Float16 d = __builtin_nontemporal_load(b + i);
#else
    const _Float16 d = b[i];
#endif
    return (half_depth_bits(__builtin_bit_cast(uint16_t, d)) << 16) | static_cast<uint32_t>(l);
  }
  __device__ static __forceinline__ int index(K k) { return static_cast<int>(k & 0xFFFFu); }
};

__device__ __forceinline__ uint32_t quantise(float x, bool gamma, float inv_gamma) {
  float y = x > 0.f ? x : 0.f;  // NaN compares false -> 0
  y = y < 1.f ? y : 1.f;
  if (gamma) y = powf(y, inv_gamma);
  return static_cast<uint32_t>(floorf(fmaf(255.f, y, 0.5f)));
}

__device__ __forceinline__ uint32_t pack_rgba8(float4 v, uint32_t mode, float inv_gamma) {
  const bool g = (mode & kModeGamma) != 0;
  return quantise(v.x, g, inv_gamma) | (quantise(v.y, g, inv_gamma) << 8) |
         (quantise(v.z, g, inv_gamma) << 16) | (quantise(v.w, false, 1.f) << 24);
}

// Pixel -> finished / accumulated / displayed outputs.  Returns the pixel's
// M2 sum over RGB (0 when not accumulating or outside the image).
__device__ __forceinline__ float store_pixel(float4 x, size_t px, size_t m2_base, int P,
                                             bool inside, uint32_t mode, int n_acc, float inv_n,
                                             float inv_gamma, float* finished, float* accum,
                                             float* m2, void* final_out) {
  if (mode & kModeKeepFinished) reinterpret_cast<float4*>(finished)[px] = x;
  float4 disp = x;
  float vs = 0.f;
  if (mode & kModeAccumulate) {
    float* q = m2 + m2_base;
    float4 mu;
    float q0, q1, q2;
    if (n_acc == 1) {
      mu = x;
      q0 = q1 = q2 = 0.f;
    } else {
      mu = reinterpret_cast<const float4*>(accum)[px];
      q0 = q[0];
      q1 = q[P];
      q2 = q[2 * P];
      const float d0 = x.x - mu.x, d1 = x.y - mu.y, d2 = x.z - mu.z, d3 = x.w - mu.w;
      mu.x = fmaf(d0, inv_n, mu.x);
      mu.y = fmaf(d1, inv_n, mu.y);
      mu.z = fmaf(d2, inv_n, mu.z);
      mu.w = fmaf(d3, inv_n, mu.w);
      q0 = fmaf(d0, x.x - mu.x, q0);
      q1 = fmaf(d1, x.y - mu.y, q1);
      q2 = fmaf(d2, x.z - mu.z, q2);
    }
    reinterpret_cast<float4*>(accum)[px] = mu;
    q[0] = q0;
    q[P] = q1;
    q[2 * P] = q2;
    if (inside) vs = q0 + q1 + q2;
    disp = mu;
  }
  if (mode & kModeFmtRGBA8) {
    static_cast<uint32_t*>(final_out)[px] = pack_rgba8(disp, mode, inv_gamma);
  } else if (mode & kModeFmtF32) {
    static_cast<float4*>(final_out)[px] = disp;
  }
  return vs;
}

struct Unit {
  int t, sx0, sy0, x0, y0;  // tile, unit origin inside the tile, tile origin in the image
};

__device__ __forceinline__ int unit_pixel(const FrameArgs& a, const Unit& u, int q, bool& inside) {
  const int qy = a.work_shift >= 0 ? (q >> a.work_shift) : q / a.work_w;
  const int qx = q - qy * a.work_w;
  const int ty = u.sy0 + qy, tx = u.sx0 + qx;
  inside = (u.x0 + tx < a.width) && (u.y0 + ty < a.height);
  return ty * a.tile_w + tx;
}

__device__ __forceinline__ float finish_px(const FrameArgs& a, const Unit& u, int p, bool inside,
                                           float4 x) {
  const size_t px = static_cast<size_t>(u.t) * a.P + p;
  const size_t mb = static_cast<size_t>(u.t) * 3 * a.P + p;
  return store_pixel(x, px, mb, a.P, inside, a.mode, a.n_acc, a.inv_n, a.inv_gamma, a.finished,
                     a.accum, a.m2, a.final_out);
}

// ---------------------------------------------------------------- K <= 32
// One lane per pixel.  All five planes of the pixel's K fragments are loaded
// up front (one memory round trip per pixel, 5K loads in flight); colours
// stay in registers indexed by layer, so only the sorted walk needs dynamic
// indexing: wl points at this lane's column of a [KMAX][NT] LDS array, the
// lane writes alpha of layer l to wl[l*NT] and the walk overwrites it with
// the transmittance in front of layer l.  No lane reads another lane's
// column, so no barrier is needed.
template <typename FT, int KMAX>
__device__ __forceinline__ float4 composite_px_upfront(float& Tout, const FrameArgs& a,
                                                       const int64_t* __restrict__ loff, int K,
                                                       int off, int p, float* __restrict__ wl,
                                                       int NT) {
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  const uint32_t up = static_cast<uint32_t>(p);
  using SK = SortKey<FT>;
  typename SK::K key[KMAX];
  float alp[KMAX], cr[KMAX], cg[KMAX], cb[KMAX];
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l < K) {
      const FT* __restrict__ b = frag + loff[l];
      key[l] = SK::make(b, 4 * P + up, l);
      alp[l] = ldf<FT>(b, 3 * P + up);
      cr[l] = ldf<FT>(b, up);
      cg[l] = ldf<FT>(b, P + up);
      cb[l] = ldf<FT>(b, 2 * P + up);
    } else {
      key[l] = SK::kPad;
    }
  }
#pragma unroll
  for (int l = 0; l < KMAX; ++l)
    if (l < K) wl[l * NT] = alp[l];
  sort_network<KMAX>(key, typename SK::CE());
  float T = 1.f, A = 0.f;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    if (i < K) {
      const int l = SK::index(key[i]);
      const float al = wl[l * NT];
      wl[l * NT] = T;
      A = fmaf(T, al, A);
      T = T * (1.f - al);
      if (a.mode & kModeKeepOrder)
        a.order[static_cast<size_t>(off + i) * P + p] = static_cast<uint16_t>(l);
    }
  }
  float R = 0.f, G = 0.f, B = 0.f;
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l < K) {
      const float w = wl[l * NT];
      R = fmaf(w, cr[l], R);
      G = fmaf(w, cg[l], G);
      B = fmaf(w, cb[l], B);
    }
  }
  Tout = T;
  return make_float4(R, G, B, A);
}

// Larger K: 5K values per lane no longer fit the register file next to the
// keys, so depth and alpha are loaded first and the colours only after the
// walk (two memory round trips per pixel, half the registers).
template <typename FT, int KMAX>
__device__ __forceinline__ float4 composite_px_two_phase(float& Tout, const FrameArgs& a,
                                                         const int64_t* __restrict__ loff, int K,
                                                         int off, int p, float* __restrict__ wl,
                                                         int NT) {
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  const uint32_t up = static_cast<uint32_t>(p);
  using SK = SortKey<FT>;
  typename SK::K key[KMAX];
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l < K) {
      const FT* __restrict__ b = frag + loff[l];
      key[l] = SK::make(b, 4 * P + up, l);
      wl[l * NT] = ldf<FT>(b, 3 * P + up);
    } else {
      key[l] = SK::kPad;
    }
  }
  sort_network<KMAX>(key, typename SK::CE());
  float T = 1.f, A = 0.f;
#pragma unroll
  for (int i = 0; i < KMAX; ++i) {
    if (i < K) {
      const int l = SK::index(key[i]);
      const float al = wl[l * NT];
      wl[l * NT] = T;
      A = fmaf(T, al, A);
      T = T * (1.f - al);
      if (a.mode & kModeKeepOrder)
        a.order[static_cast<size_t>(off + i) * P + p] = static_cast<uint16_t>(l);
    }
  }
  float R = 0.f, G = 0.f, B = 0.f;
#pragma unroll
  for (int l = 0; l < KMAX; ++l) {
    if (l < K) {
      const FT* __restrict__ b = frag + loff[l];
      const float w = wl[l * NT];
      R = fmaf(w, ldf<FT>(b, up), R);
      G = fmaf(w, ldf<FT>(b, P + up), G);
      B = fmaf(w, ldf<FT>(b, 2 * P + up), B);
    }
  }
  Tout = T;
  return make_float4(R, G, B, A);
}

// Up-front loads for buckets up to upfront_max(KCAP): one memory round trip
// per pixel instead of two, at the cost of registers.  The fp32 16-layer
// kernel stays at 3 waves per SIMD with all its buckets up front (2048^2
// bricks: 139 against 144 us); the fp16 one would drop from 4 to 3, so its
// 12/16 buckets load in two phases.  The fp32 32-layer kernel stays at 2
// waves with the 24 bucket up front (4096x1024: 225 against 232 us); its 32
// bucket loads in two phases.  The fp16 32-layer kernel loads up to 12
// layers up front: 168 VGPRs, 3 waves per SIMD instead of 2 with the 24
// bucket up front (211 VGPRs): the 4096x1024 fp16 frame takes 164 instead of
// 186 us.
#ifndef DFB_UPFRONT_F16_K32
#define DFB_UPFRONT_F16_K32 12   // largest up-front bucket of the fp16 32-layer kernel
#endif
template <typename FT>
constexpr int upfront_max(int kcap) {
  return DFB_UPFRONT_MAX > 0 ? DFB_UPFRONT_MAX
                             : (kcap <= 16 ? (sizeof(FT) == 4 ? 16 : 8) : (sizeof(FT) == 4 ? 24 : DFB_UPFRONT_F16_K32));
}

template <typename FT, int KMAX, int KCAP>
__device__ __forceinline__ float4 composite_px(float& T, const FrameArgs& a, const int64_t* __restrict__ loff,
                                               int K, int off, int p, float* __restrict__ wl,
                                               int NT) {
  if constexpr (KMAX <= upfront_max<FT>(KCAP)) return composite_px_upfront<FT, KMAX>(T, a, loff, K, off, p, wl, NT);
  else return composite_px_two_phase<FT, KMAX>(T, a, loff, K, off, p, wl, NT);
}

// The background (the generation-0 tile) behind whatever transmittance T is
// left: a constant colour, or a per-pixel image when one is configured.
__device__ __forceinline__ float4 with_background(const FrameArgs& a, int t, int p, float4 x, float T) {
  float4 bg;
  if (a.bg_image) {
    bg = reinterpret_cast<const float4*>(a.bg_image)[static_cast<size_t>(t) * a.P + p];
  } else {
    bg = make_float4(a.bg[0], a.bg[1], a.bg[2], a.bg[3]);
  }
  return make_float4(fmaf(T, bg.x, x.x), fmaf(T, bg.y, x.y), fmaf(T, bg.z, x.z), fmaf(T, bg.w, x.w));
}

template <typename FT, int KMAX, int KCAP>
__device__ float unit_reg(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff, int K, int off,
                          float* lds) {
  static_assert(KMAX <= KCAP, "bucket within the kernel's capacity");
  const int NT = blockDim.x, tid = threadIdx.x;
  float vs = 0.f;
  for (int q = tid; q < a.work_px; q += NT) {
    bool inside;
    const int p = unit_pixel(a, u, q, inside);
    float T;
    const float4 x = composite_px<FT, KMAX, KCAP>(T, a, loff, K, off, p, lds + tid, NT);
    vs += finish_px(a, u, p, inside, with_background(a, u.t, p, x, T));
  }
  return vs;
}

__device__ float unit_background(const FrameArgs& a, const Unit& u) {
  const int NT = blockDim.x;
  float vs = 0.f;
  for (int q = threadIdx.x; q < a.work_px; q += NT) {
    bool inside;
    const int p = unit_pixel(a, u, q, inside);
    vs += finish_px(a, u, p, inside, with_background(a, u.t, p, make_float4(0.f, 0.f, 0.f, 0.f), 1.f));
  }
  return vs;
}

// Rank-order list (the paper's alternative when a per-rank order is correct):
// the tile's layers, ordered by generation (their source_id) back to front,
// are blended front to back from the highest generation down -- no depth is
// read and nothing is sorted.
template <typename FT>
__device__ float unit_list(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff, int K,
                           int off) {
  const int NT = blockDim.x;
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  float vs = 0.f;
  for (int q = threadIdx.x; q < a.work_px; q += NT) {
    bool inside;
    const int p = unit_pixel(a, u, q, inside);
    const uint32_t up = static_cast<uint32_t>(p);
    float R = 0.f, G = 0.f, B = 0.f, A = 0.f, T = 1.f;
    int i = 0;
    for (; i + 4 <= K; i += 4) {  // 4 layers' loads in flight
      float cr[4], cg[4], cb[4], al[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const FT* __restrict__ b = frag + loff[K - 1 - (i + j)];
        cr[j] = ldf<FT>(b, up);
        cg[j] = ldf<FT>(b, P + up);
        cb[j] = ldf<FT>(b, 2 * P + up);
        al[j] = ldf<FT>(b, 3 * P + up);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        R = fmaf(T, cr[j], R);
        G = fmaf(T, cg[j], G);
        B = fmaf(T, cb[j], B);
        A = fmaf(T, al[j], A);
        T = T * (1.f - al[j]);
        if (a.mode & kModeKeepOrder)
          a.order[static_cast<size_t>(off + i + j) * P + p] = static_cast<uint16_t>(K - 1 - (i + j));
      }
    }
    for (; i < K; ++i) {
      const FT* __restrict__ b = frag + loff[K - 1 - i];
      const float al = ldf<FT>(b, 3 * P + up);
      R = fmaf(T, ldf<FT>(b, up), R);
      G = fmaf(T, ldf<FT>(b, P + up), G);
      B = fmaf(T, ldf<FT>(b, 2 * P + up), B);
      A = fmaf(T, al, A);
      T = T * (1.f - al);
      if (a.mode & kModeKeepOrder)
        a.order[static_cast<size_t>(off + i) * P + p] = static_cast<uint16_t>(K - 1 - i);
    }
    vs += finish_px(a, u, p, inside, with_background(a, u.t, p, make_float4(R, G, B, A), T));
  }
  return vs;
}

// 16-byte plane loads: V consecutive elements of one plane (4 fp32 or 8
// fp16 pixels), converted to float.  The element offset is a multiple of V
// and the block start is 16-byte aligned (checked on the host).
template <typename FT>
struct VecWidth;
template <>
struct VecWidth<float> {
  static constexpr int V = 4;
};
template <>
struct VecWidth<_Float16> {
  static constexpr int V = 8;
};

template <typename FT>
__device__ __forceinline__ void ldv(const FT* __restrict__ base, uint32_t i, float* out);
template <>
__device__ __forceinline__ void ldv<float>(const float* __restrict__ base, uint32_t i, float* out) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  const f4 v = __builtin_nontemporal_load(reinterpret_cast<const f4*>(base + i));
  out[0] = v.x;
  out[1] = v.y;
  out[2] = v.z;
  out[3] = v.w;
}
template <>
__device__ __forceinline__ void ldv<_Float16>(const _Float16* __restrict__ base, uint32_t i, float* out) {
  typedef _Float16 h8 __attribute__((ext_vector_type(8)));
  const h8 v = __builtin_nontemporal_load(reinterpret_cast<const h8*>(base + i));
#pragma unroll
  for (int k = 0; k < 8; ++k) out[k] = static_cast<float>(v[k]);
}

// Block offsets of a tile's layers [base, base + 64) held one per lane, so a
// layer's offset is a register read (no dependent scalar load in the loop).
__device__ __forceinline__ int64_t lane_offsets(const int64_t* __restrict__ loff, int base, int K) {
  const int l = base + static_cast<int>(__lane_id());
  return (l >= 0 && l < K) ? loff[l] : 0;
}
__device__ __forceinline__ int64_t offset_of(int64_t held, int k) {
  const uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(held), k);
  const uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(static_cast<uint64_t>(held) >> 32), k);
  return static_cast<int64_t>((static_cast<uint64_t>(hi) << 32) | lo);
}

// V pixels of one unit row per lane; the finished pixels go through the same
// per-pixel epilogue as the scalar path.
template <int V, bool BG>
__device__ __forceinline__ float finish_row(const FrameArgs& a, const Unit& u, int q0, int p0, const float* R,
                                            const float* G, const float* B, const float* A, const float* T) {
  float vs = 0.f;
#pragma unroll
  for (int v = 0; v < V; ++v) {
    bool inside;
    unit_pixel(a, u, q0 + v, inside);
    float4 x = make_float4(R[v], G[v], B[v], A[v]);
    if constexpr (BG) x = with_background(a, u.t, p0 + v, x, T[v]);
    vs += finish_px(a, u, p0 + v, inside, x);
  }
  return vs;
}

// The list operation with 16-byte loads: C layers' four planes in flight per
// lane, blended front to back from the highest generation.
template <typename FT>
__device__ float unit_list_vec(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff, int K,
                               int off) {
  constexpr int V = VecWidth<FT>::V;
  constexpr int C = DFB_OP_CHUNK;
  const int NT = blockDim.x;
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  float vs = 0.f;
  // whole waves run the loop (the held offsets need every lane); lanes past
  // the unit's end load a valid row again and store nothing
  const int lane = static_cast<int>(threadIdx.x & 63);
  for (int base = static_cast<int>(threadIdx.x >> 6) * 64 * V; base < a.work_px; base += NT * V) {
    const bool act = base + lane * V < a.work_px;
    const int q0 = act ? base + lane * V : base;
    bool in0;
    const int p0 = unit_pixel(a, u, q0, in0);
    const uint32_t up = static_cast<uint32_t>(p0);
    float R[V], G[V], B[V], A[V], T[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R[v] = G[v] = B[v] = A[v] = 0.f;
      T[v] = 1.f;
    }
    int i = 0;
    int64_t held = 0;
    for (; i + C <= K; i += C) {
      if ((i & 63) == 0) held = lane_offsets(loff, K - 64 - i, K);  // layers K-64-i .. K-1-i
      float x[C][4][V];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const FT* __restrict__ b = frag + offset_of(held, 63 - ((i + j) & 63));
#pragma unroll
        for (int c = 0; c < 4; ++c) ldv<FT>(b, c * P + up, x[j][c]);
      }
#pragma unroll
      for (int j = 0; j < C; ++j) {
#pragma unroll
        for (int v = 0; v < V; ++v) {
          R[v] = fmaf(T[v], x[j][0][v], R[v]);
          G[v] = fmaf(T[v], x[j][1][v], G[v]);
          B[v] = fmaf(T[v], x[j][2][v], B[v]);
          A[v] = fmaf(T[v], x[j][3][v], A[v]);
          T[v] = T[v] * (1.f - x[j][3][v]);
        }
        if ((a.mode & kModeKeepOrder) && act) {
#pragma unroll
          for (int v = 0; v < V; ++v)
            a.order[static_cast<size_t>(off + i + j) * P + p0 + v] = static_cast<uint16_t>(K - 1 - (i + j));
        }
      }
    }
    for (; i < K; ++i) {
      if ((i & 63) == 0) held = lane_offsets(loff, K - 64 - i, K);
      float x[4][V];
      const FT* __restrict__ b = frag + offset_of(held, 63 - (i & 63));
#pragma unroll
      for (int c = 0; c < 4; ++c) ldv<FT>(b, c * P + up, x[c]);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        R[v] = fmaf(T[v], x[0][v], R[v]);
        G[v] = fmaf(T[v], x[1][v], G[v]);
        B[v] = fmaf(T[v], x[2][v], B[v]);
        A[v] = fmaf(T[v], x[3][v], A[v]);
        T[v] = T[v] * (1.f - x[3][v]);
      }
      if ((a.mode & kModeKeepOrder) && act) {
#pragma unroll
        for (int v = 0; v < V; ++v)
          a.order[static_cast<size_t>(off + i) * P + p0 + v] = static_cast<uint16_t>(K - 1 - i);
      }
    }
    if (act) vs += finish_row<V, true>(a, u, q0, p0, R, G, B, A, T);
  }
  return vs;
}

// The averaging operation with 16-byte loads (layers summed in layer order;
// K > 0: a tile without renders is the background, handled by the caller).
template <typename FT>
__device__ float unit_average_vec(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff, int K) {
  constexpr int V = VecWidth<FT>::V;
  constexpr int C = DFB_OP_CHUNK;
  const int NT = blockDim.x;
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  const float inv = K > 0 ? 1.f / static_cast<float>(K) : 0.f;
  float vs = 0.f;
  // whole waves run the loop (the held offsets need every lane); lanes past
  // the unit's end load a valid row again and store nothing
  const int lane = static_cast<int>(threadIdx.x & 63);
  for (int base = static_cast<int>(threadIdx.x >> 6) * 64 * V; base < a.work_px; base += NT * V) {
    const bool act = base + lane * V < a.work_px;
    const int q0 = act ? base + lane * V : base;
    bool in0;
    const int p0 = unit_pixel(a, u, q0, in0);
    const uint32_t up = static_cast<uint32_t>(p0);
    float S[4][V];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < V; ++v) S[c][v] = 0.f;
    int l = 0;
    int64_t held = 0;
    for (; l + C <= K; l += C) {
      if ((l & 63) == 0) held = lane_offsets(loff, l, K);
      float x[C][4][V];
#pragma unroll
      for (int j = 0; j < C; ++j) {
        const FT* __restrict__ b = frag + offset_of(held, (l + j) & 63);
#pragma unroll
        for (int c = 0; c < 4; ++c) ldv<FT>(b, c * P + up, x[j][c]);
      }
#pragma unroll
      for (int j = 0; j < C; ++j)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
          for (int v = 0; v < V; ++v) S[c][v] += x[j][c][v];
    }
    for (; l < K; ++l) {
      if ((l & 63) == 0) held = lane_offsets(loff, l, K);
      float x[4][V];
      const FT* __restrict__ b = frag + offset_of(held, l & 63);
#pragma unroll
      for (int c = 0; c < 4; ++c) ldv<FT>(b, c * P + up, x[c]);
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int v = 0; v < V; ++v) S[c][v] += x[c][v];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int v = 0; v < V; ++v) S[c][v] *= inv;
    if (act) vs += finish_row<V, false>(a, u, q0, p0, S[0], S[1], S[2], S[3], nullptr);
  }
  return vs;
}

// Averaging tile operation (redundant sampling, the paper's dynamic load
// balancing): the finished pixel is the mean of the K tiles' RGBA; a tile
// with no layers shows the background.
template <typename FT>
__device__ float unit_average(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff, int K) {
  const int NT = blockDim.x;
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  const float inv = K > 0 ? 1.f / static_cast<float>(K) : 0.f;
  float vs = 0.f;
  for (int q = threadIdx.x; q < a.work_px; q += NT) {
    bool inside;
    const int p = unit_pixel(a, u, q, inside);
    const uint32_t up = static_cast<uint32_t>(p);
    float R = 0.f, G = 0.f, B = 0.f, A = 0.f;
    int l = 0;
    for (; l + 4 <= K; l += 4) {
      float v[4][4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const FT* __restrict__ b = frag + loff[l + j];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[j][c] = ldf<FT>(b, c * P + up);
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        R += v[j][0];
        G += v[j][1];
        B += v[j][2];
        A += v[j][3];
      }
    }
    for (; l < K; ++l) {
      const FT* __restrict__ b = frag + loff[l];
      R += ldf<FT>(b, up);
      G += ldf<FT>(b, P + up);
      B += ldf<FT>(b, 2 * P + up);
      A += ldf<FT>(b, 3 * P + up);
    }
    const float4 x = K > 0 ? make_float4(R * inv, G * inv, B * inv, A * inv)
                           : with_background(a, u.t, p, make_float4(0.f, 0.f, 0.f, 0.f), 1.f);
    vs += finish_px(a, u, p, inside, x);
  }
  return vs;
}

// ---------------------------------------------------------------- K > 32
// The workgroup handles G pixels at a time.  LDS holds one row per pixel:
// Kp keys (u64) and, in a second array of the same shape, Kp floats (alpha,
// later the transmittance T); and the unit's layer offsets.  Position i of a
// row is stored at i + i/16 (one pad slot per 16) and rows are
// RS = Kp*17/16 + 1 slots apart, so the fill (lanes across rows), the LDS
// sort passes (lanes along a row) and the register blocks (a lane per 16
// consecutive keys) all hit distinct banks.
//
// Lane (g, s), s < S = NT / G, owns layers s, s + S, s + 2S, ... of pixel g.
// It loads their depth, alpha and colour together at the start of the group
// (the colours of its first kBigC layers wait in registers until the walk
// has produced the weights), so one memory round trip serves the group.
//
// Sort: bitonic, every comparator min-to-lower.  Comparators closer than 16
// positions never leave a 16-key block, so each block is sorted (sizes
// 2..16) or half-cleaned (strides 8..1 of every later merge) by one lane in
// registers.  The strides >= 16 of a merge go through LDS up to four at a
// time: a lane loads the 2^m keys that m consecutive stages compare only
// among themselves, runs the m stages in registers and writes the keys
// back, one barrier per pass.  For Kp = 512 that is 6 LDS passes, not 15.
// Positions K..Kp-1 hold the padding key, which no real key exceeds; as
// every comparator is min-to-lower they keep it throughout, so blocks and
// groups that lie wholly in the padding are skipped.
//
// The walk: the S lanes of a pixel take a product scan over S chunks of the
// sorted row; then colour sums in layer order and a fixed-order reduction
// over the S lanes.
#ifndef DFB_BLK_LOG
#define DFB_BLK_LOG 4
#endif
constexpr int kBlkLog = DFB_BLK_LOG;   // keys sorted per lane in registers: 2^kBlkLog
constexpr int kBlk = 1 << kBlkLog;
// Layers per lane whose colours are loaded with the keys (held in registers
// through the sort: 16 keeps the LDS-sort kernel at 247 VGPRs, 2 waves per
// SIMD, which its LDS allows anyway; 32 drops it to one), and the most merge
// stages one LDS pass runs.
#ifndef DFB_BIG_C
#define DFB_BIG_C 16
#endif
#ifndef DFB_MAX_M
#define DFB_MAX_M 4
#endif
// Layers per lane whose depth and alpha loads are in flight together past
// the first kBigC, and layers per lane whose colour loads are in flight
// together after the walk.  On the 8192^2 heavy-tailed frame (16, 16, 8)
// takes 34.4 ms against 35.7 ms for (8, 8, 4); larger batches of depth and
// alpha past the first 8 layers were slower (24, 24: 38.0-38.1 ms).
#ifndef DFB_BIG_FILL
#define DFB_BIG_FILL 16
#endif
#ifndef DFB_BIG_COLS
#define DFB_BIG_COLS 8
#endif
constexpr int kBigFill = DFB_BIG_FILL;
constexpr int kBigCols = DFB_BIG_COLS;
constexpr int kBigC = DFB_BIG_C;

__device__ __forceinline__ int kslot(int i) { return i + (i >> 4); }

// Plane loads of the K > 32 path.
template <typename FT>
__device__ __forceinline__ float ldb(const FT* __restrict__ base, uint32_t i) {
#if DFB_BIGK_NT
  return ldf<FT>(base, i);
#else
  return static_cast<float>(base[i]);
#endif
}


// a block is read as runs of 16 keys, none of which straddles a pad slot
__device__ __forceinline__ void block_load(const uint64_t* r, int base, uint64_t (&k)[kBlk]) {
#pragma unroll
  for (int h = 0; h < kBlk / 16; ++h) {
    const uint64_t* q = r + kslot(base + 16 * h);
#pragma unroll
    for (int i = 0; i < 16; ++i) k[16 * h + i] = q[i];
  }
}
__device__ __forceinline__ void block_store(uint64_t* r, int base, const uint64_t (&k)[kBlk]) {
#pragma unroll
  for (int h = 0; h < kBlk / 16; ++h) {
    uint64_t* q = r + kslot(base + 16 * h);
#pragma unroll
    for (int i = 0; i < 16; ++i) q[i] = k[16 * h + i];
  }
}
// strides 8, 4, 2, 1 of a merge larger than the block (half-cleaners)
__device__ __forceinline__ void block_half_clean(uint64_t (&k)[kBlk]) {
#pragma unroll
  for (int str = kBlk / 2; str > 0; str >>= 1)
#pragma unroll
    for (int i = 0; i < kBlk; ++i)
      if ((i & str) == 0) KeyMinMax()(k[i], k[i + str]);
}

// One LDS pass over every row: M consecutive stages of the merge of size
// 2^ls, the first with stride 2^lt, the last with stride 2^lo (lo = lt-M+1).
// Group c of a row is the positions b + r 2^lo (r < 2^M), b being c with M
// zero bits inserted at lo..lt; these meet only each other in the M stages.
// When lt = ls - 1 the first stage is the merge's mirrored one (x against
// x ^ (2^ls - 1)) and the upper half of a group is the mirror image of its
// lower half, in increasing position order.
template <int M>
__device__ __forceinline__ void lds_stages(uint64_t* keys, int RS, int G, int lk, int ls, int lt,
                                           int K, int NT, int tid) {
  constexpr int N = 1 << M, H = N / 2, U = M >= 3 ? 1 : (M == 2 ? 2 : 4);  // groups in flight
  const int lo = lt - M + 1, glog = lk - M, total = G << glog;
  const bool mirror = lt == ls - 1;
  const int mask = (2 << lt) - 1;
  for (int e0 = tid; e0 < total; e0 += U * NT) {
    uint64_t v[U][N];
    int ix[U][N];
    bool act[U];
#pragma unroll
    for (int w = 0; w < U; ++w) {
      const int e = e0 + w * NT;
      const int g = e >> glog, c = e & ((1 << glog) - 1);
      const int b = ((c >> lo) << (lt + 1)) | (c & ((1 << lo) - 1));
      act[w] = e < total && b < K;  // b is the group's lowest position
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int pos = (mirror && r >= H) ? ((b + ((N - 1 - r) << lo)) ^ mask) : b + (r << lo);
        ix[w][r] = g * RS + kslot(pos);
        v[w][r] = act[w] ? keys[ix[w][r]] : kKeyPad;
      }
    }
#pragma unroll
    for (int w = 0; w < U; ++w) {
      if (mirror) {
#pragma unroll
        for (int r = 0; r < H; ++r) KeyMinMax()(v[w][r], v[w][N - 1 - r]);
      } else {
#pragma unroll
        for (int r = 0; r < H; ++r) KeyMinMax()(v[w][r], v[w][r + H]);
      }
#pragma unroll
      for (int k = M - 2; k >= 0; --k)
#pragma unroll
        for (int r = 0; r < N; ++r)
          if ((r & (1 << k)) == 0) KeyMinMax()(v[w][r], v[w][r | (1 << k)]);
      if (act[w]) {
#pragma unroll
        for (int r = 0; r < N; ++r) keys[ix[w][r]] = v[w][r];
      }
    }
  }
}

// G (pixels per group) for a padded layer count 2^lk and an LDS budget.
__device__ __forceinline__ int bigk_group(int lk, int budget, int NT) {
  const int RS = (1 << lk) + (1 << (lk - 4)) + 1;
  int G = budget / (RS * 12);
  G = G > NT ? NT : G;
  G = G > 64 ? 64 : G;
  while (G & (G - 1)) G &= G - 1;  // power of two
  return G;
}

template <typename FT>
__device__ float unit_bigk(const FrameArgs& a, const Unit& u, const int64_t* __restrict__ loff,
                           int K, int off, char* lds) {
  const int NT = blockDim.x, tid = threadIdx.x;
  const uint32_t P = static_cast<uint32_t>(a.P);
  const FT* __restrict__ frag = static_cast<const FT*>(a.frag);
  int lk = 6;                       // log2(Kp), Kp >= 64
  while ((1 << lk) < K) ++lk;
  const int Kp = 1 << lk;
  const int RS = Kp + (Kp >> 4) + 1;
  const int G = bigk_group(lk, a.big_lds, NT);
  int lg = 0;
  while ((1 << lg) < G) ++lg;
  const int S = NT / G;                   // lanes per pixel
  const int C = Kp / S > 0 ? Kp / S : 1;  // layers (and sorted positions) per lane
  uint64_t* keys = reinterpret_cast<uint64_t*>(lds);
  float* wv = reinterpret_cast<float*>(keys + static_cast<size_t>(G) * RS);
  float4* red = reinterpret_cast<float4*>(lds + a.big_lds);  // [NT]
  float* tend = reinterpret_cast<float*>(red + NT);           // [G], G <= 64
  int64_t* lofs = reinterpret_cast<int64_t*>(tend + 64);      // [K]
  for (int i = tid; i < K; i += NT) lofs[i] = loff[i];
  lds_barrier();
  const int gm = tid & (G - 1), sm = tid >> lg;
  const int nblk = G << (lk - kBlkLog);  // register blocks over all rows
  uint64_t* krow = keys + gm * RS;
  float* wrow = wv + gm * RS;
  float vs = 0.f;
  for (int q0 = 0; q0 < a.work_px; q0 += G) {
    const int qme = q0 + gm;
    const bool live = qme < a.work_px;
    bool in_me = false;
    const int p_me = live ? unit_pixel(a, u, qme, in_me) : 0;
    // 1. depth, alpha and colour of the lane's layers l = sm + j S, all
    //    loads issued before the first LDS store; padding keys sort last
    float cr[kBigC], cg[kBigC], cb[kBigC];
    {
      float dv[kBigC], av[kBigC];
#pragma unroll
      for (int j = 0; j < kBigC; ++j) {
        const int l = sm + j * S;
        dv[j] = 0.f;
        av[j] = 0.f;
        cr[j] = 0.f;
        cg[j] = 0.f;
        cb[j] = 0.f;
        if (j < C && live && l < K) {
          const FT* __restrict__ b = frag + lofs[l];
          dv[j] = ldb<FT>(b, 4 * P + p_me);
          av[j] = ldb<FT>(b, 3 * P + p_me);
        }
      }
#pragma unroll
      for (int j = 0; j < kBigC; ++j) {
        const int l = sm + j * S;
        if (j < C && live && l < K) {
          const FT* __restrict__ b = frag + lofs[l];
          cr[j] = ldb<FT>(b, p_me);
          cg[j] = ldb<FT>(b, P + p_me);
          cb[j] = ldb<FT>(b, 2 * P + p_me);
        }
      }
#pragma unroll
      for (int j = 0; j < kBigC; ++j) {
        const int l = sm + j * S;
        if (j < C) {
          krow[kslot(l)] = (live && l < K)
                               ? big_key(depth_bits(dv[j]), l) : kKeyPad;
          wrow[kslot(l)] = av[j];
        }
      }
    }
    for (int j0 = kBigC; j0 < C; j0 += kBigFill) {  // more layers than kBigC per lane: keys only here
      float dv[kBigFill], av[kBigFill];
#pragma unroll
      for (int j = 0; j < kBigFill; ++j) {
        const int l = sm + (j0 + j) * S;
        dv[j] = 0.f;
        av[j] = 0.f;
        if (j0 + j < C && live && l < K) {
          const FT* __restrict__ b = frag + lofs[l];
          dv[j] = ldb<FT>(b, 4 * P + p_me);
          av[j] = ldb<FT>(b, 3 * P + p_me);
        }
      }
#pragma unroll
      for (int j = 0; j < kBigFill; ++j) {
        const int l = sm + (j0 + j) * S;
        if (j0 + j < C) {
          krow[kslot(l)] = (live && l < K)
                               ? big_key(depth_bits(dv[j]), l) : kKeyPad;
          wrow[kslot(l)] = av[j];
        }
      }
    }
    lds_barrier();
    // 2. sort every row: blocks of 16 in registers first
    for (int b = tid; b < nblk; b += NT) {
      uint64_t k[kBlk];
      uint64_t* r = keys + (b >> (lk - kBlkLog)) * RS;
      const int base = (b & ((1 << (lk - kBlkLog)) - 1)) * kBlk;
      if (base < K) {
        block_load(r, base, k);
        sort_network<kBlk>(k, KeyMinMax());
        block_store(r, base, k);
      }
    }
    lds_barrier();
    for (int ls = kBlkLog + 1; ls <= lk; ++ls) {  // merge size 2^ls
      for (int lt = ls - 1; lt >= kBlkLog;) {     // strides >= kBlk through LDS
        const int m = lt - kBlkLog + 1 >= DFB_MAX_M ? DFB_MAX_M : lt - kBlkLog + 1;
        if (m == 4) lds_stages<4>(keys, RS, G, lk, ls, lt, K, NT, tid);
        else if (m == 3) lds_stages<3>(keys, RS, G, lk, ls, lt, K, NT, tid);
        else if (m == 2) lds_stages<2>(keys, RS, G, lk, ls, lt, K, NT, tid);
        else lds_stages<1>(keys, RS, G, lk, ls, lt, K, NT, tid);
        lt -= m;
        lds_barrier();
      }
      for (int b = tid; b < nblk; b += NT) {     // strides 8..1 in registers
        uint64_t k[kBlk];
        uint64_t* r = keys + (b >> (lk - kBlkLog)) * RS;
        const int base = (b & ((1 << (lk - kBlkLog)) - 1)) * kBlk;
        if (base < K) {
          block_load(r, base, k);
          block_half_clean(k);
          block_store(r, base, k);
        }
      }
      lds_barrier();
    }
    // 3. front-to-back walk: chunk products, exclusive scan over the S chunks.
    //    Rows past the unit's last pixel hold only padding keys: skipped.
    const int i0 = sm * C, i1 = live ? ((i0 + C < K) ? i0 + C : K) : 0;
    float prod = 1.f;
#pragma unroll 8
    for (int i = i0; i < i1; ++i) {
      const int l = key_layer(krow[kslot(i)]);
      prod = prod * (1.f - wrow[kslot(l)]);
    }
    red[tid].x = prod;
    lds_barrier();
    float T = 1.f;
    for (int s2 = 0; s2 < sm; ++s2) T = T * red[s2 * G + gm].x;
    lds_barrier();
    float Ap = 0.f;
#pragma unroll 4
    for (int i = i0; i < i1; ++i) {
      const int l = key_layer(krow[kslot(i)]);
      const float al = wrow[kslot(l)];
      wrow[kslot(l)] = T;
      Ap = fmaf(T, al, Ap);
      T = T * (1.f - al);
      if (a.mode & kModeKeepOrder)
        a.order[static_cast<size_t>(off + i) * P + p_me] = static_cast<uint16_t>(l);
    }
    lds_barrier();
    // 4. colour sums in layer order: T_l * c_l
    float R = 0.f, Gc = 0.f, B = 0.f;
    int sm4 = sm;
    asm volatile("" : "+v"(sm4));  // addresses are recomputed here, not kept across the sort
    if (live) {
#pragma unroll
      for (int j = 0; j < kBigC; ++j) {
        const int l = sm4 + j * S;
        if (j < C && l < K) {
          const float w = wrow[kslot(l)];
          R = fmaf(w, cr[j], R);
          Gc = fmaf(w, cg[j], Gc);
          B = fmaf(w, cb[j], B);
        }
      }
      int l = sm4 + kBigC * S;
      for (; l + (kBigCols - 1) * S < K; l += kBigCols * S) {
        float w[kBigCols], r4[kBigCols], g4[kBigCols], b4[kBigCols];
#pragma unroll
        for (int j = 0; j < kBigCols; ++j) {
          const FT* __restrict__ b = frag + lofs[l + j * S];
          w[j] = wrow[kslot(l + j * S)];
          r4[j] = ldb<FT>(b, p_me);
          g4[j] = ldb<FT>(b, P + p_me);
          b4[j] = ldb<FT>(b, 2 * P + p_me);
        }
#pragma unroll
        for (int j = 0; j < kBigCols; ++j) {
          R = fmaf(w[j], r4[j], R);
          Gc = fmaf(w[j], g4[j], Gc);
          B = fmaf(w[j], b4[j], B);
        }
      }
      for (; l < K; l += S) {
        const FT* __restrict__ b = frag + lofs[l];
        const float w = wrow[kslot(l)];
        R = fmaf(w, ldb<FT>(b, p_me), R);
        Gc = fmaf(w, ldb<FT>(b, P + p_me), Gc);
        B = fmaf(w, ldb<FT>(b, 2 * P + p_me), B);
      }
    }
    // lanes whose chunk is the last non-empty one hold the final T
    const int last = (K - 1) / C;
    red[tid] = make_float4(R, Gc, B, Ap);
    if (sm == last) tend[gm] = T;
    lds_barrier();
    if (sm == 0 && live) {
      float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
      for (int s2 = 0; s2 < S; ++s2) {
        const float4 v = red[s2 * G + gm];
        acc.x += v.x;
        acc.y += v.y;
        acc.z += v.z;
        acc.w += v.w;
      }
      vs += finish_px(a, u, p_me, in_me, with_background(a, u.t, p_me, acc, tend[gm]));
    }
    lds_barrier();
  }
  return vs;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float variance_of_mean(float sum, int inside_px, int n) {
  if (n < 2) return __int_as_float(0x7f800000);
  return sum / (3.f * static_cast<float>(inside_px) * static_cast<float>(n) *
                static_cast<float>(n - 1));
}

// Work queue.  The work list is cut into blocks of B = queue_block
// consecutive positions (the units of one tile); counter s (of S = n_queues)
// holds the blocks congruent to s, in order.  Workgroup b starts on counter
// b mod S, and its first unit there is its rank r = b / S among those
// workgroups (no atomic).  Each ticket c of a counter names its unit g + c,
// g being the number of workgroups that start on it.  Lane 0 of wave 0
// takes the next ticket at the start of a unit and the result is read at
// its end, so the atomic's latency hides behind the unit's work.  A drained
// counter sends the workgroup on to the next one (s + 1, s + 2, ... mod S);
// a coherent read skips counters that are already drained without an
// atomic.  Workgroups are dealt to the 8 XCDs in turn and S is a multiple of
// 8 on every grid of 8 workgroups or more, so the units of one tile run at
// about the same time under one XCD's L2: unit rows that share cache lines
// (fp16 planes, units narrower than a line) are fetched from memory once.
struct Queue {
  uint32_t* ctr;
  int s, g, n;  // counter, workgroups starting on it, units it holds
};

__device__ __forceinline__ Queue queue_of(const FrameArgs& a, int s) {
  const int S = a.n_queues, B = a.queue_block;
  const int nb = (a.n_work + B - 1) / B;  // blocks
  const int cnt = s < nb ? (nb - s + S - 1) / S : 0;
  Queue q;
  q.s = s;
  q.g = (static_cast<int>(gridDim.x) - s + S - 1) / S;
  q.n = cnt * B;
  if (cnt > 0 && s + (cnt - 1) * S == nb - 1 && a.n_work % B) q.n -= B - a.n_work % B;  // partial last block
  q.ctr = a.queue + static_cast<size_t>(s) * kQueueStride + a.slot;
  return q;
}

// Work-list position of the j-th unit of a counter (j < q.n).
__device__ __forceinline__ int unit_at(const FrameArgs& a, const Queue& q, int j) {
  const int B = a.queue_block;
  return ((j / B) * a.n_queues + q.s) * B + j % B;
}

__device__ __forceinline__ uint32_t take_ticket(const Queue& q) {
  uint32_t v = 0;
  if (__lane_id() == 0) v = atomicAdd(q.ctr, 1u);
  return v;
}

__device__ __forceinline__ int ticket_to_unit(const FrameArgs& a, const Queue& q, uint32_t v) {
  const int64_t j = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(v)) + q.g;
  return j < q.n ? unit_at(a, q, static_cast<int>(j)) : a.n_work;
}

// Whether a counter may still hand out a unit (never wrong the other way:
// counters only grow within a frame).
__device__ __forceinline__ bool queue_open(const Queue& q) {
  uint32_t v = 0;
  if (__lane_id() == 0) v = __hip_atomic_load(q.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return static_cast<int64_t>(__builtin_amdgcn_readfirstlane(v)) + q.g < q.n;
}

// A unit's M2 sum (all waves) -> var_partial[w].  Runs on all lanes of wave
// 0; the combine into per-tile values is a separate kernel (no fences here).
__device__ __forceinline__ void store_partial(const FrameArgs& a, int w, const float* s_red,
                                              int n_waves) {
  float sum = 0.f;
  for (int i = 0; i < 4; ++i)
    if (i < n_waves) sum += s_red[i];
  if (__lane_id() == 0) a.var_partial[w] = sum;
}

// The persistent frame kernel.  Control flow that contains barriers is
// uniform across the workgroup; code that only lane 0 runs is a single
// store or atomic, so no lane can be left behind in a loop that holds a
// barrier.
#ifndef DFB_WAVES_F16_K32
#define DFB_WAVES_F16_K32 0
#endif
constexpr int min_waves(int kcap, bool half) {
  return kcap <= 8 ? (DFB_WAVES_K8 > 0 ? DFB_WAVES_K8 : 1)
                   : kcap <= 16 ? (DFB_WAVES_K16 > 0 ? DFB_WAVES_K16 : 1)
                                : (half && DFB_WAVES_F16_K32 > 0 ? DFB_WAVES_F16_K32
                                                                 : (DFB_WAVES_K32 > 0 ? DFB_WAVES_K32 : 1));
}

__device__ __forceinline__ uint32_t* finish_counters(const FrameArgs& a) {
  return a.queue + static_cast<size_t>(kQueues) * kQueueStride;
}
__device__ __forceinline__ FrameState* frame_state(const FrameArgs& a) { return a.state; }

// The frame's sequence number and accumulation count, read once per
// workgroup from the device state and shared through LDS.  The load's value
// is stored to LDS before the barrier, so it has returned before anything
// else of the workgroup runs; the last workgroup to finish advances the
// state only after every workgroup has counted itself finished, hence after
// every read of this frame.
__device__ __forceinline__ uint32_t read_frame_state(FrameArgs& a, uint32_t* s_state) {
  if (threadIdx.x == 0) {
    const FrameState* st = frame_state(a);
    s_state[0] = __hip_atomic_load(&st->seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_state[1] = static_cast<uint32_t>(__hip_atomic_load(&st->n_acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
  lds_barrier();
  const uint32_t seq = __builtin_amdgcn_readfirstlane(s_state[0]);
  const int n_prev = static_cast<int>(__builtin_amdgcn_readfirstlane(s_state[1]));
  a.slot = static_cast<int32_t>(seq % kSlots);
  a.clear_slot = static_cast<int32_t>((seq + kSlots / 2) % kSlots);
  a.n_acc = (a.mode & kModeAccumulate) ? n_prev + 1 : n_prev;
  a.inv_n = a.n_acc > 0 ? 1.f / static_cast<float>(a.n_acc) : 1.f;
  return seq;
}

// KCAP 8, 16, 32: register-sort capacity (tiles with more layers are the
// KCAP 0 launch's); KCAP 0: only the tiles with more than kRegMax layers.
template <typename FT, int KCAP, int OP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(min_waves(KCAP, sizeof(FT) == 2))))
frame_kernel_t(FrameArgs args, const int32_t* __restrict__ tile_off,
               const int64_t* __restrict__ layer_off, const int32_t* __restrict__ work_list) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int s_item;
  __shared__ float s_red[4];
  __shared__ uint32_t s_state[2];
  const int tid = threadIdx.x;
  const int n_waves = static_cast<int>(blockDim.x >> 6);
  const bool wave0 = __builtin_amdgcn_readfirstlane(tid) < 64;  // uniform per wave
  FrameArgs a = args;
  const uint32_t seq = read_frame_state(a, s_state);
  if (blockIdx.x == 0 && tid <= kQueues)  // recycle the slot of the frame kSlots/2 ahead (counters, finish count)
    __hip_atomic_store(a.queue + static_cast<size_t>(tid) * kQueueStride + a.clear_slot, 0u, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  const int home = static_cast<int>(blockIdx.x) % a.n_queues;
  Queue q = queue_of(a, home);
  int drained = 0;  // counters this workgroup has found empty
  const int r = static_cast<int>(blockIdx.x) / a.n_queues;
  int it = r < q.n ? unit_at(a, q, r) : a.n_work;  // the first unit is static
  while (it < a.n_work) {
    // the next unit's ticket is taken now and read after this unit's work
    const uint32_t next = wave0 ? take_ticket(q) : 0u;
    const int w = work_list ? work_list[it] : it;
    Unit u;
    u.t = w / a.subs_per_tile;
    const int s = w - u.t * a.subs_per_tile;
    u.sy0 = (s / a.subs_x) * a.work_h;
    u.sx0 = (s - (s / a.subs_x) * a.subs_x) * a.work_w;
    u.y0 = (u.t / a.tiles_x) * a.tile_h;
    u.x0 = (u.t - (u.t / a.tiles_x) * a.tiles_x) * a.tile_w;
    const int off = tile_off[u.t];
    const int K = tile_off[u.t + 1] - off;
    const int64_t* __restrict__ blk = layer_off + off;
    float* wl = reinterpret_cast<float*>(lds);
    float vs = 0.f;
    bool mine = true;  // uniform: this launch composites the unit
    if constexpr (KCAP == 0) {
      mine = K > kRegMax;
      if (mine) vs = unit_bigk<FT>(a, u, blk, K, off, lds);
    } else if constexpr (OP == DFB_OP_AVERAGE) {
      vs = (a.vec_ok && K > 0) ? unit_average_vec<FT>(a, u, blk, K) : unit_average<FT>(a, u, blk, K);
    } else if constexpr (OP == DFB_OP_LIST) {
      vs = K == 0 ? unit_background(a, u)
                  : (a.vec_ok ? unit_list_vec<FT>(a, u, blk, K, off) : unit_list<FT>(a, u, blk, K, off));
    } else {
    mine = K <= KCAP;
    if (K == 0) vs = unit_background(a, u);
    else if (K <= 1) vs = unit_reg<FT, 1, KCAP>(a, u, blk, K, off, wl);
    else if (K <= 2) vs = unit_reg<FT, 2, KCAP>(a, u, blk, K, off, wl);
    else if (K <= 3) vs = unit_reg<FT, 3, KCAP>(a, u, blk, K, off, wl);
    else if (K <= 4) vs = unit_reg<FT, 4, KCAP>(a, u, blk, K, off, wl);
    else if (K <= 6) vs = unit_reg<FT, 6, KCAP>(a, u, blk, K, off, wl);
    else if (K <= 8) vs = unit_reg<FT, 8, KCAP>(a, u, blk, K, off, wl);
    else if constexpr (KCAP >= 16) {
      // the kernel of a frame whose tiles have at most KCAP layers carries
      // no code for more: K <= KCAP here (the host picks KCAP >= the
      // frame's largest tile)
      if (K <= 12) vs = unit_reg<FT, 12, KCAP>(a, u, blk, K, off, wl);
      else if (KCAP == 16 || K <= 16) vs = unit_reg<FT, 16, KCAP>(a, u, blk, K, off, wl);
      else if constexpr (KCAP >= 32) {
        if (K <= 24) vs = unit_reg<FT, 24, KCAP>(a, u, blk, K, off, wl);
        else if (K <= 32) vs = unit_reg<FT, 32, KCAP>(a, u, blk, K, off, wl);
      }
    }
    }
    const bool acc = (a.mode & kModeAccumulate) != 0 && mine;
    if (acc) {
      vs = wave_sum(vs);  // fixed-order reductions only: deterministic
      if ((tid & 63) == 0) s_red[tid >> 6] = vs;
    }
    lds_barrier();  // s_red complete; every lane has read s_item
    if (wave0) {
      if (acc) store_partial(a, w, s_red, n_waves);
      int v = ticket_to_unit(a, q, next);
      while (v == a.n_work && ++drained < a.n_queues) {  // move on to the next counter
        q = queue_of(a, (home + drained) % a.n_queues);
        if (queue_open(q)) v = ticket_to_unit(a, q, take_ticket(q));
      }
      if (__lane_id() == 0) s_item = v;
    }
    lds_barrier();
    it = __builtin_amdgcn_readfirstlane(s_item);
  }
  // Count this workgroup finished; the last one advances the frame state
  // for the next launch (sequence number, and the accumulation count of an
  // accumulating frame).  Every queue access of this workgroup has returned
  // its value before this point.
  uint32_t done = 0;
  if (tid == 0)
    done = __hip_atomic_fetch_add(finish_counters(a) + a.slot, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  done = __builtin_amdgcn_readfirstlane(done);
  const bool last = a.advance && wave0 && done == gridDim.x - 1;
  if (last && tid == 0)
    __hip_atomic_store(&frame_state(a)->seq, seq + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (last && tid == 0 && (a.mode & kModeAccumulate))
    __hip_atomic_store(&frame_state(a)->n_acc, a.n_acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Per-tile variance of the mean from the units' partial M2 sums, added in
// unit order (deterministic): one thread per tile.
__global__ void __launch_bounds__(256) tile_variance_kernel_t(VarianceArgs a) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= a.n_tiles) return;
  float sum = 0.f;
  for (int i = 0; i < a.subs_per_tile; ++i) sum += a.var_partial[t * a.subs_per_tile + i];
  const int x0 = (t % a.tiles_x) * a.tile_w, y0 = (t / a.tiles_x) * a.tile_h;
  const int wx = a.width - x0, wy = a.height - y0;
  const int inside = (wx < a.tile_w ? wx : a.tile_w) * (wy < a.tile_h ? wy : a.tile_h);
  a.tile_var[t] = variance_of_mean(sum, inside, a.state->n_acc);
}

// Unfused accumulation of the stored finished tiles: one workgroup per tile.
__global__ void __launch_bounds__(256) accumulate_kernel_t(AccumArgs a) {
  __shared__ float s_red[4];
  const int t = blockIdx.x, tid = threadIdx.x;
  const int n_acc = a.state->n_acc + 1;  // the state kernel after this launch advances it
  const float inv_n = 1.f / static_cast<float>(n_acc);
  const int x0 = (t % a.tiles_x) * a.tile_w, y0 = (t / a.tiles_x) * a.tile_h;
  float vs = 0.f;
  for (int p = tid; p < a.P; p += blockDim.x) {
    const int py = p / a.tile_w, pxl = p - py * a.tile_w;
    const bool inside = (x0 + pxl < a.width) && (y0 + py < a.height);
    const size_t px = static_cast<size_t>(t) * a.P + p;
    const float4 x = reinterpret_cast<const float4*>(a.finished)[px];
    vs += store_pixel(x, px, static_cast<size_t>(t) * 3 * a.P + p, a.P, inside,
                      (a.mode & ~kModeKeepFinished) | kModeAccumulate, n_acc, inv_n,
                      a.inv_gamma, nullptr, a.accum, a.m2, a.final_out);
  }
  vs = wave_sum(vs);
  if ((tid & 63) == 0) s_red[tid >> 6] = vs;
  lds_barrier();
  if (__builtin_amdgcn_readfirstlane(tid) < 64) {
    const int n_waves = static_cast<int>(blockDim.x >> 6);
    float sum = 0.f;
    for (int i = 0; i < 4; ++i)
      if (i < n_waves) sum += s_red[i];
    const int wx = a.width - x0, wy = a.height - y0;
    const int inside = (wx < a.tile_w ? wx : a.tile_w) * (wy < a.tile_h ? wy : a.tile_h);
    if (__lane_id() == 0) a.tile_var[t] = variance_of_mean(sum, inside, n_acc);
  }
}

// Accumulation count of a handle's frame state, set (value >= 0) or advanced
// by one (value < 0), stream-ordered with the frames around it.
__global__ void state_kernel_t(FrameState* st, int32_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) st->n_acc = value >= 0 ? value : st->n_acc + 1;
}

// n words of p set to v (grid-stride).
__global__ void fill_u32_kernel_t(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

// Longest-first work list on the device, from the per-tile CSR offsets:
// a counting sort of the tiles by layer count, descending (one workgroup of
// kLptThreads lanes; equal counts in any order, which changes only the
// order units are taken in, never a result), then every tile's units in
// order.  work[pos * subs + u] = t * subs + u for the tile t at sorted
// position pos.
constexpr int kLptBins = kMaxLayers + 1;                                // K = 0 .. kMaxLayers
constexpr int kLptPer = (kLptBins + kLptThreads - 1) / kLptThreads;    // bins per lane in the scan
__global__ void __launch_bounds__(kLptThreads) lpt_work_kernel_t(const int32_t* __restrict__ tile_off,
                                                                 int32_t n_tiles, int32_t subs,
                                                                 int32_t* __restrict__ work) {
  __shared__ int32_t cnt[kLptBins];     // bin j holds layer count K = kMaxLayers - j
  __shared__ int32_t wave_tot[kLptThreads / 64];
  const int tid = threadIdx.x;
  for (int j = tid; j < kLptBins; j += kLptThreads) cnt[j] = 0;
  __syncthreads();
  for (int t = tid; t < n_tiles; t += kLptThreads) {
    int K = tile_off[t + 1] - tile_off[t];
    K = K < 0 ? 0 : (K > kMaxLayers ? kMaxLayers : K);
    atomicAdd(&cnt[kMaxLayers - K], 1);
  }
  __syncthreads();
  // exclusive scan of the bins: each lane sums kLptPer consecutive bins,
  // the lane sums are scanned within waves and across the waves
  int local[kLptPer];
  int sum = 0;
#pragma unroll
  for (int i = 0; i < kLptPer; ++i) {
    const int j = tid * kLptPer + i;
    local[i] = j < kLptBins ? cnt[j] : 0;
    sum += local[i];
  }
  int incl = sum;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if ((tid & 63) >= o) incl += v;
  }
  if ((tid & 63) == 63) wave_tot[tid >> 6] = incl;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < (tid >> 6); ++w) base += wave_tot[w];
  int run = base + incl - sum;   // exclusive prefix of this lane's first bin
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kLptPer; ++i) {
    const int j = tid * kLptPer + i;
    if (j < kLptBins) cnt[j] = run;
    run += local[i];
  }
  __syncthreads();
  for (int t = tid; t < n_tiles; t += kLptThreads) {
    int K = tile_off[t + 1] - tile_off[t];
    K = K < 0 ? 0 : (K > kMaxLayers ? kMaxLayers : K);
    const int pos = atomicAdd(&cnt[kMaxLayers - K], 1);
    for (int u = 0; u < subs; ++u) work[static_cast<int64_t>(pos) * subs + u] = t * subs + u;
  }
}

// NaN scan of every layer's depth plane: one workgroup per layer.
template <typename FT>
__global__ void __launch_bounds__(256) validate_kernel_t(ValidateArgs a) {
  const int l = blockIdx.x;
  if (l >= a.n_layers) return;
  const FT* __restrict__ b = static_cast<const FT*>(a.frag) + a.layer_off[l];
  bool bad = false;
  for (int p = threadIdx.x; p < a.P; p += blockDim.x) {
    const float d = ldf<FT>(b, 4 * static_cast<uint32_t>(a.P) + p);
    bad |= (d != d);
  }
  if (bad) atomicOr(a.bad, 1u);
}

}  // namespace

const void* frame_kernel(int dtype, int kcap, int op) {
  if (kcap == 0)
    return dtype == 0 ? reinterpret_cast<const void*>(&frame_kernel_t<float, 0, 0>)
                      : reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 0, 0>);
  if (dtype == 0) {
    if (op == DFB_OP_LIST) return reinterpret_cast<const void*>(&frame_kernel_t<float, 8, DFB_OP_LIST>);
    if (op == DFB_OP_AVERAGE) return reinterpret_cast<const void*>(&frame_kernel_t<float, 8, DFB_OP_AVERAGE>);
    if (kcap <= 8) return reinterpret_cast<const void*>(&frame_kernel_t<float, 8, 0>);
    if (kcap <= 16) return reinterpret_cast<const void*>(&frame_kernel_t<float, 16, 0>);
    return reinterpret_cast<const void*>(&frame_kernel_t<float, 32, 0>);
  }
  if (op == DFB_OP_LIST) return reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 8, DFB_OP_LIST>);
  if (op == DFB_OP_AVERAGE) return reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 8, DFB_OP_AVERAGE>);
  if (kcap <= 8) return reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 8, 0>);
  if (kcap <= 16) return reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 16, 0>);
  return reinterpret_cast<const void*>(&frame_kernel_t<_Float16, 32, 0>);
}

const void* accumulate_kernel() { return reinterpret_cast<const void*>(&accumulate_kernel_t); }

const void* tile_variance_kernel() { return reinterpret_cast<const void*>(&tile_variance_kernel_t); }

const void* state_kernel() { return reinterpret_cast<const void*>(&state_kernel_t); }

const void* fill_u32_kernel() { return reinterpret_cast<const void*>(&fill_u32_kernel_t); }

const void* lpt_work_kernel() { return reinterpret_cast<const void*>(&lpt_work_kernel_t); }

const void* validate_kernel(int dtype) {
  return dtype == 0 ? reinterpret_cast<const void*>(&validate_kernel_t<float>)
                    : reinterpret_cast<const void*>(&validate_kernel_t<_Float16>);
}

int big_lds_bytes(int max_layers) {
  // 16 pixels per group at 512 padded layers needs 16 * 545 * 12 bytes
  return max_layers > 256 ? kBigLdsBytes : (max_layers > 128 ? 96 * 1024 : 64 * 1024);
}

size_t frame_lds_bytes(int kcap, int threads, int max_layers, int big_lds) {
  if (kcap > 0) return static_cast<size_t>(kcap) * threads * sizeof(float);  // the walk's alpha / T columns
  // keys + alpha, the reduction rows [threads] float4, T_end [64], layer offsets [max_layers]
  return big_lds + static_cast<size_t>(threads) * 16 + 64 * 4 + static_cast<size_t>(max_layers) * 8;
}

}  // namespace dfb
