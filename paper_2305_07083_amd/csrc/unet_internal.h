// Internal interface between the denoiser runtime (unet_runtime.hip) and its
// gfx950 kernels (unet_kernels.hip).  Not part of the C ABI.
//
// Layouts: activations NHWC; bf16 maps are stored as uint16 bit patterns;
// a map may be a channel slice of a wider buffer (row stride `ld`, first
// channel `off`).  conv3x3 weights (f32 master) are [3][3][ci][co]; the
// kernels read two bf16 copies: fwd [9][co][ci] and dgrad [9][ci][co].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dfb_internal.h"

namespace dfb {
namespace unet {

struct Map {          // bf16 NHWC map (or a channel slice of one)
  uint16_t* p;
  int ld, off, c;     // row stride (channels), first channel, channels
};
struct MapF {         // f32 NHWC map
  float* p;
  int ld, off, c;
};
struct Shape {
  int n, h, w;        // batch, height, width
  __host__ __device__ long long pixels() const { return static_cast<long long>(n) * h * w; }
};

// y = bf16(relu(conv3x3(x') + b)) at the output shape s, where x' = x, or
// with `up` the nearest-neighbour 2x up-sampling of x (x at s/2).  x channels
// must be a multiple of 8; s.h and s.w even with `up` or `pool`.  With `pool`,
// also pool = bf16(2x2 average of y) at s/2.  With `x2`, the input is the
// channel concatenation of x and x2 (x.c a multiple of 32, x2.ld == x.ld):
// two maps that are each written with full 64- or 128-byte pixel rows.
hipError_t conv3x3_fwd(const Map& x, const uint16_t* w_fwd, const float* bias, const Map& y,
                       const Shape& s, hipStream_t st, bool up = false, const Map* pool = nullptr,
                       const Map* x2 = nullptr);
// g = bf16(dy * (y > 0)), the ReLU-gated output gradient (g.c == dy.c, a
// multiple of 8 dividing 2048; rows and offsets of y and g multiples of 8),
// and db[c] = sum_p dy*(y>0) in f32.  `partial` needs conv3x3_wgrad_scratch
// floats.
hipError_t conv3x3_gate(const MapF& dy, const Map& y, const Map& g, float* db, float* partial, const Shape& s,
                        hipStream_t st);
// dx = conv3x3^T(g) (overwrites dx).
hipError_t conv3x3_dgrad(const Map& g, const uint16_t* w_dgrad, const MapF& dx, const Shape& s, hipStream_t st);
// dw[9][ci][co] = sum_p x[p + tap] * g[p] for ci < ci_out (ci_out < x.c when
// x carries zero padding channels).  `partial` needs conv3x3_wgrad_scratch
// floats; g's row stride and offset are multiples of 4 elements.
hipError_t conv3x3_wgrad(const Map& x, const Map& g, float* dw, float* partial, const Shape& s, hipStream_t st,
                         int ci_out);
size_t conv3x3_wgrad_scratch(int ci, int co, const Shape& s);

hipError_t avgpool2(const Map& x, const Map& y, const Shape& s_in, hipStream_t st);
hipError_t avgpool2_backward_add(const MapF& dy, const MapF& dx, const Shape& s_in, hipStream_t st);
hipError_t upsample2(const Map& x, const Map& y, const Shape& s_in, hipStream_t st);
hipError_t upsample2_backward(const MapF& dy, const MapF& dx, const Shape& s_in, hipStream_t st);
hipError_t add_into(const MapF& src, const MapF& dst, const Shape& s, hipStream_t st);

// The first conv3x3 (8 input channels -> 32, ReLU, bf16) with the nine
// taps packed into a 72-deep contraction, reading the packed bf16 input x
// (x.c == 8).
hipError_t conv3x3_in_fwd(const Map& x, const uint16_t* w_fwd, const float* bias, const Map& y, const Shape& s,
                          hipStream_t st);
// out[p][c] = base[p][c] + b[c] + sum_i x[p][i] w[i][c]   (c < 3, f32)
hipError_t out_conv_fwd(const Map& x, const float* w, const float* b, const float* base,
                        int base_ld, float* out, const Shape& s, hipStream_t st);
// dout = 2 (out - target) / count; loss partial sums; dx = dout w^T; dw, db.
hipError_t out_conv_backward(const Map& x, const float* out, const float* target, const float* w,
                             const MapF& dx, float* dw, float* db, float* loss, float* partial,
                             const Shape& s, hipStream_t st);
size_t out_conv_scratch(const Shape& s);

// bf16 input [p][8] from f32 [p][in_ld] (first 6 channels), channels 6,7 zero.
hipError_t pack_input(const float* in, int in_ld, uint16_t* x, const Shape& s, hipStream_t st);

// Adam over a flat f32 parameter vector, then refresh the bf16 weight copies.
hipError_t adam_update(float* w, const float* g, float* m, float* v, long long n, float lr,
                       float beta1, float beta2, float eps, float c1, float c2, hipStream_t st);
hipError_t refresh_bf16(const float* w_master, uint16_t* w_fwd, uint16_t* w_dgrad, int ci, int co,
                        hipStream_t st);

// Compositor glue: NHWC denoiser input from tile-major mean / tile variance.
using dfb::FrameGlue;
hipError_t frame_to_input(const FrameGlue& g, float* in6, hipStream_t st);
// conv3x3_in_fwd reading that input straight from the frame (one image of
// the frame's size), without materialising it.
hipError_t conv3x3_in_frame(const FrameGlue& g, const uint16_t* w_fwd, const float* bias, const Map& y,
                            const Shape& s, hipStream_t st);
// The last conv3x3 (32 -> 32, ReLU, bf16) fused with the output conv and
// written into the frame: with out[p][c] = mean[p][c] + ob[c] + sum_i y[p][i]
// ow[i][c] (y the conv's bf16 output, not stored), den[e] = (out, mean
// alpha), or the mean where the tile falls back
// (n >= 2 and variance > tau); padding pixels of ragged edge tiles get the
// mean; then the display value of every pixel in final_out by mode
// (kModeFmtRGBA8 / kModeFmtF32, kModeGamma).  den is required; final_out
// when mode has a format.
hipError_t conv3x3_out_frame(const Map& x, const uint16_t* w_fwd, const float* bias, const float* ow, const float* ob,
                             const FrameGlue& g, float tau, float* den, void* final_out, uint32_t mode,
                             float inv_gamma, const Shape& s, hipStream_t st);

}  // namespace unet
}  // namespace dfb
