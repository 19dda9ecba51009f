// Host runtime of include/dfb_denoise.h: parameters, buffers and the order
// of the denoiser's kernels for the forward pass, the backward pass and Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/dfb_denoise.h"
#include "dfb_internal.h"
#include "unet_internal.h"

using dfb::unet::Map;
using dfb::unet::MapF;
using dfb::unet::Shape;

namespace {

struct Conv {
  const char* name;
  int ci, co;
  int level;  // resolution of the output: 0 full, 1 half, 2 quarter
};
// the network (same order as the parameter layout)
const Conv kConv[12] = {
    {"enc1a", 6, 32, 0},   {"enc1b", 32, 32, 0},  {"enc2a", 32, 64, 1},  {"enc2b", 64, 64, 1},
    {"enc3a", 64, 128, 2}, {"enc3b", 128, 128, 2}, {"up2", 128, 64, 1},  {"dec2a", 128, 64, 1},
    {"dec2b", 64, 64, 1},  {"up1", 64, 32, 0},    {"dec1a", 64, 32, 0},  {"dec1b", 32, 32, 0},
};
enum { ENC1A, ENC1B, ENC2A, ENC2B, ENC3A, ENC3B, UP2, DEC2A, DEC2B, UP1, DEC1A, DEC1B };

int64_t param_count() {
  int64_t n = 0;
  for (const Conv& c : kConv) n += 9LL * c.ci * c.co + c.co;
  return n + 32 * 3 + 3;
}

std::string g_err;

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
double normal(uint64_t& s) {  // Box-Muller
  const double u1 = (static_cast<double>(splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = (static_cast<double>(splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
}

}  // namespace

struct dfb_denoiser_ctx {
  dfb_unet_config cfg{};
  hipStream_t stream = nullptr;
  std::string err;
  bool sticky = false;
  int64_t n_params = 0;
  int64_t off_w[12], off_b[12], off_ow, off_ob;
  float* w = nullptr;   // master parameters
  float* g = nullptr;   // gradients
  float* m = nullptr;   // Adam
  float* v = nullptr;
  uint16_t* wf[12] = {};  // bf16 forward copies [9][co][ci_pad]
  uint16_t* wd[12] = {};  // bf16 dgrad copies [9][ci_pad][co]
  int step = 0;
  // activations (bf16) at the maximum size
  int64_t P0 = 0;
  uint16_t *xin = nullptr, *e1a = nullptr, *cat1 = nullptr, *pool1 = nullptr, *e2a = nullptr, *cat2 = nullptr,
           *pool2 = nullptr, *e3a = nullptr, *e3b = nullptr, *up3 = nullptr, *d2a = nullptr, *d2b = nullptr,
           *upd2 = nullptr, *d1a = nullptr, *d1b = nullptr;
  float* out = nullptr;  // [P0][3] network output of the last forward
  // gradients (f32)
  float *g_d1b = nullptr, *g_d1a = nullptr, *g_cat1 = nullptr, *g_upd2 = nullptr, *g_d2b = nullptr,
        *g_d2a = nullptr, *g_cat2 = nullptr, *g_up3 = nullptr, *g_e3b = nullptr, *g_e3a = nullptr,
        *g_pool2 = nullptr, *g_e2a = nullptr, *g_pool1 = nullptr, *g_e1a = nullptr;
  float* scratch = nullptr;
  size_t scratch_n = 0;
  uint16_t* gate = nullptr;  // gated output gradient of the layer in the backward pass (bf16)
  float* loss_dev = nullptr;
  Shape last{0, 0, 0};
  bool planar = false;  // the last forward kept the skip concatenations as separate maps
  bool lean = false;    // the last forward fused the output conv and did not store dec1b
  std::vector<void*> allocs;
};

namespace {

dfb_status nfail(dfb_denoiser_ctx* n, dfb_status s, const std::string& msg) {
  if (n) n->err = msg;
  else g_err = msg;
  return s;
}

#define NHIP(n, call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (n)->sticky = true;                                                      \
      return nfail((n), DFB_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    }                                                                          \
  } while (0)

template <typename T>
dfb_status dalloc(dfb_denoiser_ctx* n, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    return nfail(n, DFB_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed");
  }
  n->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return DFB_OK;
}

Map mp(uint16_t* p, int ld, int off, int c) { return Map{p, ld, off, c}; }
MapF mf(float* p, int ld, int off, int c) { return MapF{p, ld, off, c}; }

dfb_status check_shape(dfb_denoiser_ctx* n, int32_t b, int32_t h, int32_t w) {
  if (b <= 0 || h <= 0 || w <= 0 || h % 4 || w % 4)
    return nfail(n, DFB_ERR_INVALID_ARG, "batch, height, width must be positive; height, width multiples of 4");
  if (static_cast<int64_t>(b) * h * w > n->P0)
    return nfail(n, DFB_ERR_INVALID_ARG, "n*h*w exceeds the configured max_pixels");
  return DFB_OK;
}

dfb_status refresh(dfb_denoiser_ctx* n) {
  for (int i = 0; i < 12; ++i)
    NHIP(n, dfb::unet::refresh_bf16(n->w + n->off_w[i], n->wf[i], n->wd[i], kConv[i].ci, kConv[i].co, n->stream));
  return DFB_OK;
}

// Where the halves of the two skip concatenations live.  Training keeps
// each concatenation interleaved per pixel (cat1 [p][64], cat2 [p][128]), as
// the backward pass reads it; inference stores each half as a map of its own
// inside the same allocation (cat1: [p][32] up1, then [p][32] enc1b; cat2:
// [p][64] up2, then [p][64] enc2b), so that every layer writes and reads
// whole pixel rows and no 64-byte half-line is written on its own.
struct CatLayout {
  Map up1, enc1b, up2, enc2b;
};
CatLayout cat_layout(const dfb_denoiser_ctx* n, const Shape& s0, bool planar) {
  const int64_t p0 = s0.pixels(), p1 = p0 / 4;
  if (planar)
    return {mp(n->cat1, 32, 0, 32), mp(n->cat1 + p0 * 32, 32, 0, 32), mp(n->cat2, 64, 0, 64),
            mp(n->cat2 + p1 * 64, 64, 0, 64)};
  return {mp(n->cat1, 64, 0, 32), mp(n->cat1, 64, 32, 32), mp(n->cat2, 128, 0, 64), mp(n->cat2, 128, 64, 64)};
}

// forward on in (f32 NHWC 6 ch) -> n->out.  The 2x2 pools come out of the
// enc1b / enc2b epilogues and the up-sampling is read through by up2 / up1;
// `training` also materialises the up-sampled maps the backward pass reads
// and keeps the skip concatenations interleaved.  With a frame `fv`
// (inference; in unused) the first layer reads its input from the frame's
// accumulation, and the last computes the output conv in its epilogue and
// writes the frame's denoised and display pixels (fallback threshold tau)
// instead of storing dec1b and n->out.
dfb_status forward(dfb_denoiser_ctx* n, const float* in, const Shape& s0, bool training,
                   const dfb::FrameView* fv = nullptr, float tau = 0.f) {
  const bool lean = fv && !training;
  const Shape s1{s0.n, s0.h / 2, s0.w / 2}, s2{s0.n, s0.h / 4, s0.w / 4};
  hipStream_t st = n->stream;
  const float* W = n->w;
  auto B = [&](int i) { return W + n->off_b[i]; };
  using dfb::unet::conv3x3_fwd;
  const Map pool1 = mp(n->pool1, 32, 0, 32), pool2 = mp(n->pool2, 64, 0, 64);
  const CatLayout c = cat_layout(n, s0, !training);
  if (lean) {
    NHIP(n, dfb::unet::conv3x3_in_frame(fv->glue, n->wf[ENC1A], B(ENC1A), mp(n->e1a, 32, 0, 32), s0, st));
  } else {
    NHIP(n, dfb::unet::pack_input(in, 6, n->xin, s0, st));
    NHIP(n, dfb::unet::conv3x3_in_fwd(mp(n->xin, 8, 0, 8), n->wf[ENC1A], B(ENC1A), mp(n->e1a, 32, 0, 32), s0, st));
  }
  NHIP(n, conv3x3_fwd(mp(n->e1a, 32, 0, 32), n->wf[ENC1B], B(ENC1B), c.enc1b, s0, st, false, &pool1));
  NHIP(n, conv3x3_fwd(pool1, n->wf[ENC2A], B(ENC2A), mp(n->e2a, 64, 0, 64), s1, st));
  NHIP(n, conv3x3_fwd(mp(n->e2a, 64, 0, 64), n->wf[ENC2B], B(ENC2B), c.enc2b, s1, st, false, &pool2));
  NHIP(n, conv3x3_fwd(pool2, n->wf[ENC3A], B(ENC3A), mp(n->e3a, 128, 0, 128), s2, st));
  NHIP(n, conv3x3_fwd(mp(n->e3a, 128, 0, 128), n->wf[ENC3B], B(ENC3B), mp(n->e3b, 128, 0, 128), s2, st));
  if (training) NHIP(n, dfb::unet::upsample2(mp(n->e3b, 128, 0, 128), mp(n->up3, 128, 0, 128), s2, st));
  NHIP(n, conv3x3_fwd(mp(n->e3b, 128, 0, 128), n->wf[UP2], B(UP2), c.up2, s1, st, true));
  if (training)
    NHIP(n, conv3x3_fwd(mp(n->cat2, 128, 0, 128), n->wf[DEC2A], B(DEC2A), mp(n->d2a, 64, 0, 64), s1, st));
  else
    NHIP(n, conv3x3_fwd(c.up2, n->wf[DEC2A], B(DEC2A), mp(n->d2a, 64, 0, 64), s1, st, false, nullptr, &c.enc2b));
  NHIP(n, conv3x3_fwd(mp(n->d2a, 64, 0, 64), n->wf[DEC2B], B(DEC2B), mp(n->d2b, 64, 0, 64), s1, st));
  if (training) NHIP(n, dfb::unet::upsample2(mp(n->d2b, 64, 0, 64), mp(n->upd2, 64, 0, 64), s1, st));
  NHIP(n, conv3x3_fwd(mp(n->d2b, 64, 0, 64), n->wf[UP1], B(UP1), c.up1, s0, st, true));
  if (training)
    NHIP(n, conv3x3_fwd(mp(n->cat1, 64, 0, 64), n->wf[DEC1A], B(DEC1A), mp(n->d1a, 32, 0, 32), s0, st));
  else
    NHIP(n, conv3x3_fwd(c.up1, n->wf[DEC1A], B(DEC1A), mp(n->d1a, 32, 0, 32), s0, st, false, nullptr, &c.enc1b));
  if (lean) {
    NHIP(n, dfb::unet::conv3x3_out_frame(mp(n->d1a, 32, 0, 32), n->wf[DEC1B], B(DEC1B), W + n->off_ow, W + n->off_ob,
                                         fv->glue, tau, fv->denoised, fv->final_out, fv->display_mode, fv->inv_gamma,
                                         s0, st));
  } else {
    NHIP(n, conv3x3_fwd(mp(n->d1a, 32, 0, 32), n->wf[DEC1B], B(DEC1B), mp(n->d1b, 32, 0, 32), s0, st));
    NHIP(n, dfb::unet::out_conv_fwd(mp(n->d1b, 32, 0, 32), W + n->off_ow, W + n->off_ob, in, 6, n->out, s0, st));
  }
  n->last = s0;
  n->planar = !training;
  n->lean = lean;
  return DFB_OK;
}

dfb_status backward(dfb_denoiser_ctx* n, const float* target, const Shape& s0) {
  const Shape s1{s0.n, s0.h / 2, s0.w / 2}, s2{s0.n, s0.h / 4, s0.w / 4};
  hipStream_t st = n->stream;
  float* G = n->g;
  auto gw = [&](int i) { return G + n->off_w[i]; };
  auto gb = [&](int i) { return G + n->off_b[i]; };
  float* S = n->scratch;
  using namespace dfb::unet;
  NHIP(n, out_conv_backward(mp(n->d1b, 32, 0, 32), n->out, target, n->w + n->off_ow, mf(n->g_d1b, 32, 0, 32),
                            G + n->off_ow, G + n->off_ob, n->loss_dev, S, s0, st));
  // one conv layer: gate its output gradient dy (output y) once, with the
  // bias gradient, then the data gradient into dx (unless null) and the
  // weight gradient
  auto layer = [&](int L, const MapF& dy, const Map& y, const Map& x, const MapF* dx, const Shape& sh, int ci_out) {
    const Map gm{n->gate, dy.c, 0, dy.c};
    hipError_t e = conv3x3_gate(dy, y, gm, gb(L), S, sh, st);
    if (e == hipSuccess && dx) e = conv3x3_dgrad(gm, n->wd[L], *dx, sh, st);
    if (e == hipSuccess) e = conv3x3_wgrad(x, gm, gw(L), S, sh, st, ci_out);
    return e;
  };
  const MapF dx_d1a = mf(n->g_d1a, 32, 0, 32), dx_cat1 = mf(n->g_cat1, 64, 0, 64), dx_upd2 = mf(n->g_upd2, 64, 0, 64);
  const MapF dx_d2a = mf(n->g_d2a, 64, 0, 64), dx_cat2 = mf(n->g_cat2, 128, 0, 128), dx_up3 = mf(n->g_up3, 128, 0, 128);
  const MapF dx_e3a = mf(n->g_e3a, 128, 0, 128), dx_pool2 = mf(n->g_pool2, 64, 0, 64), dx_e2a = mf(n->g_e2a, 64, 0, 64);
  const MapF dx_pool1 = mf(n->g_pool1, 32, 0, 32), dx_e1a = mf(n->g_e1a, 32, 0, 32);
  // dec1b, dec1a
  NHIP(n, layer(DEC1B, mf(n->g_d1b, 32, 0, 32), mp(n->d1b, 32, 0, 32), mp(n->d1a, 32, 0, 32), &dx_d1a, s0, 32));
  NHIP(n, layer(DEC1A, mf(n->g_d1a, 32, 0, 32), mp(n->d1a, 32, 0, 32), mp(n->cat1, 64, 0, 64), &dx_cat1, s0, 64));
  // up1 (input: upsampled dec2b), output cat1[0:32]
  NHIP(n, layer(UP1, mf(n->g_cat1, 64, 0, 32), mp(n->cat1, 64, 0, 32), mp(n->upd2, 64, 0, 64), &dx_upd2, s0, 64));
  NHIP(n, upsample2_backward(mf(n->g_upd2, 64, 0, 64), mf(n->g_d2b, 64, 0, 64), s1, st));
  // dec2b, dec2a
  NHIP(n, layer(DEC2B, mf(n->g_d2b, 64, 0, 64), mp(n->d2b, 64, 0, 64), mp(n->d2a, 64, 0, 64), &dx_d2a, s1, 64));
  NHIP(n, layer(DEC2A, mf(n->g_d2a, 64, 0, 64), mp(n->d2a, 64, 0, 64), mp(n->cat2, 128, 0, 128), &dx_cat2, s1, 128));
  // up2 (input: upsampled enc3b), output cat2[0:64]
  NHIP(n, layer(UP2, mf(n->g_cat2, 128, 0, 64), mp(n->cat2, 128, 0, 64), mp(n->up3, 128, 0, 128), &dx_up3, s1, 128));
  NHIP(n, upsample2_backward(mf(n->g_up3, 128, 0, 128), mf(n->g_e3b, 128, 0, 128), s2, st));
  // enc3b, enc3a
  NHIP(n, layer(ENC3B, mf(n->g_e3b, 128, 0, 128), mp(n->e3b, 128, 0, 128), mp(n->e3a, 128, 0, 128), &dx_e3a, s2, 128));
  NHIP(n, layer(ENC3A, mf(n->g_e3a, 128, 0, 128), mp(n->e3a, 128, 0, 128), mp(n->pool2, 64, 0, 64), &dx_pool2, s2, 64));
  // skip 2: the enc2b output also fed pool2
  NHIP(n, avgpool2_backward_add(mf(n->g_pool2, 64, 0, 64), mf(n->g_cat2, 128, 64, 64), s1, st));
  NHIP(n, layer(ENC2B, mf(n->g_cat2, 128, 64, 64), mp(n->cat2, 128, 64, 64), mp(n->e2a, 64, 0, 64), &dx_e2a, s1, 64));
  NHIP(n, layer(ENC2A, mf(n->g_e2a, 64, 0, 64), mp(n->e2a, 64, 0, 64), mp(n->pool1, 32, 0, 32), &dx_pool1, s1, 32));
  // skip 1: the enc1b output also fed pool1
  NHIP(n, avgpool2_backward_add(mf(n->g_pool1, 32, 0, 32), mf(n->g_cat1, 64, 32, 32), s0, st));
  NHIP(n, layer(ENC1B, mf(n->g_cat1, 64, 32, 32), mp(n->cat1, 64, 32, 32), mp(n->e1a, 32, 0, 32), &dx_e1a, s0, 32));
  NHIP(n, layer(ENC1A, mf(n->g_e1a, 32, 0, 32), mp(n->e1a, 32, 0, 32), mp(n->xin, 8, 0, 8), nullptr, s0, 6));
  return DFB_OK;
}

dfb_status usable(dfb_denoiser_ctx* n) {
  if (!n) return DFB_ERR_INVALID_ARG;
  if (n->sticky) return nfail(n, DFB_ERR_HIP, "an earlier HIP error left the denoiser unusable: " + n->err);
  return DFB_OK;
}

}  // namespace

extern "C" {

int64_t dfb_denoiser_param_count(void) { return param_count(); }

const char* dfb_denoiser_last_error(dfb_denoiser n) { return n ? n->err.c_str() : g_err.c_str(); }

dfb_status dfb_denoiser_destroy(dfb_denoiser n) {
  if (!n) return DFB_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(n->stream);
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
  return DFB_OK;
}

dfb_status dfb_denoiser_create(const dfb_unet_config* cfg, void* hip_stream, dfb_denoiser* out) {
  if (!cfg || !out) return nfail(nullptr, DFB_ERR_INVALID_ARG, "null argument");
  *out = nullptr;
  if (cfg->max_pixels < 16 || cfg->max_pixels > (int64_t(1) << 27))
    return nfail(nullptr, DFB_ERR_INVALID_ARG, "max_pixels must be in [16, 2^27]");
  dfb_denoiser_ctx* n = new (std::nothrow) dfb_denoiser_ctx();
  if (!n) return nfail(nullptr, DFB_ERR_OOM, "host allocation failed");
  n->cfg = *cfg;
  if (n->cfg.beta1 == 0.f) n->cfg.beta1 = 0.9f;
  if (n->cfg.beta2 == 0.f) n->cfg.beta2 = 0.999f;
  if (n->cfg.eps == 0.f) n->cfg.eps = 1e-8f;
  n->stream = static_cast<hipStream_t>(hip_stream);
  n->n_params = param_count();
  int64_t o = 0;
  for (int i = 0; i < 12; ++i) {
    n->off_w[i] = o;
    o += 9LL * kConv[i].ci * kConv[i].co;
    n->off_b[i] = o;
    o += kConv[i].co;
  }
  n->off_ow = o;
  n->off_ob = o + 96;
  auto bail = [&](dfb_status s) {
    g_err = n->err;
    dfb_denoiser_destroy(n);
    return s;
  };
  dfb_status s;
  const size_t np = static_cast<size_t>(n->n_params);
  if ((s = dalloc(n, &n->w, np)) || (s = dalloc(n, &n->g, np)) || (s = dalloc(n, &n->m, np)) ||
      (s = dalloc(n, &n->v, np)))
    return bail(s);
  for (int i = 0; i < 12; ++i) {
    const size_t wn = 9ull * ((kConv[i].ci + 7) / 8 * 8) * kConv[i].co;
    if ((s = dalloc(n, &n->wf[i], wn)) || (s = dalloc(n, &n->wd[i], wn))) return bail(s);
  }
  const int64_t P0 = cfg->max_pixels, P1 = P0 / 4 + 1, P2 = P0 / 16 + 1;
  n->P0 = P0;
  struct {
    uint16_t** p;
    int64_t n;
  } acts[] = {{&n->xin, P0 * 8},   {&n->e1a, P0 * 32},   {&n->cat1, P0 * 64}, {&n->pool1, P1 * 32},
              {&n->e2a, P1 * 64},  {&n->cat2, P1 * 128}, {&n->pool2, P2 * 64}, {&n->e3a, P2 * 128},
              {&n->e3b, P2 * 128}, {&n->up3, P1 * 128},  {&n->d2a, P1 * 64},  {&n->d2b, P1 * 64},
              {&n->upd2, P0 * 64}, {&n->d1a, P0 * 32},   {&n->d1b, P0 * 32}};
  for (auto& a : acts)
    if ((s = dalloc(n, a.p, static_cast<size_t>(a.n)))) return bail(s);
  struct {
    float** p;
    int64_t n;
  } grads[] = {{&n->g_d1b, P0 * 32},  {&n->g_d1a, P0 * 32},  {&n->g_cat1, P0 * 64},  {&n->g_upd2, P0 * 64},
               {&n->g_d2b, P1 * 64},  {&n->g_d2a, P1 * 64},  {&n->g_cat2, P1 * 128}, {&n->g_up3, P1 * 128},
               {&n->g_e3b, P2 * 128}, {&n->g_e3a, P2 * 128}, {&n->g_pool2, P2 * 64}, {&n->g_e2a, P1 * 64},
               {&n->g_pool1, P1 * 32}, {&n->g_e1a, P0 * 32}, {&n->out, P0 * 3}};
  for (auto& a : grads)
    if ((s = dalloc(n, a.p, static_cast<size_t>(a.n)))) return bail(s);
  size_t sc = dfb::unet::out_conv_scratch(Shape{1, 1, static_cast<int>(P0)});
  for (int i = 0; i < 12; ++i) {
    const int lvl = kConv[i].level;
    const int64_t px = lvl == 0 ? P0 : (lvl == 1 ? P1 : P2);
    const int ci_store = kConv[i].ci == 6 ? 8 : kConv[i].ci;
    sc = std::max(sc, dfb::unet::conv3x3_wgrad_scratch(ci_store, kConv[i].co, Shape{1, 1, static_cast<int>(px)}));
  }
  n->scratch_n = sc;
  if ((s = dalloc(n, &n->scratch, sc)) || (s = dalloc(n, &n->loss_dev, 4))) return bail(s);
  if ((s = dalloc(n, &n->gate, static_cast<size_t>(std::max(P0 * 32, std::max(P1 * 64, P2 * 128)))))) return bail(s);
  // initial parameters: He-normal conv3x3 weights, zero biases, N(0, 0.01) output weights
  std::vector<float> h(np, 0.f);
  uint64_t st = 0x5DEECE66Dull ^ cfg->seed;
  for (int i = 0; i < 12; ++i) {
    const double sd = std::sqrt(2.0 / (9.0 * kConv[i].ci));
    for (int64_t k = 0; k < 9LL * kConv[i].ci * kConv[i].co; ++k) h[n->off_w[i] + k] = static_cast<float>(normal(st) * sd);
  }
  for (int k = 0; k < 96; ++k) h[n->off_ow + k] = static_cast<float>(normal(st) * 0.01);
  if ((s = dfb_denoiser_set_params(n, h.data(), n->n_params)) != DFB_OK) return bail(s);
  *out = n;
  return DFB_OK;
}

dfb_status dfb_denoiser_set_params(dfb_denoiser n, const float* host, int64_t count) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  if (!host || count != n->n_params) return nfail(n, DFB_ERR_INVALID_ARG, "expected dfb_denoiser_param_count() floats");
  const size_t bytes = static_cast<size_t>(count) * sizeof(float);
  NHIP(n, hipMemcpyAsync(n->w, host, bytes, hipMemcpyHostToDevice, n->stream));
  NHIP(n, hipMemsetAsync(n->m, 0, bytes, n->stream));
  NHIP(n, hipMemsetAsync(n->v, 0, bytes, n->stream));
  NHIP(n, hipMemsetAsync(n->g, 0, bytes, n->stream));
  n->step = 0;
  s = refresh(n);
  if (s != DFB_OK) return s;
  NHIP(n, hipStreamSynchronize(n->stream));
  return DFB_OK;
}

dfb_status dfb_denoiser_get_params(dfb_denoiser n, int32_t what, float* host, int64_t count) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  if (!host || count != n->n_params || what < 0 || what > 3) return nfail(n, DFB_ERR_INVALID_ARG, "bad arguments");
  const float* src = what == 0 ? n->w : what == 1 ? n->g : what == 2 ? n->m : n->v;
  NHIP(n, hipMemcpyAsync(host, src, static_cast<size_t>(count) * sizeof(float), hipMemcpyDeviceToHost, n->stream));
  NHIP(n, hipStreamSynchronize(n->stream));
  return DFB_OK;
}

dfb_status dfb_denoiser_forward(dfb_denoiser n, const float* in, float* out, int32_t b, int32_t h, int32_t w) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  if (!in || !out) return nfail(n, DFB_ERR_INVALID_ARG, "null tensor");
  if ((s = check_shape(n, b, h, w)) != DFB_OK) return s;
  const Shape s0{b, h, w};
  if ((s = forward(n, in, s0, false)) != DFB_OK) return s;
  NHIP(n, hipMemcpyAsync(out, n->out, static_cast<size_t>(s0.pixels()) * 3 * sizeof(float), hipMemcpyDeviceToDevice,
                         n->stream));
  return DFB_OK;
}

dfb_status dfb_denoiser_train_step(dfb_denoiser n, const float* in, const float* target, int32_t b, int32_t h,
                                   int32_t w, float lr, int32_t apply_update, float* loss_out) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  if (!in || !target) return nfail(n, DFB_ERR_INVALID_ARG, "null tensor");
  if ((s = check_shape(n, b, h, w)) != DFB_OK) return s;
  const Shape s0{b, h, w};
  if ((s = forward(n, in, s0, true)) != DFB_OK) return s;
  if ((s = backward(n, target, s0)) != DFB_OK) return s;
  if (apply_update) {
    n->step += 1;
    const float c1 = 1.f / (1.f - std::pow(n->cfg.beta1, static_cast<float>(n->step)));
    const float c2 = 1.f / (1.f - std::pow(n->cfg.beta2, static_cast<float>(n->step)));
    NHIP(n, dfb::unet::adam_update(n->w, n->g, n->m, n->v, n->n_params, lr, n->cfg.beta1, n->cfg.beta2, n->cfg.eps,
                                   c1, c2, n->stream));
    if ((s = refresh(n)) != DFB_OK) return s;
  }
  if (loss_out) {
    float sum = 0.f;
    NHIP(n, hipMemcpyAsync(&sum, n->loss_dev, sizeof(float), hipMemcpyDeviceToHost, n->stream));
    NHIP(n, hipStreamSynchronize(n->stream));
    *loss_out = sum / static_cast<float>(s0.pixels() * 3);
  }
  return DFB_OK;
}

dfb_status dfb_denoiser_read_activation(dfb_denoiser n, int32_t layer, void* host, int64_t bytes) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  if (layer < 0 || layer > 11 || !host) return nfail(n, DFB_ERR_INVALID_ARG, "layer must be 0..11");
  const Shape& s0 = n->last;
  if (s0.n == 0) return nfail(n, DFB_ERR_STATE, "no forward pass yet");
  const int lvl = kConv[layer].level;
  const int64_t px = s0.pixels() >> (2 * lvl);
  const int co = kConv[layer].co;
  if (bytes != px * co * 2) return nfail(n, DFB_ERR_INVALID_ARG, "wrong byte count for this layer");
  if (layer == 11 && n->lean) return nfail(n, DFB_ERR_STATE, "dec1b is not stored by dfb_denoise");
  // where each layer's output lives (ld, off)
  const CatLayout c = cat_layout(n, s0, n->planar);
  const Map loc[12] = {mp(n->e1a, 32, 0, 32),   c.enc1b, mp(n->e2a, 64, 0, 64), c.enc2b,
                       mp(n->e3a, 128, 0, 128), mp(n->e3b, 128, 0, 128), c.up2, mp(n->d2a, 64, 0, 64),
                       mp(n->d2b, 64, 0, 64),   c.up1,   mp(n->d1a, 32, 0, 32), mp(n->d1b, 32, 0, 32)};
  const Map& L = loc[layer];
  NHIP(n, hipMemcpy2DAsync(host, co * 2, L.p + L.off, L.ld * 2, co * 2, px, hipMemcpyDeviceToHost, n->stream));
  NHIP(n, hipStreamSynchronize(n->stream));
  return DFB_OK;
}

dfb_status dfb_denoiser_frame_input(dfb_handle h, float* in_dev) {
  dfb::FrameView fv;
  dfb_status s = dfb::frame_view(h, &fv, false);
  if (s != DFB_OK) return s;
  if (!in_dev) return DFB_ERR_INVALID_ARG;
  if (dfb::unet::frame_to_input(fv.glue, in_dev, fv.stream) != hipSuccess) return DFB_ERR_HIP;
  return DFB_OK;
}

dfb_status dfb_denoise(dfb_handle h, dfb_denoiser n, float var_threshold) {
  dfb_status s = usable(n);
  if (s != DFB_OK) return s;
  dfb::FrameView fv;
  if ((s = dfb::frame_view(h, &fv, true)) != DFB_OK) return nfail(n, s, "compositor has no accumulated frame");
  const int W = fv.glue.width, H = fv.glue.height;
  if (W % 4 || H % 4) return nfail(n, DFB_ERR_UNSUPPORTED, "frame width and height must be multiples of 4");
  const int64_t px = static_cast<int64_t>(W) * H;
  if (px > n->P0) return nfail(n, DFB_ERR_INVALID_ARG, "frame larger than the denoiser's max_pixels");
  if (n->stream != fv.stream) {
    // order the compositor's stream before ours
    hipEvent_t e;
    NHIP(n, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    NHIP(n, hipEventRecord(e, fv.stream));
    NHIP(n, hipStreamWaitEvent(n->stream, e, 0));
    NHIP(n, hipEventDestroy(e));
  }
  if ((s = forward(n, nullptr, Shape{1, H, W}, false, &fv, var_threshold)) != DFB_OK) return s;
  if (n->stream != fv.stream) {
    hipEvent_t e;
    NHIP(n, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    NHIP(n, hipEventRecord(e, n->stream));
    NHIP(n, hipStreamWaitEvent(fv.stream, e, 0));
    NHIP(n, hipEventDestroy(e));
  }
  return DFB_OK;
}

}  // extern "C"
