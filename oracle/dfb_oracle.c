/*
 * dfb_oracle.c -- plain, slow, FP64 CPU reference of per-tile sort-last
 * compositing (Distributed FrameBuffer, Usher et al., EuroVis 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no header, helper or table with the GPU
 * path: it declares its own layer record and its own fp16 decoder.
 *
 * Every step is written as the plain definition of what the method computes,
 * in the order the paper states it:
 *   O1 group   -- collect the generation-1 tiles of every tile (Sec. 3.1,
 *                 Listing 1 "Tile"; arrival order is not fixed, Sec. 3.1.1).
 *   O2 check   -- the background tile (the only generation-0 member) declares
 *                 how many children to expect; the tree is complete when that
 *                 many arrived (Sec. 3.1.1, Sec. 4.2, Listing 4).
 *   O3 key     -- per fragment (is_nan(depth), depth with -0 == +0, source id),
 *                 compared lexicographically (reading: smaller depth is
 *                 nearer, ties broken by the contributor's id).
 *   O4 sort    -- per pixel, not per rank (Sec. 4.2).
 *   O5 blend   -- front-to-back premultiplied "over", then the background
 *                 colour, or a background texture, behind everything
 *                 (Sec. 4.2).
 *   O5L list   -- when a rank-order sort is correct the tree is a list of
 *                 tiles ordered back to front by generation (end of
 *                 Sec. 4.2): starting from the background, each generation
 *                 in increasing order is put "over" what is behind it.
 *   O5A average -- redundant renders of one tile with different seeds are
 *                 averaged (Sec. 4.1.1, dynamic load balancing).
 *   O6 accumulate -- progressive refinement as the running mean since the
 *                 last reset, with Welford's M2 (Listing 1 accumulationID,
 *                 accumulation and variance tiles).
 *   O7 variance -- per-tile variance of the mean over in-image pixels and RGB
 *                 (Sec. 4.1.1: tiles with higher variance get more samples).
 *   O8 tonemap -- pixel operation + display-format conversion to RGBA8
 *                 (Sec. 3.1.2, Sec. 3.1).
 * All arithmetic is in double.  Build with -O2 -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* One generation-1 tile handed over by a contributor (the paper's Tile:
 * tile id, the contributor, and where its pixel planes sit). */
typedef struct {
  int32_t tile_id;
  uint32_t source_id;
  int64_t block;
} orc_layer;

enum { ORC_OK = 0, ORC_ERR_ARG = -1, ORC_ERR_INCOMPLETE = -3, ORC_ERR_DUPLICATE = -4 };

/* ---- fp16 -> double, written from the IEEE 754 binary16 definition ----- */
double orc_half_to_double(uint16_t h) {
  int sign = (h >> 15) & 1;
  int expo = (h >> 10) & 0x1f;
  int mant = h & 0x3ff;
  double v;
  if (expo == 0) {
    v = ldexp((double)mant, -24); /* subnormal: mant * 2^-14 * 2^-10 */
  } else if (expo == 31) {
    v = mant ? NAN : INFINITY;
  } else {
    v = ldexp((double)(mant + 1024), expo - 25); /* (1 + m/1024) * 2^(e-15) */
  }
  return sign ? -v : v;
}

/* read plane c (0..4 = R,G,B,A,depth) of pixel p of block b */
static double frag_value(const void* frag, int dtype, int64_t P, int64_t b, int c, int64_t p) {
  int64_t i = (b * 5 + c) * P + p;
  if (dtype == 0) return (double)((const float*)frag)[i];
  return orc_half_to_double(((const uint16_t*)frag)[i]);
}

/* ---- O3: the depth key ------------------------------------------------- */
typedef struct {
  int nan;       /* 1 if the depth is NaN: sorts after every number */
  double v;      /* depth, with -0 mapped to +0 */
  uint32_t sid;  /* source id: unique within a tile */
  int slot;      /* which of the tile's layers it came from */
} orc_key;

static orc_key make_key(double depth, uint32_t sid, int slot) {
  orc_key k;
  k.nan = isnan(depth) ? 1 : 0;
  k.v = k.nan ? 0.0 : (depth == 0.0 ? 0.0 : depth);
  k.sid = sid;
  k.slot = slot;
  return k;
}

static int key_cmp(const void* pa, const void* pb) {
  const orc_key* a = (const orc_key*)pa;
  const orc_key* b = (const orc_key*)pb;
  if (a->nan != b->nan) return a->nan < b->nan ? -1 : 1;
  if (a->v != b->v) return a->v < b->v ? -1 : 1;
  if (a->sid != b->sid) return a->sid < b->sid ? -1 : 1;
  return 0;
}

/* ---- O1 + O2: group and check ------------------------------------------ */
typedef struct {
  int32_t n_tiles;
  int32_t* count;   /* [n_tiles] */
  int64_t* start;   /* [n_tiles + 1] */
  int32_t* members; /* [n_layers] layer indices grouped by tile, arrival order */
} orc_groups;

static void free_groups(orc_groups* g) {
  free(g->count);
  free(g->start);
  free(g->members);
}

static int group_layers(const orc_layer* layers, int32_t n_layers, int64_t n_blocks,
                        const int32_t* expected, int32_t n_tiles, orc_groups* g) {
  memset(g, 0, sizeof(*g));
  g->n_tiles = n_tiles;
  g->count = (int32_t*)calloc((size_t)n_tiles, sizeof(int32_t));
  g->start = (int64_t*)calloc((size_t)n_tiles + 1, sizeof(int64_t));
  g->members = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_layers > 0 ? n_layers : 1));
  if (!g->count || !g->start || !g->members) return ORC_ERR_ARG;
  for (int32_t i = 0; i < n_layers; ++i) {
    if (layers[i].tile_id < 0 || layers[i].tile_id >= n_tiles) return ORC_ERR_ARG;
    if (layers[i].block < 0 || layers[i].block >= n_blocks) return ORC_ERR_ARG;
    g->count[layers[i].tile_id]++;
  }
  for (int32_t t = 0; t < n_tiles; ++t) g->start[t + 1] = g->start[t] + g->count[t];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_tiles);
  if (!fill) return ORC_ERR_ARG;
  for (int32_t t = 0; t < n_tiles; ++t) fill[t] = g->start[t];
  for (int32_t i = 0; i < n_layers; ++i) g->members[fill[layers[i].tile_id]++] = i;
  free(fill);
  /* a contributor hands over at most one tile per tile id */
  for (int32_t t = 0; t < n_tiles; ++t)
    for (int64_t a = g->start[t]; a < g->start[t + 1]; ++a)
      for (int64_t b = a + 1; b < g->start[t + 1]; ++b)
        if (layers[g->members[a]].source_id == layers[g->members[b]].source_id)
          return ORC_ERR_DUPLICATE;
  /* O2: the background tile's declared children must all have arrived */
  if (expected)
    for (int32_t t = 0; t < n_tiles; ++t)
      if (g->count[t] != expected[t]) return ORC_ERR_INCOMPLETE;
  return ORC_OK;
}

/* ---- O4 + O5 for one tile ---------------------------------------------- */
typedef struct {
  const void* frag;
  int dtype;
  const orc_layer* layers;
  const orc_groups* g;
  int32_t tile_w, tile_h;
  double bg[4];
  const double* bg_image; /* nullable [n_tiles][P][4] */
  int op;                 /* 0 sort + blend, 1 list, 2 average */
  const int32_t* out_tiles;
  int32_t n_out;
  double* out_rgba;     /* [n_out][P][4] */
  double* out_mag;      /* [n_out][P][4] nullable: sum of T_i |c_i| + T |bg| */
  uint32_t* out_order;  /* [n_out][P][kmax] nullable: source ids nearest first */
  int32_t kmax;
  int32_t next;         /* shared work counter */
  pthread_mutex_t lock;
} orc_job;

/* the background of pixel p of tile t */
static void background(const orc_job* job, int32_t t, int64_t P, int64_t p, double out[4]) {
  for (int c = 0; c < 4; ++c) out[c] = job->bg_image ? job->bg_image[((int64_t)t * P + p) * 4 + c] : job->bg[c];
}

static void store(orc_job* job, int32_t oi, int64_t P, int64_t p, const double v[4], const double m[4]) {
  double* o = job->out_rgba + (oi * P + p) * 4;
  for (int c = 0; c < 4; ++c) o[c] = v[c];
  if (job->out_mag) {
    double* q = job->out_mag + (oi * P + p) * 4;
    for (int c = 0; c < 4; ++c) q[c] = m[c];
  }
}

/* O5L: back to front, generation by generation, each tile "over" the rest */
static void list_tile(orc_job* job, int32_t oi) {
  const int32_t t = job->out_tiles[oi];
  const int64_t P = (int64_t)job->tile_w * job->tile_h;
  const orc_groups* g = job->g;
  const int32_t K = g->count[t];
  /* the tile's layers by increasing generation (= source id) */
  int32_t* byg = (int32_t*)malloc(sizeof(int32_t) * (size_t)(K > 0 ? K : 1));
  for (int32_t i = 0; i < K; ++i) byg[i] = g->members[g->start[t] + i];
  for (int32_t i = 1; i < K; ++i)
    for (int32_t j = i; j > 0 && job->layers[byg[j - 1]].source_id > job->layers[byg[j]].source_id; --j) {
      int32_t x = byg[j]; byg[j] = byg[j - 1]; byg[j - 1] = x;
    }
  for (int64_t p = 0; p < P; ++p) {
    double v[4], m[4];
    background(job, t, P, p, v);
    for (int c = 0; c < 4; ++c) m[c] = fabs(v[c]);
    for (int32_t i = 0; i < K; ++i) {
      const orc_layer* L = &job->layers[byg[i]];
      const double a = frag_value(job->frag, job->dtype, P, L->block, 3, p);
      for (int c = 0; c < 4; ++c) {
        const double x = frag_value(job->frag, job->dtype, P, L->block, c, p);
        v[c] = x + (1.0 - a) * v[c];
        m[c] = fabs(x) + (1.0 - a) * m[c];
      }
      /* nearest first: generation K-1-i sits at position i of the order */
      if (job->out_order) job->out_order[(oi * P + p) * job->kmax + (K - 1 - i)] = L->source_id;
    }
    store(job, oi, P, p, v, m);
  }
  free(byg);
}

/* O5A: the mean of the tile's layers; none -> the background */
static void average_tile(orc_job* job, int32_t oi) {
  const int32_t t = job->out_tiles[oi];
  const int64_t P = (int64_t)job->tile_w * job->tile_h;
  const orc_groups* g = job->g;
  const int32_t K = g->count[t];
  for (int64_t p = 0; p < P; ++p) {
    double v[4] = {0.0, 0.0, 0.0, 0.0}, m[4] = {0.0, 0.0, 0.0, 0.0};
    if (K == 0) {
      background(job, t, P, p, v);
      for (int c = 0; c < 4; ++c) m[c] = fabs(v[c]);
    } else {
      for (int32_t i = 0; i < K; ++i) {
        const orc_layer* L = &job->layers[g->members[g->start[t] + i]];
        for (int c = 0; c < 4; ++c) {
          const double x = frag_value(job->frag, job->dtype, P, L->block, c, p);
          v[c] += x;
          m[c] += fabs(x);
        }
      }
      for (int c = 0; c < 4; ++c) {
        v[c] /= (double)K;
        m[c] /= (double)K;
      }
    }
    store(job, oi, P, p, v, m);
  }
}

static void composite_tile(orc_job* job, int32_t oi) {
  if (job->op == 1) { list_tile(job, oi); return; }
  if (job->op == 2) { average_tile(job, oi); return; }
  const int32_t t = job->out_tiles[oi];
  const int64_t P = (int64_t)job->tile_w * job->tile_h;
  const orc_groups* g = job->g;
  const int32_t K = g->count[t];
  orc_key* keys = (orc_key*)malloc(sizeof(orc_key) * (size_t)(K > 0 ? K : 1));
  for (int64_t p = 0; p < P; ++p) {
    for (int32_t i = 0; i < K; ++i) {
      const orc_layer* L = &job->layers[g->members[g->start[t] + i]];
      keys[i] = make_key(frag_value(job->frag, job->dtype, P, L->block, 4, p), L->source_id, i);
    }
    qsort(keys, (size_t)K, sizeof(orc_key), key_cmp); /* O4 */
    double C[3] = {0.0, 0.0, 0.0}, A = 0.0, T = 1.0;   /* O5 */
    double M[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t i = 0; i < K; ++i) {
      const orc_layer* L = &job->layers[g->members[g->start[t] + keys[i].slot]];
      double a = frag_value(job->frag, job->dtype, P, L->block, 3, p);
      for (int c = 0; c < 3; ++c) {
        double col = frag_value(job->frag, job->dtype, P, L->block, c, p);
        C[c] += T * col;
        M[c] += T * fabs(col);
      }
      A += T * a;
      M[3] += T * fabs(a);
      T *= (1.0 - a);
      if (job->out_order) job->out_order[(oi * P + p) * job->kmax + i] = keys[i].sid;
    }
    double bg[4];
    background(job, t, P, p, bg);
    for (int c = 0; c < 3; ++c) {
      C[c] += T * bg[c];
      M[c] += T * fabs(bg[c]);
    }
    A += T * bg[3];
    M[3] += T * fabs(bg[3]);
    double* o = job->out_rgba + (oi * P + p) * 4;
    o[0] = C[0]; o[1] = C[1]; o[2] = C[2]; o[3] = A;
    if (job->out_mag) {
      double* m = job->out_mag + (oi * P + p) * 4;
      m[0] = M[0]; m[1] = M[1]; m[2] = M[2]; m[3] = M[3];
    }
  }
  free(keys);
}

static void* worker(void* arg) {
  orc_job* job = (orc_job*)arg;
  for (;;) {
    pthread_mutex_lock(&job->lock);
    int32_t oi = job->next++;
    pthread_mutex_unlock(&job->lock);
    if (oi >= job->n_out) break;
    composite_tile(job, oi);
  }
  return NULL;
}

/*
 * Composite the listed tiles of one frame.
 *   frag       host copy of the fragment blocks; block b, plane c (R,G,B,A,
 *              depth), pixel p at element (b*5 + c)*P + p; dtype 0 = f32,
 *              1 = f16 (IEEE binary16 bits).
 *   layers     generation-1 tiles in any order.
 *   expected   nullable, [n_tiles]: the background tile's children count.
 *   bg         nullable RGBA background colour (default 0).
 *   op         0: per-pixel sort + blend; 1: list by generation (source id
 *              >= 1 is the generation); 2: average.
 *   bg_image   nullable [n_tiles][P][4]: a background texture, used instead
 *              of bg.
 *   out_tiles  tile ids to compute; outputs are in this order.
 *   out_order  nullable, [n_out][P][kmax]: source ids, nearest first (not
 *              with op 2).
 * Returns 0, or a negative error (bad id / duplicate / incomplete tree).
 */
int orc_composite(const void* frag, int dtype, int64_t n_blocks, const orc_layer* layers,
                  int32_t n_layers, const int32_t* expected, int32_t width, int32_t height,
                  int32_t tile_w, int32_t tile_h, const double* bg, int32_t op,
                  const double* bg_image, const int32_t* out_tiles, int32_t n_out,
                  double* out_rgba, double* out_mag, uint32_t* out_order, int32_t kmax,
                  int32_t n_threads) {
  if (width <= 0 || height <= 0 || tile_w <= 0 || tile_h <= 0 || (dtype != 0 && dtype != 1))
    return ORC_ERR_ARG;
  if (op < 0 || op > 2 || (op == 2 && out_order)) return ORC_ERR_ARG;
  if (op == 1)
    for (int32_t i = 0; i < n_layers; ++i)
      if (layers[i].source_id == 0) return ORC_ERR_ARG; /* generation 0 is the background */
  const int32_t tiles_x = (width + tile_w - 1) / tile_w;
  const int32_t tiles_y = (height + tile_h - 1) / tile_h;
  const int32_t n_tiles = tiles_x * tiles_y;
  orc_groups g;
  int rc = group_layers(layers, n_layers, n_blocks, expected, n_tiles, &g);
  if (rc != ORC_OK) { free_groups(&g); return rc; }
  for (int32_t i = 0; i < n_out; ++i) {
    if (out_tiles[i] < 0 || out_tiles[i] >= n_tiles) { free_groups(&g); return ORC_ERR_ARG; }
    if (out_order && g.count[out_tiles[i]] > kmax) { free_groups(&g); return ORC_ERR_ARG; }
  }
  orc_job job;
  job.frag = frag; job.dtype = dtype; job.layers = layers; job.g = &g;
  job.tile_w = tile_w; job.tile_h = tile_h;
  for (int c = 0; c < 4; ++c) job.bg[c] = bg ? bg[c] : 0.0;
  job.bg_image = bg_image;
  job.op = op;
  job.out_tiles = out_tiles; job.n_out = n_out;
  job.out_rgba = out_rgba; job.out_mag = out_mag; job.out_order = out_order; job.kmax = kmax;
  job.next = 0;
  pthread_mutex_init(&job.lock, NULL);
  if (n_threads < 1) n_threads = 1;
  if (n_threads > 256) n_threads = 256;
  pthread_t th[256];
  for (int i = 0; i < n_threads; ++i) pthread_create(&th[i], NULL, worker, &job);
  for (int i = 0; i < n_threads; ++i) pthread_join(th[i], NULL);
  pthread_mutex_destroy(&job.lock);
  free_groups(&g);
  return ORC_OK;
}

/* number of layers of every tile: [n_tiles]; validates like orc_composite */
int orc_tile_counts(const orc_layer* layers, int32_t n_layers, int64_t n_blocks,
                    const int32_t* expected, int32_t n_tiles, int32_t* counts) {
  orc_groups g;
  int rc = group_layers(layers, n_layers, n_blocks, expected, n_tiles, &g);
  if (rc == ORC_OK) memcpy(counts, g.count, sizeof(int32_t) * (size_t)n_tiles);
  free_groups(&g);
  return rc;
}

/* ---- O6: Welford update of one frame into the running mean --------------
 * mu [n_px][4] (RGBA), m2 [n_px][3] (RGB), x [n_px][4]; n = number of frames
 * including this one (n >= 1).  For n == 1 this sets mu = x and m2 = 0. */
void orc_accumulate(double* mu, double* m2, const double* x, int64_t n_px, int32_t n) {
  for (int64_t p = 0; p < n_px; ++p) {
    for (int c = 0; c < 4; ++c) {
      double xi = x[p * 4 + c];
      double delta = xi - mu[p * 4 + c];
      if (n == 1) {
        mu[p * 4 + c] = xi;
        if (c < 3) m2[p * 3 + c] = 0.0;
        continue;
      }
      mu[p * 4 + c] += delta / (double)n;
      if (c < 3) m2[p * 3 + c] += delta * (xi - mu[p * 4 + c]);
    }
  }
}

/* ---- O7: per-tile variance of the mean ---------------------------------
 * m2 [n_out][P][3] for the listed tiles; v_t = sum over in-image pixels and
 * RGB of m2 / (3 * P_t * n * (n - 1)); +inf when n < 2 (nothing measured). */
void orc_tile_variance(const double* m2, const int32_t* out_tiles, int32_t n_out, int32_t width,
                       int32_t height, int32_t tile_w, int32_t tile_h, int32_t n, double* v) {
  const int32_t tiles_x = (width + tile_w - 1) / tile_w;
  const int64_t P = (int64_t)tile_w * tile_h;
  for (int32_t oi = 0; oi < n_out; ++oi) {
    if (n < 2) { v[oi] = INFINITY; continue; }
    const int32_t t = out_tiles[oi];
    const int32_t x0 = (t % tiles_x) * tile_w, y0 = (t / tiles_x) * tile_h;
    double s = 0.0;
    int64_t inside = 0;
    for (int32_t py = 0; py < tile_h; ++py)
      for (int32_t px = 0; px < tile_w; ++px) {
        if (x0 + px >= width || y0 + py >= height) continue;
        ++inside;
        const double* q = m2 + ((int64_t)oi * P + (int64_t)py * tile_w + px) * 3;
        s += q[0] + q[1] + q[2];
      }
    v[oi] = s / (3.0 * (double)inside * (double)n * (double)(n - 1));
  }
}

/* ---- O8: tonemap pixel operation + RGBA8 display conversion ------------
 * y = clamp(x, 0, 1) (NaN -> 0); colour channels raised to 1/gamma when
 * gamma != 1; code = floor(255 y + 0.5). */
void orc_tonemap(const double* x, int64_t n_px, double gamma, uint8_t* out) {
  for (int64_t p = 0; p < n_px; ++p)
    for (int c = 0; c < 4; ++c) {
      double y = x[p * 4 + c];
      if (isnan(y)) y = 0.0;
      if (y < 0.0) y = 0.0;
      if (y > 1.0) y = 1.0;
      if (c < 3 && gamma != 1.0) y = pow(y, 1.0 / gamma);
      out[p * 4 + c] = (uint8_t)floor(255.0 * y + 0.5);
    }
}
