/*
 * dfb.h -- C ABI of an MI355X (gfx950) per-tile sort-last compositor: the
 * data-parallel tile operation of the Distributed FrameBuffer (Usher, Wald,
 * Amstutz, Guenther, Brownlee, Pascucci: "Scalable Ray Tracing Using the
 * Distributed FrameBuffer", EuroVis 2019).
 *
 * One handle owns one GPU's share of a framebuffer: every tile it composites
 * is "owned" by it in the paper's sense (Sec. 3, Listing 1 TileDescriptor).
 * Per frame the caller hands over every contributor's generation-1 tiles
 * (Sec. 3.1.1; Listing 3: one tile per (tile, contributing brick)), and the
 * library runs, on the GPU, the sort-and-blend tile operation (Sec. 4.2,
 * Listing 4), the progressive-refinement accumulation with its variance
 * (Listing 1: accumulationID, accumulation and variance tiles), the
 * tone-mapping pixel operation (Sec. 3.1.2) and the display-format
 * conversion (Sec. 3.1: RGBA8, RGBAF32 or NONE).
 *
 * Conventions shared by every call:
 *  - Every call returns a dfb_status; no C++ exception crosses the ABI.
 *  - Device pointers are HIP device addresses on the device that was current
 *    when the handle was created.  Host pointers are plain process memory.
 *  - Work is enqueued on the HIP stream given to dfb_create (which may be 0,
 *    the null stream).  Results are visible to the host only after
 *    dfb_synchronize or a synchronisation of that stream.
 *  - A HIP error is sticky: once one is seen, every later call on the handle
 *    returns DFB_ERR_HIP.
 *  - One host thread at a time per handle.  dfb_last_error returns a string
 *    owned by the handle, valid until its next call.
 */
#ifndef DFB_H
#define DFB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dfb_ctx* dfb_handle;

typedef enum {
  DFB_OK = 0,
  DFB_ERR_INVALID_ARG = -1,  /* null pointer, bad size, id out of range */
  DFB_ERR_STATE = -2,        /* call out of order (e.g. composite before set_fragments) */
  DFB_ERR_INCOMPLETE = -3,   /* a tile's layer count differs from its declared children */
  DFB_ERR_DUPLICATE = -4,    /* two layers with the same (tile_id, source_id) */
  DFB_ERR_BAD_VALUE = -5,    /* DFB_VALIDATE found a NaN depth */
  DFB_ERR_OOM = -6,          /* a device or host allocation failed */
  DFB_ERR_HIP = -7,          /* a HIP call failed (sticky) */
  DFB_ERR_UNSUPPORTED = -8,  /* e.g. more layers in one tile than the kernels handle */
  DFB_ERR_TREE = -9          /* a dependency tree received more tiles than its parents declared */
} dfb_status;

typedef enum { DFB_F32 = 0, DFB_F16 = 1 } dfb_dtype;   /* storage of all five planes */

/* Display formats of the final pixels (Sec. 3.1): NONE stores nothing. */
typedef enum { DFB_FMT_RGBA8 = 0, DFB_FMT_RGBAF32 = 1, DFB_FMT_NONE = 2 } dfb_format;

/* Tile operations (Sec. 3.1: the tile operation interprets a tile's
 * dependency tree; Sec. 4.1.1; Sec. 4.2).
 *  ALPHA_BLEND  per pixel, sort the layers by depth and blend with "over"
 *               (Sec. 4.2, Listing 4).
 *  LIST         the tree is a list ordered back to front by generation (the
 *               end of Sec. 4.2: valid when a rank-order sort is correct):
 *               a tile's layers are blended in source_id order, the highest
 *               in front, and no depth is read or sorted.  With
 *               dfb_set_fragments, pass each layer's generation (>= 1) as its
 *               source_id; dfb_set_fragments_tree does that itself.
 *  AVERAGE      the mean RGBA of a tile's layers: redundant renders of one
 *               tile with different seeds (Sec. 4.1.1, dynamic load
 *               balancing); the number of layers may differ between tiles;
 *               a tile with none shows the background.  No depth is read. */
typedef enum { DFB_OP_ALPHA_BLEND = 0, DFB_OP_LIST = 1, DFB_OP_AVERAGE = 2 } dfb_tile_op;

typedef enum {
  DFB_BUF_FINAL = 0,          /* display pixels: RGBA8 as uint8[n][P][4], RGBAF32 as float[n][P][4] */
  DFB_BUF_FINISHED_F32 = 1,   /* finished (composited) tile, float[n][P][4]; needs DFB_KEEP_FINISHED */
  DFB_BUF_ACCUM_F32 = 2,      /* running mean, float[n][P][4] */
  DFB_BUF_M2_F32 = 3,         /* Welford M2 of R,G,B, float[n][3][P] (planar per tile) */
  DFB_BUF_TILE_VARIANCE = 4,  /* per-tile variance of the mean, float[n]; +inf while n < 2 */
  DFB_BUF_SORT_ORDER = 5,     /* debug, needs DFB_KEEP_SORT_ORDER: see below */
  DFB_BUF_DENOISED_F32 = 6    /* result of dfb_denoise (dfb_denoise.h), float[n][P][4] */
} dfb_buffer;

/* dfb_config.flags */
#define DFB_VALIDATE 0x1u        /* scan depths on the device; NaN -> DFB_ERR_BAD_VALUE */
#define DFB_KEEP_SORT_ORDER 0x2u /* debug: store each pixel's sorted layer order */
#define DFB_KEEP_FINISHED 0x4u   /* store the finished FP32 tile every frame */

/* dfb_composite_frame frame_flags */
#define DFB_ACCUMULATE 0x1u      /* fold this frame into the running mean (fused) */
#define DFB_REPLAY 0x2u          /* launch the frame as a replay of a HIP graph the handle keeps */

typedef struct {
  int32_t width, height;   /* framebuffer, pixels */
  int32_t tile_w, tile_h;  /* DFB tile: the unit contributors hand over (Listing 1 TILE_SIZE).
                              Tile grid is ceil(W/tw) x ceil(H/th), row-major ids; edge tiles
                              are stored whole, pixels past the image edge are composited but
                              excluded from the variance. */
  int32_t work_w, work_h;  /* GPU scheduling unit inside a tile; must divide tile_w / tile_h.
                              0,0 = autotune over the squares {16,32,64,128}^2 that divide the
                              tile and full-width strips tile_w x (s*s/tile_w) of the same sizes. */
  int32_t waves_per_tile;  /* 64-lane waves per work unit: 1, 2 or 4; 0 = autotune */
  int32_t frag_dtype;      /* dfb_dtype */
  int32_t format;          /* dfb_format */
  float background[4];     /* premultiplied RGBA of the generation-0 background tile (Sec. 4.2) */
  float tonemap_gamma;     /* 1 = clamp only; else colour channels raised to 1/gamma */
  uint32_t flags;          /* DFB_VALIDATE | DFB_KEEP_SORT_ORDER | DFB_KEEP_FINISHED */
  int32_t tile_op;         /* dfb_tile_op; DFB_KEEP_SORT_ORDER needs ALPHA_BLEND or LIST */
  const float* background_image; /* NULL, or a background texture (Sec. 4.2: the background
                              tile holds the background colour or a texture): device
                              float[n_tiles][P][4], premultiplied RGBA, tile-major like the
                              finished tiles, 16-byte aligned.  Borrowed: it must stay valid
                              while frames that use it run; replace it with
                              dfb_set_background_image. */
} dfb_config;

/* One generation-1 tile from one contributor (Listing 1 Tile; Listing 3).
 * Its pixels are block `block` of the fragment buffer: plane c in
 * {0:R, 1:G, 2:B, 3:A, 4:depth} of pixel p (row-major inside the tile) is
 * element frag[(block*5 + c)*P + p], P = tile_w*tile_h, colour premultiplied.
 * source_id names the contributor (a rank, or a rank's brick: Sec. 4.2 allows
 * several bricks per rank); it breaks depth ties, nearer-first by smaller id. */
typedef struct {
  int32_t tile_id;
  uint32_t source_id;
  int64_t block;
} dfb_layer;

typedef struct {
  int32_t n_tiles, tiles_x, tiles_y;
  int32_t n_layers, max_layers_per_tile;
  int32_t work_w, work_h, waves_per_tile;  /* the launch shape in use (after autotune) */
  int32_t accumulation_id;                 /* frames folded in since the last reset (read from
                                              the device: counts graph replays too) */
  int32_t grid_size;                       /* persistent workgroups per frame */
  int64_t n_fragments;                     /* sum over tiles of layers * P */
} dfb_info;

/* Create a compositor: the tile owner's state of Sec. 3 and the buffers of
 * Listing 1's tile operation (finished, accumulation and variance tiles,
 * final pixels in the display format of Sec. 3.1).  Validates cfg and
 * allocates those device buffers on the current device; the accumulation
 * buffers are allocated by the first accumulating frame.
 * hip_stream: a hipStream_t (may be 0); every call of the handle enqueues
 * on it.  On success *out is a new handle owned by the caller; errors leave
 * *out NULL and the reason in dfb_last_error(NULL). */
dfb_status dfb_create(const dfb_config* cfg, void* hip_stream, dfb_handle* out);

/* End of the DFB instance (Sec. 3; Listing 1's buffers): waits for pending
 * work on the handle's stream, then frees every device buffer, the frame
 * graphs and the handle.  Device buffers the caller lent (fragments,
 * background texture) are not touched.  NULL -> DFB_ERR_INVALID_ARG. */
dfb_status dfb_destroy(dfb_handle h);

/* Hand over one frame's generation-1 tiles (Sec. 3.1 setTile; Sec. 3.1.1).
 *   frag_dev   device buffer of n_blocks blocks in cfg.frag_dtype (layout above).
 *              Borrowed, not copied: it must stay unchanged until the frame's
 *              composite has completed on the stream.
 *   layers     host array, any order (arrival order is not fixed, Sec. 3.1.1);
 *              copied during the call.
 *   expected   host int32[n_tiles] or NULL: the children count each tile's
 *              background tile declares (Sec. 4.2).  When given, every tile must
 *              have exactly that many layers, else DFB_ERR_INCOMPLETE.
 * Errors: bad tile id or block -> DFB_ERR_INVALID_ARG, repeated
 * (tile_id, source_id) -> DFB_ERR_DUPLICATE, more than 4096 layers in one
 * tile -> DFB_ERR_UNSUPPORTED.  A tile with no layers is the background. */
dfb_status dfb_set_fragments(dfb_handle h, const void* frag_dev, int64_t n_blocks,
                             const dfb_layer* layers, int32_t n_layers, const int32_t* expected);

/* Composite every tile of the frame in one persistent launch on the handle's
 * stream that takes tiles from a device work queue in longest-first order:
 * per pixel, sort the layers by (depth with NaN last and -0 == +0,
 * source_id), blend front to back with premultiplied "over", put the
 * background colour behind (Sec. 4.2, Listing 4).  With DFB_ACCUMULATE the
 * same launch folds the frame into the running mean (Welford) and writes the
 * display pixels of the mean, and a second, small launch combines its
 * per-unit sums into the per-tile variance of the mean; without it the
 * display pixels are those of this frame.
 * Tonemap: y = clamp(x,0,1) (NaN -> 0), colour ^ (1/gamma), code
 * floor(255 y + 0.5).  If work_w/waves_per_tile are 0, the first frame of a
 * new layer layout first autotunes them (synchronously).
 * Per-frame state (the work queue's counter slot, the accumulation count)
 * lives in device memory and is advanced by the frame's own kernels, so the
 * launches of one call are the same for every frame of a layer table:
 *  - DFB_REPLAY launches the frame as a replay of a HIP graph (frame kernel,
 *    then the variance combine of an accumulating frame) that the handle
 *    builds on first use for the current layer table, launch shape,
 *    fragment buffer and flags, and keeps (up to 8 buffers and flag sets)
 *    until the layer layout, the shape or the background texture changes.
 *  - The caller may also capture a call on the handle's stream into a graph
 *    of its own and replay that graph once per frame.  Under capture the
 *    call fails with DFB_ERR_STATE if the layout's launch shape is not
 *    chosen yet (composite one frame first) or, with DFB_ACCUMULATE, if no
 *    frame was accumulated yet; it does no timing.  The graph holds the
 *    fragment buffer given to the last dfb_set_fragments and the layer
 *    table: replays see what those hold when they run.
 * Errors: before any dfb_set_fragments -> DFB_ERR_STATE; unknown flags ->
 * DFB_ERR_INVALID_ARG. */
dfb_status dfb_composite_frame(dfb_handle h, uint32_t frame_flags);

/* Replace the background texture (NULL: back to cfg.background) for the
 * frames composited after this call.  Layout and ownership as
 * dfb_config.background_image; a pointer that is not 16-byte aligned ->
 * DFB_ERR_INVALID_ARG. */
dfb_status dfb_set_background_image(dfb_handle h, const float* image_dev);

/* One layer's place in its tile's dependency tree (Sec. 3.1.1; Listing 1
 * Tile.generation / Tile.children). */
typedef struct {
  int32_t generation;  /* >= 1; generation 0 is the background tile */
  int32_t children;    /* >= 0: tiles this one adds to generation + 1 */
} dfb_tree_node;

/* dfb_set_fragments with general per-tile dependency trees (Sec. 3.1.1):
 * tree[i] places layers[i]; bg_children[t] (host int32[n_tiles]) is what the
 * background tile of tile t declares for generation 1.  Every tile's tree is
 * checked with the same bookkeeping as dfb_tree_add, the layers taken in
 * array order as arrival order; a tree still waiting for tiles after the
 * last layer -> DFB_ERR_INCOMPLETE, more tiles in a generation than its
 * parents declared -> DFB_ERR_TREE.  ALPHA_BLEND and AVERAGE then treat all
 * generations alike; LIST needs exactly one tile per generation and blends
 * them by generation, the highest in front. */
dfb_status dfb_set_fragments_tree(dfb_handle h, const void* frag_dev, int64_t n_blocks,
                                  const dfb_layer* layers, const dfb_tree_node* tree,
                                  int32_t n_layers, const int32_t* bg_children);

/* Host-side dependency-tree bookkeeping for tiles that arrive one at a time
 * (Sec. 3.1.1; Listing 4's process): per tile, generation 0 starts with one
 * expected tile; a generation is done when as many of its tiles arrived as
 * its parents declared children, and the next generation then expects the
 * sum of the children its tiles declared; the tree is complete when a done
 * generation declared no children.  Tiles may arrive in any generation
 * order: later generations are counted until their parents are done.
 * No GPU is involved. */
typedef struct dfb_tree_s* dfb_tree;

/* n_tiles >= 1 trees, each waiting for its generation-0 tile. */
dfb_status dfb_tree_create(int32_t n_tiles, dfb_tree* out);
dfb_status dfb_tree_destroy(dfb_tree t);

/* Forget every arrival: each tile again waits for its generation-0 tile. */
dfb_status dfb_tree_new_frame(dfb_tree t);

/* One tile arrives.  *completed (nullable) = 1 if this arrival completed the
 * tile's tree, else 0.  generation outside [0, 65535], children < 0 or tile_id
 * out of range -> DFB_ERR_INVALID_ARG; a tile that makes some generation hold
 * more tiles than declared, found as soon as all generations before it are
 * done (also any tile after completion) -> DFB_ERR_TREE, and the tile's tree
 * stays in error until dfb_tree_new_frame. */
dfb_status dfb_tree_add(dfb_tree t, int32_t tile_id, int32_t generation, int32_t children,
                        int32_t* completed);

/* State of one tile's tree: *state = 1 complete, 0 waiting, -1 error;
 * *generation = the generation being completed (the last one when complete);
 * *missing = tiles that generation still waits for (0 when complete).
 * Each output is nullable. */
dfb_status dfb_tree_query(dfb_tree t, int32_t tile_id, int32_t* state, int32_t* generation,
                          int32_t* missing);

/* Variance-driven assignment of extra samples (Sec. 4.1.1: tiles with a
 * higher variance get more renders).  Distributes `extra` (0 <= extra <
 * 2^31) additional tile renders over the n_tiles tiles in proportion to each
 * tile's variance of the mean, by largest remainders:
 *   w_t = v_t where finite and > 0, else 0;  S = sum of w_t in tile order,
 *   in double;  q_t = extra * w_t / S (double);  c_t = floor(q_t); the
 *   extra - sum c_t renders left go one each to the tiles of largest
 *   q_t - c_t, ties to the smaller tile id.
 * S == 0 -> uniform: floor(extra / n_tiles) each and one more for the first
 * extra mod n_tiles tiles.  counts: host int32[n_tiles]. */
dfb_status dfb_assign_samples_host(const float* variance, int32_t n_tiles, int64_t extra,
                                   int32_t* counts);

/* The same from the handle's per-tile variance (DFB_BUF_TILE_VARIANCE of the
 * last accumulated frame; uniform before two frames are accumulated).
 * Synchronises the handle's stream. */
dfb_status dfb_assign_samples(dfb_handle h, int64_t extra, int32_t* counts);

/* Progressive refinement (Listing 1: accumulationID and the accumulation
 * and variance tiles), unfused: fold the last finished frame into the
 * running mean as frame n = accumulationID + 1, with the same Welford
 * update, per-tile variance of the mean and display conversion as
 * DFB_ACCUMULATE, in a separate pass.  Needs a frame composited with
 * DFB_KEEP_FINISHED and without DFB_ACCUMULATE that was not accumulated
 * yet, else DFB_ERR_STATE (a frame is never folded in twice). */
dfb_status dfb_accumulate(dfb_handle h);

/* Restart progressive refinement (Listing 1: accumulationID := 0, as when
 * the camera moves): the next accumulated frame is n = 1 and replaces the
 * mean.  Stream-ordered: frames enqueued before it still accumulate. */
dfb_status dfb_reset_accumulation(dfb_handle h);

/* Read out finished pixels (Listing 1: finalPixels, in the display format
 * of Sec. 3.1) or another of the tile operation's buffers.
 * Copy tiles [first_tile, first_tile + n_tiles) of one buffer to dst (host, or
 * device if dst_is_device; the caller owns dst, which must hold
 * dfb_buffer_bytes for the range), stream-ordered: a host dst is complete
 * after dfb_synchronize.  Bad range or NULL dst -> DFB_ERR_INVALID_ARG; no
 * composited frame, or a buffer its flag or format did not enable ->
 * DFB_ERR_STATE.  DFB_BUF_SORT_ORDER holds, for
 * each tile in id order, uint16[K_t][P]: entry (i, p) is the index, among the
 * tile's layers ordered by ascending source_id, of the i-th nearest fragment
 * of pixel p; it is only kept for the last composited frame. */
dfb_status dfb_read_tiles(dfb_handle h, dfb_buffer which, int32_t first_tile, int32_t n_tiles,
                          void* dst, int dst_is_device);

/* Bytes dfb_read_tiles would copy for that range (0 if not available). */
int64_t dfb_buffer_bytes(dfb_handle h, dfb_buffer which, int32_t first_tile, int32_t n_tiles);

/* Plumbing, no paper counterpart: wait for everything enqueued on the
 * handle's stream; a device fault is returned here (and stays sticky). */
dfb_status dfb_synchronize(dfb_handle h);

/* Shape of the current frame and launch (plumbing).  Reads the
 * accumulation count from the device: synchronises the stream, so not
 * during a capture. */
dfb_status dfb_get_info(dfb_handle h, dfb_info* out);

/* Average device time (ms) of the frame kernel over the timed composites
 * since the last dfb_set_timing call, measured with HIP events recorded right
 * before and after the frame kernel on the handle's stream; -1 if none were
 * timed.  dfb_set_timing(h, n): time the first composite after the call and
 * every n-th one after it (n = 1: every composite; n <= 0: none).  Each timed
 * composite adds the two event records to the stream (a few microseconds). */
dfb_status dfb_set_timing(dfb_handle h, int every);
double dfb_kernel_ms(dfb_handle h);

/* The individual timings behind dfb_kernel_ms (plumbing): copies the first
 * min(cap, count) per-frame times (ms, frame order) to ms (host float[cap])
 * and returns count, the number timed since dfb_set_timing; -1 on a bad
 * argument or HIP error.  Waits for the timed frames to finish. */
int32_t dfb_kernel_times(dfb_handle h, float* ms, int32_t cap);

/* Host-only check of one frame's layer list against a config, without a GPU:
 * the same validation dfb_set_fragments does.  counts: nullable int32[n_tiles]
 * that receives each tile's layer count. */
dfb_status dfb_validate_layers(const dfb_config* cfg, int64_t n_blocks, const dfb_layer* layers,
                               int32_t n_layers, const int32_t* expected, int32_t* counts);

/* Entry point for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): one plain frame -- the same frame kernel as
 * dfb_composite_frame, without accumulation -- into caller-owned outputs.
 * It calls no allocator: its work queue's counters, the frame state and the
 * longest-first work list (built on the device from tile_off_dev) live in a
 * static device array of DFB_NOALLOC_MAX_WORK work units plus 72 KiB, one
 * per GPU, held until the process ends; the first call on a device clears
 * it (a fill kernel on hip_stream).  All calls on one GPU share that array:
 * calls that overlap in time on one GPU (different streams or threads)
 * race and give wrong results; calls ordered on one stream are safe.
 *   cfg           as for dfb_create; work_w, work_h and waves_per_tile must
 *                 be set (no autotuning); DFB_VALIDATE and
 *                 DFB_KEEP_SORT_ORDER -> DFB_ERR_UNSUPPORTED.
 *   frag_dev      fragment blocks (layout of dfb_layer), cfg.frag_dtype.
 *   tile_off_dev  device int32[n_tiles + 1]: tile t's layers are entries
 *                 tile_off[t] .. tile_off[t+1]-1 of layer_off_dev.
 *   layer_off_dev device int64[n_layers]: element offset block * 5 * P of
 *                 each layer's block in frag_dev; a tile's layers ordered by
 *                 ascending source_id (depth ties go to the earlier one).
 *   max_layers    at least the largest layer count of any tile (<= 4096):
 *                 it picks the kernel; a tile with more layers is not
 *                 composited correctly.
 *   final_dev     display pixels per cfg.format (NULL for DFB_FMT_NONE).
 *   finished_dev  float[n_tiles][P][4] with DFB_KEEP_FINISHED, else NULL.
 *   hip_stream    every launch is enqueued on it; nothing synchronises.
 * A frame of more than DFB_NOALLOC_MAX_WORK work units (n_tiles * units per
 * tile) -> DFB_ERR_UNSUPPORTED before any GPU work.  Errors are reported in
 * dfb_last_error(NULL). */
#define DFB_NOALLOC_MAX_WORK 1048576
dfb_status dfb_composite_noalloc(const dfb_config* cfg, const void* frag_dev, const int32_t* tile_off_dev,
                                 const int64_t* layer_off_dev, int32_t max_layers, void* final_dev,
                                 float* finished_dev, void* hip_stream);

/* Human-readable last error of the handle (or of the last failed create when
 * h is NULL). */
const char* dfb_last_error(dfb_handle h);
const char* dfb_status_string(dfb_status s);

#ifdef __cplusplus
}
#endif
#endif /* DFB_H */
