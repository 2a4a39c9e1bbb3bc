/*
 * dcgs.h -- C ABI of the DiskChunGS mapping-step hot path on MI355X (gfx950).
 *
 * The paper (DiskChunGS, arXiv 2511.23030) optimises a chunked 3D Gaussian
 * Splatting map one keyframe at a time (Sec. III-E "Optimization"): the chunks
 * the keyframe sees are found by frustum culling (Sec. III-D "Frustum
 * Culling"), loaded into device memory under an LRU budget (Sec. III-E, "LRU
 * Eviction Strategy"), the visible Gaussians are indexed into one buffer, the
 * rasterizer renders RGB and depth, and the losses of Eqs. (2)-(4) drive an
 * optimiser step.  Each call below is one of those steps.
 *
 * Conventions
 *  - Every call returns a dcgs_status.  No C++ exception or abort crosses the
 *    ABI; after an error dcgs_last_error(ctx) holds a message.
 *  - "device" pointers are HIP device memory (e.g. a torch tensor's
 *    data_ptr()); "host" pointers are CPU memory.  The caller owns every
 *    pointer it passes; the library never frees caller memory.  The context,
 *    render states and pools own their internal scratch.
 *  - `stream` is a hipStream_t passed as void*.  Calls are asynchronous on
 *    it unless marked SYNC (the call waits for the stream and returns after
 *    the work it names is complete).
 *  - A context and everything created from it belong to one host thread and
 *    one device.
 *
 * Parameter block (SoA, float32): rows of length >= n with a row stride
 *    row 0..2   mean x, y, z (world metres)
 *    row 3..5   log-scale of the three local axes
 *    row 6..9   quaternion w, x, y, z (need not be normalised)
 *    row 10     opacity logit
 *    row 11+3k+c  SH coefficient k = l*l + l + m of colour channel c
 *  R = 11 + 3 (deg + 1)^2 rows; deg in {0, 1, 2, 3}.
 *
 * Rendering model (the paper cites 3D Gaussian Splatting for it and states
 * no formula of its own; this library implements this exact reading):
 *  s = exp(log_scale), o = sigmoid(logit), Sigma = R(q/|q|) S S^T R^T;
 *  camera (X, Y, Z) = R_cw mu + t_cw, u = fx X/Z + cx, v = fy Y/Z + cy,
 *  pixel (i, j) centred at (i + .5, j + .5);
 *  Sigma2 = J R_cw Sigma R_cw^T J^T + 0.3 I (EWA, J the pinhole Jacobian);
 *  culled if Z <= z_near, |X/Z| > 1.3 (W/2)/fx, |Y/Z| > 1.3 (H/2)/fy,
 *  o < 1/255 or an empty pixel box; pixel box = axis-aligned box of the
 *  ellipse where o exp(-d^T Sigma2^-1 d / 2) >= 1/255, clipped to the image;
 *  colour = max(sum_k f_k Y_k(d) + 0.5, 0), d from the camera centre to mu,
 *  real orthonormal SH without Condon-Shortley phase;
 *  per pixel, Gaussians whose box holds it in (float32 depth, index) order:
 *  alpha = min(0.99, o e^{-d^T Q d / 2}), skipped below 1/255, compositing
 *  stops before T would fall below 1e-4; C = sum c alpha T + T bg,
 *  D = sum Z alpha T.
 */
#ifndef DCGS_H
#define DCGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum dcgs_status {
  DCGS_OK = 0,
  DCGS_E_INVALID = 1,      /* null pointer, bad size or shape, bad enum    */
  DCGS_E_CAPACITY = 2,     /* an output buffer is too small; see *_required */
  DCGS_E_BUDGET = 3,       /* visible set exceeds the residency budget      */
  DCGS_E_NOT_RESIDENT = 4, /* a chunk id is not resident / not in the pool  */
  DCGS_E_HIP = 5,          /* a HIP runtime call failed                     */
  DCGS_E_RANGE = 6         /* a chunk coordinate outside Eq. (6)'s range   */
} dcgs_status;

typedef struct dcgs_ctx dcgs_ctx;
typedef struct dcgs_state dcgs_state;
typedef struct dcgs_pool dcgs_pool;

/* Pinhole camera, world -> camera.  R is row-major 3x3. */
typedef struct dcgs_camera {
  double R[9];
  double t[3];
  double fx, fy, cx, cy;
  int32_t width, height;
  double z_near, z_far;
} dcgs_camera;

/* Adam settings: learning rate per parameter group (0 means, 1 log-scales,
 * 2 quaternions, 3 opacity logit, 4 SH degree 0, 5 higher SH). */
typedef struct dcgs_adam_config {
  float lr[6];
  float beta1, beta2, eps;
} dcgs_adam_config;

/* ---- context ------------------------------------------------------------ */

/* Library version string (static storage). */
const char *dcgs_version(void);

/* Create a context on HIP device `device`.  *out is set on success. */
int dcgs_create(dcgs_ctx **out, int device);
void dcgs_destroy(dcgs_ctx *ctx);
/* Message of the last failed call on `ctx` (static until the next call). */
const char *dcgs_last_error(const dcgs_ctx *ctx);

/* ---- chunks: Sec. III-D, Eqs. (5) and (6) --------------------------------- */

/* EncodedID of the chunk of each Gaussian: c_i = floor((p_i + s/2)/s)
 * (Eq. 5, float64), ID = (cx+2^20) 2^42 + (cy+2^20) 2^21 + (cz+2^20)
 * (Eq. 6).  mean: device [3][stride]; out_ids: device [n].  A coordinate
 * outside [-2^20, 2^20-1] gives id UINT64_MAX and, SYNC, DCGS_E_RANGE. */
int dcgs_chunk_ids(dcgs_ctx *ctx, const float *mean, int64_t n, int64_t stride,
                   double chunk_size, uint64_t *out_ids, void *stream);

/* Visible chunks (Sec. III-D "Frustum Culling", Sec. III-E): chunk c is
 * visible in a view iff its closed cubic cell [c s - s/2, c s + s/2]^3 meets
 * the closed frustum {z_near <= Z <= z_far, 0 <= u <= W, 0 <= v <= H}
 * (separating-axis test in float64; the paper's hierarchical plane test is
 * a faster route to the same set).  The distance filter is the z_far plane.
 *   cams: host [n_views], 1 <= n_views <= 16
 *   ids:  device [n_chunks] ascending EncodedIDs of the occupied chunks
 *   out_ids: device [n_chunks] visible ids, ascending (union over views)
 *   out_mask: device [n_chunks] bit v set when view v sees the chunk
 *   out_count: device int32, number of visible ids written.
 * Asynchronous on `stream`.  Its scratch belongs to the stream: calls on
 * different streams of one context may overlap (a look-ahead selection on
 * a side stream while the compute stream selects its own view). */
int dcgs_select_chunks(dcgs_ctx *ctx, const dcgs_camera *cams, int n_views,
                       const uint64_t *ids, int n_chunks, double chunk_size,
                       uint64_t *out_ids, uint16_t *out_mask,
                       int32_t *out_count, void *stream);

/* ---- keyframe selection: Sec. III-F ---------------------------------------- */

/* SYNC.  For n_keyframes keyframes (host cameras; keyframe k's position p_k
 * is its camera centre -R^T t, float64, each product and sum rounded in
 * order) and the chunk grid ids (device, as for dcgs_select_chunks):
 *   in_set[k] = 1 when floor(p_k / grid) = floor(p_latest / grid) per axis
 *     (exact floor), i.e. k is in the spatial candidate set K(p_latest) of
 *     Eq. (8), latest the index of the most recently added keyframe;
 *   n_visible[k] = |C_v(k)|, the chunks keyframe k sees (the visibility
 *     test of dcgs_select_chunks);
 *   n_overlap[k] = |C_v(k) & C_active|, C_active = active_ids (host,
 *     n_active, strictly ascending; e.g. the resident chunks);
 *   overlap[k] = n_overlap[k] / n_visible[k] in float64 (Eq. 7), and 1 for
 *     a keyframe that sees no chunk (it needs nothing loaded).
 * window (host int32 [n_window], nullable): the batching window formed from
 * the candidate set, the keyframes of K(p_latest) with the highest overlap,
 * ties to the more recent (higher index) keyframe; *n_window_out gets its
 * size (min(n_window, |K(p_latest)|)).  The paper picks keyframes inside
 * K(p_latest) with CaRtGS's usage-based rule instead, which is not built.
 * Per-keyframe outputs: host arrays [n_keyframes], each nullable.
 * 1 <= n_keyframes <= 65536. */
int dcgs_keyframe_overlap(dcgs_ctx *ctx, const dcgs_camera *keyframes, int n_keyframes,
                          int latest, double grid, const uint64_t *ids, int n_chunks,
                          double chunk_size, const uint64_t *active_ids, int n_active,
                          uint8_t *in_set, int32_t *n_visible, int32_t *n_overlap,
                          double *overlap, int n_window, int32_t *window,
                          int32_t *n_window_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection as dcgs_select_chunks, same arguments and results, but its
 * scratch (one 16-bit view mask per chunk) is a static device array of
 * DCGS_NOALLOC_MAX_CHUNKS entries held by each device until the process
 * ends, so the call allocates nothing (nor does it time itself under
 * dcgs_profile_enable).  n_chunks > DCGS_NOALLOC_MAX_CHUNKS returns
 * DCGS_E_CAPACITY.  Every call on one device shares that array: calls that
 * overlap on one device (two streams, two contexts or two threads at once)
 * race; calls ordered on one stream do not. */
#define DCGS_NOALLOC_MAX_CHUNKS 65536
int dcgs_select_chunks_noalloc(dcgs_ctx *ctx, const dcgs_camera *cams, int n_views,
                               const uint64_t *ids, int n_chunks, double chunk_size,
                               uint64_t *out_ids, uint16_t *out_mask,
                               int32_t *out_count, void *stream);

/* ---- residency pool: Sec. III-E "Optimization" / "LRU Eviction Strategy" --- */

/* A chunk store in pinned host memory plus a device pool holding at most
 * `budget` Gaussians (the paper's VRAM budget, counted in Gaussians).  Each
 * Gaussian carries its parameters, Adam moments m and v, and a step count. */
int dcgs_pool_create(dcgs_ctx *ctx, int sh_degree, int64_t budget,
                     dcgs_pool **out);
void dcgs_pool_destroy(dcgs_pool *pool);

/* SYNC.  Add a scene: params is a HOST parameter block [R][n] (row stride n).
 * Each Gaussian goes to the chunk of Eqs. (5)-(6) (ids computed on the
 * device); within a chunk Gaussians keep their input order.  Moments and
 * steps start at zero.  May be called once per pool. */
int dcgs_pool_ingest(dcgs_pool *pool, const float *params, int64_t n,
                     double chunk_size, void *stream);

/* Occupied chunks in ascending id order.  ids/counts: host, capacity
 * entries; *n_out gets the number of chunks (DCGS_E_CAPACITY if larger). */
int dcgs_pool_chunks(dcgs_pool *pool, uint64_t *ids, int64_t *counts,
                     int capacity, int *n_out);

/* Device array of the occupied chunk ids (ascending), for select_chunks. */
const uint64_t *dcgs_pool_device_ids(dcgs_pool *pool, int *n_out);

/* Make the chunks `ids` (host, n) resident for frame `now`: load = ids \
 * resident; if the budget would be exceeded, evict the evictable (resident,
 * not in ids) chunks oldest access first (ties: lower id), the shortest
 * such prefix that fits, writing their state back to the host store.  The
 * chunks in ids get access time `now`.  DCGS_E_BUDGET if ids alone do not
 * fit (nothing is changed then).  *loaded / *evicted (nullable) get the
 * chunk counts; loads here count as misses (not staged ahead of time).
 * Host-asynchronous: copies run on the pool's own copy stream, and
 * `stream` (the compute stream) waits, device-side, for every chunk in ids;
 * an eviction's copy waits for the compute work of the chunk's last frame.
 * `now` must not decrease from call to call. */
int dcgs_pool_require(dcgs_pool *pool, const uint64_t *ids, int n,
                      int64_t now, int *loaded, int *evicted, void *stream);

/* Stage chunks ahead of need (host-asynchronous, copy stream): each id not
 * resident is loaded, in the given order, after evicting chunks that were
 * not used in frame `now` and are not in ids (oldest first) to make room;
 * staging stops at the first chunk that does not fit.  Staged chunks get access time `now`.  *staged
 * (nullable) gets the number staged.  A later require() of a staged chunk
 * counts as a hit and only waits for its copy event. */
int dcgs_pool_prefetch(dcgs_pool *pool, const uint64_t *ids, int n,
                       int64_t now, int *staged, void *stream);

/* Counters: out[0..7] = loads, evictions, prefetched, misses, hits, bytes
 * host->device, bytes device->host, Gaussians resident (first n_out). */
int dcgs_pool_stats(dcgs_pool *pool, int64_t *out, int n_out);

/* SYNC (waits for the device).  Current state of one chunk (from the
 * device if resident, else the host store), into host arrays params/m/v
 * [R][count] and step [count]; any of them may be null. */
int dcgs_pool_read_chunk(dcgs_pool *pool, uint64_t id, float *params,
                         float *m, float *v, int32_t *step);

/* Resident chunk ids (host, capacity) and Gaussians resident. */
int dcgs_pool_resident(dcgs_pool *pool, uint64_t *ids, int capacity,
                       int *n_out, int64_t *gaussians_out);

/* ---- loop closure: Sec. III-G ----------------------------------------------- */

/* SYNC.  Correct the store after a loop closure.
 *  "Cross-Chunk Transformation": for the affected keyframes in order
 *  (keyframes: host [n_keyframes] cameras, any count), the chunks each one
 *  sees (the visibility test of dcgs_select_chunks) take that keyframe's
 *  rigid correction, a chunk seen by several taking the first one's (the
 *  global transformation mask).  corrections: host float64
 *  [n_keyframes][12], a row-major rotation R (9) then a translation t (3),
 *  mapping old world coordinates to corrected ones.  Each Gaussian of such a
 *  chunk gets mean <- R mean + t (float64, each product and sum rounded, no
 *  fused multiply-add, then rounded to float32) and quaternion <- q_R (x) q
 *  (Hamilton product, q_R the unit quaternion of R with w >= 0); its other
 *  parameters and its Adam state are kept.
 *  "Chunk Redistribution": a corrected Gaussian moves to the chunk of its
 *  new mean (Eqs. 5-6); every other Gaussian stays in its chunk.  Chunks
 *  stay in ascending id order; inside a chunk, Gaussians keep the previous
 *  order (old chunk id, then position).
 *  "Post-Correction Refinement": every Gaussian of the chunks (after
 *  redistribution) that a junction camera sees (junctions: host
 *  [n_junctions]) gets its opacity logit set to min(logit, logit(0.01))
 *  (float32 of log(0.01/0.99)), its moments m, v and its step set to 0.
 * All affected chunks are processed in one batch on the device: it needs
 * room for about two copies of them (parameters and Adam state) besides the
 * pool.  The rebuilt chunks are written to a new pinned host block and are
 * not resident afterwards; chunks that lost all their Gaussians disappear.
 * stats (host, first n_stats of 7, nullable): affected chunks, corrected
 * Gaussians, corrected Gaussians that changed chunk, chunks rebuilt (taken
 * apart), chunks written, Gaussians reset, chunks in the store afterwards.
 * DCGS_E_RANGE if a corrected mean leaves the Eq. (6) range or the batch
 * holds 2^32 slots or more (the store is unchanged then). */
int dcgs_pool_loop_closure(dcgs_pool *pool, const dcgs_camera *keyframes,
                           const double *corrections, int n_keyframes,
                           const dcgs_camera *junctions, int n_junctions, int64_t *stats,
                           int n_stats, void *stream);

/* ---- compaction: Sec. III-E ("index only the visible Gaussians") ---------- */

/* Concatenate the Gaussians of the resident chunks `ids` (host, n_ids, any
 * order; processed ascending) into out [R][out_stride] (device) and write
 * each one's pool slot to out_src (device int32).  Optional out_gmask
 * (device uint16 [n]) gets the view mask of the Gaussian's chunk taken from
 * masks (host uint16 [n_ids], parallel to ids; null -> all ones).  *n_out
 * (host) gets the number of Gaussians; DCGS_E_CAPACITY if > capacity;
 * DCGS_E_NOT_RESIDENT if a chunk is not resident. */
int dcgs_compact(dcgs_pool *pool, const uint64_t *ids, const uint16_t *masks,
                 int n_ids, float *out, int64_t out_stride, int32_t *out_src,
                 uint16_t *out_gmask, int64_t capacity, int64_t *n_out,
                 void *stream);

/* ---- differentiable rendering ------------------------------------------- */

/* A render state holds what a backward pass needs from its forward: per
 * Gaussian projection records, the depth order, the (tile, Gaussian) pairs
 * sorted by (tile, float32 depth bits, index), per-tile ranges, and per
 * pixel the final transmittance and the position of the last composited
 * Gaussian.  A state serves one forward/backward pair at a time. */
int dcgs_state_create(dcgs_ctx *ctx, dcgs_state **out);
void dcgs_state_destroy(dcgs_state *st);

/* SYNC (reads the pair count back once).  Render n_views views of one
 * parameter block in single launches (the batched window of a mapping
 * step; n_views = 1 is the plain per-view render).
 *   params: device [R][stride], n Gaussians, SH degree sh_degree
 *   gmask: device uint16 [n] or null: Gaussian i is drawn in view v only when
 *          bit v + mask_shift is set (the view mask of its chunk); null draws
 *          all Gaussians in all views.  mask_shift lets view k of a window be
 *          rendered alone from the window's compacted buffer.
 *   cams: host [n_views], 1 <= n_views <= 16, all of one width and height
 *   bg: host float[3]
 *   raster shape: tile_w x tile_h pixels per workgroup, pixels_per_lane
 *   pixels per lane (one in each of that many 8x8 cells of the tile);
 *   supported (16,16,{1,2,4}),
 *   (8,8,1), (32,16,{2,4,8}); pixels_per_lane 0 picks 2, 1 and 4.  Bits
 *   0-3 of pixels_per_lane are the forward's, bits 4-7 the backward's
 *   (0: the forward's), so the two rasters of one tile size may map pixels
 *   to lanes differently.  The image does not depend on the shape (each
 *   pixel composites only the Gaussians whose pixel box holds it), nor on
 *   the other views.
 *   rgb: device [n_views][3][H][W]; depth: device [n_views][H][W];
 *   T: device [n_views][H][W] or null.
 * Outputs are overwritten.  The state keeps what render_bwd needs.
 * DCGS_E_CAPACITY when the (tile, Gaussian) pairs, counted in 64 bits,
 * exceed 2^31 - 1 (see dcgs_pairs_fit); the state then holds no forward and
 * render_bwd on it fails with DCGS_E_INVALID. */
int dcgs_render_fwd(dcgs_ctx *ctx, dcgs_state *st, const float *params,
                    int64_t n, int64_t stride, int sh_degree,
                    const uint16_t *gmask, int mask_shift,
                    const dcgs_camera *cams, int n_views, const float *bg,
                    int tile_w, int tile_h,
                    int pixels_per_lane, float *rgb, float *depth, float *T,
                    void *stream);

/* Backward of the last render_fwd on `st` (same params): the adjoint of the
 * compositing runs back to front from each pixel's last composited Gaussian,
 * recovering each earlier transmittance by division, then chains through
 * the projection to the raw parameters, summing the views in view order
 * (float32 additions in the same order as one single-view backward per
 * view accumulating into grad).  Deterministic: no float atomics.
 *   dl_drgb: device [n_views][3][H][W]; dl_ddepth: device [n_views][H][W]
 *   or null
 *   grad: device [R][grad_stride]; accumulate != 0 adds into it, 0
 *   overwrites rows for all n Gaussians (culled ones get 0).
 *   grad2d: device [10][n_views * n] or null: per record (view v, Gaussian
 *   i at v * n + i) dL/d(u, v, Q00, Q01, Q11, o, r, g, b, Z) of the
 *   screen-space record (Q01 counted once). */
int dcgs_render_bwd(dcgs_ctx *ctx, dcgs_state *st, const float *params,
                    int64_t n, int64_t stride, const float *dl_drgb,
                    const float *dl_ddepth, float *grad, int64_t grad_stride,
                    int accumulate, float *grad2d, void *stream);

/* Eqs. (2)-(4) without SSIM over `count` values: dl_drgb = sign(rgb -
 * target) / norm (0 at equality), so norm = 3HW gives the mean over one
 * image and, for n_views images in one buffer, the sum over views of each
 * view's mean; stats (device double[2]) gets sum |rgb - target| and the sum
 * of squared error with rgb clipped to [0, 1] (for PSNR). */
int dcgs_loss_l1(dcgs_ctx *ctx, const float *rgb, const float *target,
                 int64_t count, double norm, float *dl_drgb, double *stats,
                 void *stream);

/* ---- optimiser: per-Gaussian Adam state (Sec. III-G resets it) ----------- */

/* One Adam step for the n compacted Gaussians: row r of grad (device
 * [R][grad_stride]) updates pool slot src[i] (device int32) in place:
 * t += 1, m, v moments, bias-corrected update with the group learning rate.
 * Every listed Gaussian is updated (zero gradients included). */
int dcgs_adam_step(dcgs_pool *pool, const int32_t *src, const float *grad,
                   int64_t n, int64_t grad_stride,
                   const dcgs_adam_config *cfg, void *stream);

/* The full mapping loss, Eqs. (2)-(4), for n_views images in one buffer:
 * per view (1 - lambda_s) |I - I_gt|_1 + lambda_s (1 - SSIM(I, I_gt))
 * + lambda_depth |D - D_gt|_1, summed over views; |.|_1 is the mean over
 * the view's 3HW colour (HW depth) values; SSIM is the mean over the 3HW
 * values of the per-pixel SSIM with an 11-tap Gaussian window (sigma 1.5,
 * separable, zero padding outside the image), C1 = 0.01^2, C2 = 0.03^2,
 * each colour channel on its own.  rgb, target, dl_drgb: [V][3][H][W];
 * depth, depth_target, dl_ddepth: [V][H][W] (all three nullable when
 * lambda_depth = 0; dl_ddepth alone nullable otherwise).  dl_drgb and
 * dl_ddepth are written (not accumulated).  stats (device double[4]): sum
 * |rgb - target|, sum of squared error with rgb clipped to [0, 1], sum of
 * the per-pixel SSIM, sum |depth - depth_target|; the loss is
 * (1 - lambda_s) s0 / (3HW) + lambda_s (V - s2 / (3HW)) + lambda_depth s3 / (HW).
 * Scratch is owned by ctx.  Deterministic. */
int dcgs_loss_mapping(dcgs_ctx *ctx, const float *rgb, const float *target, const float *depth,
                      const float *depth_target, int n_views, int height, int width,
                      double lambda_s, double lambda_depth, float *dl_drgb, float *dl_ddepth,
                      double *stats, void *stream);

/* The LoG sampling map of the Sampling section: P_s = max(P_L - P~, 0)
 * with P_L = min(1, beta |LoG(image)|) and P~ = min(1, beta |LoG(render)|),
 * |.| the Euclidean norm over colour channels of the per-channel LoG (sum
 * of the second-derivative Gaussian filters along rows and columns, sigma
 * in px, radius ceil(4 sigma) <= 12, mirror boundary with the edge sample
 * repeated).  image, render: [3][H][W]; u: [H][W] uniform draws (the
 * caller's); ps (nullable): [H][W] the map; out_idx [H*W]: indices y*W + x
 * of the pixels with u < P_s in raster order; out_count (device int32)
 * their number.  Scratch is owned by ctx. */
int dcgs_sample_pixels(dcgs_ctx *ctx, const float *image, const float *render, const float *u,
                       int height, int width, double beta, double sigma, float *ps,
                       int32_t *out_idx, int32_t *out_count, void *stream);

/* ---- autotuner ----------------------------------------------------------- */

/* SYNC.  Time the forward and the backward pass of every supported raster
 * shape (tile_w, tile_h, pixels_per_lane) on the given window (same
 * arguments as dcgs_render_fwd; one warm pass, then the fastest of three
 * timed passes per shape), keep the tile size whose fastest forward plus
 * fastest backward is smallest, with those two pixels-per-lane values
 * packed as in dcgs_render_fwd (out_shape[2]), and remember it in ctx
 * for windows of the same width, height, view count and size class
 * (ceil(log2(n))).  A cached answer returns at once unless force != 0.
 * Images do not depend on the shape.  Scratch images and gradients are
 * owned by ctx.  out_shape: host int[3]; times_ms: host double[n_shapes]
 * or null (filled only when shapes are timed); *n_shapes (host, nullable)
 * gets the number of shapes. */
int dcgs_autotune(dcgs_ctx *ctx, dcgs_state *st, const float *params,
                  int64_t n, int64_t stride, int sh_degree,
                  const uint16_t *gmask, const dcgs_camera *cams, int n_views,
                  int force, int *out_shape, double *times_ms, int *n_shapes,
                  void *stream);

/* ---- graph-captured mapping window ---------------------------------------- */
/*
 * One batched mapping iteration over a window of keyframes (Sec. III-E
 * "Optimization", one Adam step per window): compaction of the window's
 * chunks (a kernel launched before the graph), then one HIP graph holding
 * the projection, depth sort, pair emission, tile sort, ranges, forward
 * raster, L1 loss, backward raster, projection backward and the Adam step
 * into the pool.  The graph is recorded once at creation; each launch
 * replays it.  Results equal dcgs_render_fwd + dcgs_loss_l1 +
 * dcgs_render_bwd + dcgs_adam_step on the same window bit for bit.
 *
 * Grids are sized for `capacity` Gaussians and `pair_capacity` (tile,
 * Gaussian) pairs; the kernels read the real counts on the device.  A
 * window whose pairs exceed pair_capacity draws nothing and leaves the pool
 * unchanged, and so does every later launch: the next launch that reuses
 * its staging block (two launches later), or dcgs_window_sync, returns
 * DCGS_E_CAPACITY with the pair count needed; rebuild the window with a
 * larger pair_capacity and launch the skipped windows again, in order.
 * All buffers are caller-owned device memory that must stay valid while the
 * window exists; `targets` is read at every launch (write the window's
 * targets into it, on the launch stream, before launching).
 */
typedef struct dcgs_window dcgs_window;

typedef struct dcgs_window_config {
  int sh_degree;                 /* must equal the pool's */
  int width, height, n_views;    /* every camera of a launch has this size; 1..16 views */
  int tile_w, tile_h, pixels_per_lane;  /* a supported raster shape, backward's pixels per
                                           lane in bits 4-7 (see dcgs_render_fwd) */
  int64_t capacity;              /* Gaussians: row stride of params and grad;
                                    capacity * n_views < 2^31 */
  int64_t pair_capacity;         /* (tile, Gaussian) pairs, < 2^31 */
  float bg[3];
  double loss_norm;              /* the L1 loss is sum |rgb - target| / loss_norm */
  dcgs_adam_config adam;
  float *params, *grad;          /* [R][capacity] */
  int32_t *src;                  /* [capacity] pool slot of each compacted Gaussian */
  uint16_t *gmask;               /* [capacity] view mask of each compacted Gaussian */
  float *rgb, *depth, *dl_drgb;  /* [V][3][H][W], [V][H][W], [V][3][H][W] */
  const float *targets;          /* [V][3][H][W] */
  double *stats;                 /* sum |d| and sum d^2 of the last launch ([2]); with
                                    the full loss, the four sums of dcgs_loss_mapping ([4]) */
  /* The full mapping loss of Eqs. (2)-(4) inside the graph (dcgs_loss_mapping's
   * terms and normalisation, loss_norm unused) when lambda_s > 0 or
   * lambda_depth > 0; both 0 keeps the L1 loss above. */
  double lambda_s, lambda_depth;
  const float *depth_targets;    /* [V][H][W], read at every launch; needed when
                                    lambda_depth > 0 */
  float *dl_ddepth;              /* [V][H][W] when lambda_depth > 0 */
} dcgs_window_config;

/* SYNC.  Allocate the window's buffers and record its two graph instances. */
int dcgs_window_create(dcgs_ctx *ctx, dcgs_pool *pool, const dcgs_window_config *cfg,
                       dcgs_window **out);
/* Waits for launched work, then frees the window. */
void dcgs_window_destroy(dcgs_window *win);

/* Enqueue one window on `stream`: compaction of the chunks ids (host,
 * n_ids, ascending, resident: call dcgs_pool_require first) with view masks
 * masks (host), then the graph, for the n_views host cameras cams.
 * *n_active (nullable) gets the compacted count.  Host-asynchronous except
 * that it waits for the launch two windows back (its staging block) and
 * reports DCGS_E_CAPACITY if that or any later launch overflowed. */
int dcgs_window_launch(dcgs_window *win, const uint64_t *ids, const uint16_t *masks, int n_ids,
                       const dcgs_camera *cams, int64_t *n_active, void *stream);

/* SYNC.  Wait for every launch; DCGS_E_CAPACITY if one overflowed, with
 * *pairs_required (nullable) = the pair count that did not fit and *skipped
 * (nullable) = how many of the most recent launches (0..2) changed nothing
 * and must be launched again after a rebuild.  After DCGS_E_CAPACITY every
 * further launch fails until the window is rebuilt. */
int dcgs_window_sync(dcgs_window *win, int64_t *pairs_required, int *skipped);

/* SYNC.  Pair count of the last completed launch. */
int dcgs_window_pairs(dcgs_window *win, int64_t *n_pairs);

/* ---- learned chunk prefetch --------------------------------------------- */
/*
 * Not part of the paper's method: the paper selects chunks by the exact
 * frustum test of the current frame (Sec. III-D "Frustum Culling") and
 * loads the missing ones (Sec. III-E "Optimization"); these calls predict,
 * from the last 8 camera poses, which cells that test will select in the
 * next frames, so that their staging (dcgs_pool_prefetch) starts early.
 * The exact test stays in charge: a needed chunk that was not staged is
 * loaded by dcgs_pool_require.
 *
 * Candidates of frame t: the 64 x 64 cells (Eq. 5) of the horizontal layer
 * holding the camera centre c0, candidate q = j*64 + i at cell
 * (bx + i - 32, by + j - 32, bz).  Input row (59 floats): for history entry
 * k = 0..7 (frame max(t-k, 0)), R0 (c_k - c0) / pos_unit and the unit
 * quaternion (w, x, y, z), w >= 0, of R0 R_k^T (R = world-to-camera
 * rotation); then R0 (cell_centre - c0) / (8 s).
 *
 * Network: 59 -> 256 -> 256 -> 1, z1 = W1 x + b1, h1 = GELU(z1) (exact erf
 * form), z2 = W2 h1 + b2, h2 = GELU(z2), logit = w3 . h2 + b3.  theta: the
 * float32 master vector of DCGS_MLP_PARAMS values, W1 [256][59] row-major,
 * b1 [256], W2 [256][256], b2 [256], w3 [256], b3 [1].  wbf16: the
 * bfloat16 copy (raw bits) of W1, W2, w3 back to back (DCGS_MLP_BF16
 * values); the forward and backward use these weights and the float32
 * biases, accumulating in float32 on the matrix cores.  All arrays are
 * device memory owned by the caller unless stated otherwise.
 */
#define DCGS_MLP_PARAMS 81409
#define DCGS_MLP_BF16 80896
#define DCGS_PREFETCH_CANDIDATES 4096
#define DCGS_PREFETCH_IN 59
#define DCGS_PREFETCH_HIDDEN 256

/* labels [n_frames][4096] (uint8): 1 when candidate q of frame t meets the
 * frustum of one of frames t+1 .. t+horizon (1 <= horizon <= 16), else 0.
 * cams: host array of the whole trajectory (copied through the context's
 * pinned staging; the call waits for the previous staging copy). */
int dcgs_prefetch_labels(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames, int horizon,
                         double chunk_size, uint8_t *labels, void *stream);

/* Input rows for the frames listed in `frames` (host int32, n_sel <= 65535,
 * each in [0, n_frames)): X [n_sel][4096][59] float32; cell_ids (nullable)
 * [n_sel][4096] EncodedIDs (all ones for cells outside Eq. 6's range);
 * y (nullable, requires labels) [n_sel][4096] = labels[frame][q]. */
int dcgs_prefetch_features(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames,
                           const int32_t *frames, int n_sel, double chunk_size, double pos_unit,
                           const uint8_t *labels, float *X, uint64_t *cell_ids, uint8_t *y,
                           void *stream);

/* Forward of n rows of X [n][59] (n <= 4194240): z1, h1, z2, h2 [n][256] and
 * logit [n], all written. */
int dcgs_mlp_forward(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16, const float *X,
                     int64_t n, float *z1, float *h1, float *z2, float *h2, float *logit,
                     void *stream);

/* Gradient of the weighted binary cross-entropy, mean over the n rows of
 * pos_weight * y * softplus(-logit) + (1 - y) * softplus(logit), with
 * respect to theta (the weights' gradient taken at their bfloat16 values),
 * written (not accumulated) to grad [DCGS_MLP_PARAMS].  Inputs are the
 * forward's outputs for the same X; y [n] uint8 (0 or 1).  loss (device
 * double, nullable) gets the loss.  Reductions run in a fixed order
 * (deterministic).  Scratch is owned by ctx. */
int dcgs_mlp_backward(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16, const float *X,
                      const float *z1, const float *h1, const float *z2, const float *h2,
                      const float *logit, const uint8_t *y, int64_t n, float pos_weight,
                      float *grad, double *loss, void *stream);

/* One Adam step (step >= 1 counts from 1) on theta with moments m, v
 * [DCGS_MLP_PARAMS] (float32, updated in place; arithmetic in float64 with
 * bias corrections 1 - beta^step), then wbf16 = theta's weights rounded to
 * bfloat16 (nearest, ties to even). */
int dcgs_mlp_adam(dcgs_ctx *ctx, float *theta, uint16_t *wbf16, float *m, float *v,
                  const float *grad, int64_t step, double lr, double beta1, double beta2,
                  double eps, void *stream);

/* wbf16 = theta's weights rounded to bfloat16 (nearest, ties to even); for
 * a freshly initialised or loaded theta. */
int dcgs_mlp_round(dcgs_ctx *ctx, const float *theta, uint16_t *wbf16, void *stream);

/* Inference for the current frame: history = host array of the last 8
 * cameras, history[0] the current one, history[k] k frames back.  Writes
 * the EncodedIDs of the candidates with logit >= threshold_logit, in
 * candidate order, to out_ids [4096] and their number to out_count (device
 * int32); out_logit (nullable) [4096] gets every candidate's logit.
 * Scratch is owned by ctx. */
int dcgs_prefetch_predict(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16,
                          const dcgs_camera *history, double chunk_size, double pos_unit,
                          float threshold_logit, uint64_t *out_ids, int32_t *out_count,
                          float *out_logit, void *stream);

/* ---- stage timers -------------------------------------------------------- */

/* Stages timed with HIP events recorded on the stream each kernel runs on. */
typedef enum dcgs_stage {
  DCGS_STAGE_SELECT = 0,       /* chunk visibility + compaction of ids      */
  DCGS_STAGE_COMPACT = 1,      /* gather of active chunks into one buffer   */
  DCGS_STAGE_PREPROCESS = 2,   /* projection records                        */
  DCGS_STAGE_DEPTH_SORT = 3,   /* radix sort of Gaussians by depth key      */
  DCGS_STAGE_SCAN_EMIT = 4,    /* pair offsets + pair emission              */
  DCGS_STAGE_TILE_SORT = 5,    /* radix sort of pairs by tile               */
  DCGS_STAGE_RANGES = 6,       /* per-tile [start, end)                     */
  DCGS_STAGE_RASTER_FWD = 7,   /* front-to-back compositing                 */
  DCGS_STAGE_LOSS = 8,         /* L1 loss and its gradient                  */
  DCGS_STAGE_RASTER_BWD = 9,   /* back-to-front adjoint                     */
  DCGS_STAGE_PREPROCESS_BWD = 10, /* projection backward                    */
  DCGS_STAGE_ADAM = 11,        /* optimiser step into the pool              */
  DCGS_STAGE_COUNT = 12
} dcgs_stage;

/* Enable (1) or disable (0) stage timing on ctx; enabling clears totals. */
int dcgs_profile_enable(dcgs_ctx *ctx, int enable);

/* SYNC.  Totals since enabling: ms[s] summed milliseconds and calls[s]
 * launches of stage s, for s < n_stages (<= DCGS_STAGE_COUNT); either may
 * be null.  Totals are then cleared. */
int dcgs_profile_read(dcgs_ctx *ctx, double *ms, int64_t *calls, int n_stages);

/* ---- inspection (for tests and tools) ------------------------------------ */

/* The overflow decision every forward takes on its (tile, Gaussian) pair
 * count, summed in 64 bits on the device: DCGS_OK when n_pairs fits both
 * pair_capacity (a window's pair buffers; INT64_MAX for an eager forward,
 * whose buffers are sized after the count) and the 2^31 - 1 limit of the
 * 32-bit pair indexing, else DCGS_E_CAPACITY.  Host only, no device. */
int dcgs_pairs_fit(int64_t n_pairs, int64_t pair_capacity);

/* Sizes of the last forward on st: Gaussians, pairs, tiles in x and y. */
int dcgs_state_info(const dcgs_state *st, int64_t *n, int64_t *n_pairs,
                    int32_t *tiles_x, int32_t *tiles_y);

/* SYNC.  Work of the last forward (a measurement, outside the hot path):
 * *walk = sum over pixels of the list positions its compositing walked
 * (tile start to its last contributor), *inbox = how many of those had the
 * pixel inside the record's pixel box (the (pixel, Gaussian) evaluations
 * the raster kernels cannot skip). */
int dcgs_state_work(const dcgs_state *st, int64_t *walk, int64_t *inbox, void *stream);

/* Copy results of the last forward into device buffers (null to skip):
 *   keys [n_pairs] uint64 (tile << 32 | float32 depth bits), values [n_pairs]
 *   int32 Gaussian index, ranges [tiles][2] int32, counts [n] int32 tiles
 *   touched per Gaussian, records [10][n] float (u, v, Q00, Q01, Q11, o, r,
 *   g, b, Z), box [4][n] int32 (i0, i1, j0, j1; culled: count 0), last
 *   [H][W] int32 (position in the sorted pairs, -1 if none). */
int dcgs_state_export(const dcgs_state *st, uint64_t *keys, int32_t *values,
                      int32_t *ranges, int32_t *counts, float *records,
                      int32_t *box, int32_t *last, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* DCGS_H */
