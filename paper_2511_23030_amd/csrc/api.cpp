// C ABI of libdcgs: argument checks, error capture, and dispatch to the
// kernels and the host runtime.  No C++ exception leaves this file.
#include <cstring>
#include <mutex>

#include "internal.h"

namespace dcgs {
void pool_create(dcgs_ctx *ctx, int deg, int64_t budget, dcgs_pool **out);
void pool_destroy(dcgs_pool *p);
void pool_ingest(dcgs_pool *p, const float *params, int64_t n, double s, hipStream_t st);
void pool_require(dcgs_pool *p, const uint64_t *ids, int n, int64_t now, int *loaded,
                  int *evicted, hipStream_t st);
void pool_prefetch(dcgs_pool *p, const uint64_t *ids, int n, int64_t now, int *staged,
                   hipStream_t st);
void pool_read_chunk(dcgs_pool *p, uint64_t id, float *params, float *m, float *v,
                     int32_t *step);
void pool_compact(dcgs_pool *p, const uint64_t *ids, const uint16_t *masks, int n_ids,
                  float *out, int64_t out_stride, int32_t *out_src, uint16_t *out_gmask,
                  int64_t capacity, int64_t *n_out, hipStream_t st);
}  // namespace dcgs

namespace dcgs {
hipEvent_t take_event(dcgs_ctx *ctx) noexcept {
  if (!ctx->spare_events.empty()) {
    hipEvent_t e = ctx->spare_events.back();
    ctx->spare_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace dcgs

namespace {

// Scratch of dcgs_select_chunks_noalloc: the per-chunk view masks that the
// visibility kernel writes and the compaction kernel reads, for at most
// DCGS_NOALLOC_MAX_CHUNKS chunks (128 KB).  Each device holds its own copy
// until the process ends.  On the host the array's name is not a device
// address: the address is looked up once per device (with that device
// current) when a context is created there, and only that pointer is used.
__device__ __align__(256) uint16_t scratch[DCGS_NOALLOC_MAX_CHUNKS];

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
uint16_t *g_scratch[kScratchDevices] = {};

// The device address of `scratch` on the current device `device`.
uint16_t *scratch_address(int device) {
  DCGS_CHECK(device >= 0 && device < kScratchDevices, DCGS_E_INVALID,
             "device index out of range for the no-allocation scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    void *p = nullptr;
    DCGS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DCGS_CHECK(p != nullptr, DCGS_E_HIP, "no device address for the no-allocation scratch");
    g_scratch[device] = static_cast<uint16_t *>(p);
  }
  return g_scratch[device];
}

template <typename F>
int guarded(dcgs_ctx *ctx, F &&f) {
  try {
    f();
    if (ctx) ctx->err.clear();
    return DCGS_OK;
  } catch (const dcgs::Error &e) {
    if (ctx) ctx->err = e.msg;
    return e.status;
  } catch (const std::exception &e) {
    if (ctx) ctx->err = e.what();
    return DCGS_E_HIP;
  } catch (...) {
    if (ctx) ctx->err = "unknown error";
    return DCGS_E_HIP;
  }
}

inline hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

void check_cam(const dcgs_camera *c) {
  DCGS_CHECK(c != nullptr, DCGS_E_INVALID, "null camera");
  DCGS_CHECK(c->width > 0 && c->height > 0 && c->width < 65536 && c->height < 65536,
             DCGS_E_INVALID, "camera size out of range");
  DCGS_CHECK(c->fx > 0 && c->fy > 0 && c->z_near > 0 && c->z_far > c->z_near, DCGS_E_INVALID,
             "camera intrinsics or clip planes invalid");
}

}  // namespace

extern "C" {

const char *dcgs_version(void) { return "dcgs 0.1 gfx950"; }

int dcgs_create(dcgs_ctx **out, int device) {
  if (!out) return DCGS_E_INVALID;
  *out = nullptr;
  auto *ctx = new dcgs_ctx();
  int st = guarded(ctx, [&] {
    DCGS_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    DCGS_HIP(hipGetDeviceProperties(&prop, device));
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    ctx->noalloc_scratch = scratch_address(device);
  });
  if (st != DCGS_OK) {
    delete ctx;
    return st;
  }
  *out = ctx;
  return DCGS_OK;
}

void dcgs_destroy(dcgs_ctx *ctx) {
  if (!ctx) return;
  for (auto &m : ctx->marks) {
    (void)hipEventDestroy(m.a);
    (void)hipEventDestroy(m.b);
  }
  for (auto e : ctx->spare_events) (void)hipEventDestroy(e);
  if (ctx->pf.staged) {
    (void)hipEventSynchronize(ctx->pf.staged);
    (void)hipEventDestroy(ctx->pf.staged);
  }
  if (ctx->pf.pinned) (void)hipHostFree(ctx->pf.pinned);
  delete ctx;
}

const char *dcgs_last_error(const dcgs_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int dcgs_chunk_ids(dcgs_ctx *ctx, const float *mean, int64_t n, int64_t stride, double chunk_size,
                   uint64_t *out_ids, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(n >= 0 && stride >= n && chunk_size > 0 && (n == 0 || (mean && out_ids)),
               DCGS_E_INVALID, "chunk_ids: bad args");
    int *flag = ctx->flag.need(1);
    DCGS_HIP(hipMemsetAsync(flag, 0, sizeof(int), S(stream)));
    dcgs::launch_chunk_ids(mean, n, stride, chunk_size, out_ids, flag, S(stream));
    int h = 0;
    DCGS_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, S(stream)));
    DCGS_HIP(hipStreamSynchronize(S(stream)));
    DCGS_CHECK(h == 0, DCGS_E_RANGE, "chunk_ids: coordinate outside the range of Eq. (6)");
  });
}

int dcgs_select_chunks(dcgs_ctx *ctx, const dcgs_camera *cams, int n_views, const uint64_t *ids,
                       int n_chunks, double chunk_size, uint64_t *out_ids, uint16_t *out_mask,
                       int32_t *out_count, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(cams && n_views >= 1 && n_views <= dcgs::kMaxViews, DCGS_E_INVALID,
               "select_chunks: 1..16 views required");
    for (int v = 0; v < n_views; ++v) check_cam(&cams[v]);
    DCGS_CHECK(n_chunks >= 0 && chunk_size > 0 && out_count &&
                   (n_chunks == 0 || (ids && out_ids && out_mask)),
               DCGS_E_INVALID, "select_chunks: bad buffers");
    uint16_t *tmp;
    {
      std::lock_guard<std::mutex> lock(ctx->sel_mu);
      auto &buf = ctx->sel_mask[stream];
      if (!buf) buf = std::make_unique<dcgs::DevBuf<uint16_t>>();
      tmp = buf->need((size_t)n_chunks + 1);
    }
    dcgs::StageTimer tm(ctx, DCGS_STAGE_SELECT, S(stream));
    dcgs::launch_select(cams, n_views, ids, n_chunks, chunk_size, tmp, out_ids, out_mask,
                        out_count, S(stream));
  });
}

int dcgs_keyframe_overlap(dcgs_ctx *ctx, const dcgs_camera *keyframes, int n_keyframes,
                          int latest, double grid, const uint64_t *ids, int n_chunks,
                          double chunk_size, const uint64_t *active_ids, int n_active,
                          uint8_t *in_set, int32_t *n_visible, int32_t *n_overlap,
                          double *overlap, int n_window, int32_t *window,
                          int32_t *n_window_out, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(keyframes && n_keyframes >= 1 && n_keyframes <= 65536 && latest >= 0 &&
                   latest < n_keyframes && grid > 0,
               DCGS_E_INVALID, "keyframe_overlap: 1..65536 keyframes, latest among them, grid > 0");
    for (int k = 0; k < n_keyframes; ++k) check_cam(&keyframes[k]);
    DCGS_CHECK(n_chunks >= 0 && chunk_size > 0 && (n_chunks == 0 || ids) && n_active >= 0 &&
                   (n_active == 0 || active_ids),
               DCGS_E_INVALID, "keyframe_overlap: bad chunk arrays");
    for (int i = 1; i < n_active; ++i)
      DCGS_CHECK(active_ids[i - 1] < active_ids[i], DCGS_E_INVALID,
                 "keyframe_overlap: active ids must be strictly ascending");
    DCGS_CHECK(n_window >= 0 && (n_window == 0 || window), DCGS_E_INVALID,
               "keyframe_overlap: bad window buffer");
    dcgs::keyframe_overlap(ctx, keyframes, n_keyframes, latest, grid, ids, n_chunks, chunk_size,
                           active_ids, n_active, in_set, n_visible, n_overlap, overlap, n_window,
                           window, n_window_out, S(stream));
  });
}

int dcgs_select_chunks_noalloc(dcgs_ctx *ctx, const dcgs_camera *cams, int n_views,
                               const uint64_t *ids, int n_chunks, double chunk_size,
                               uint64_t *out_ids, uint16_t *out_mask, int32_t *out_count,
                               void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(cams && n_views >= 1 && n_views <= dcgs::kMaxViews, DCGS_E_INVALID,
               "select_chunks_noalloc: 1..16 views required");
    for (int v = 0; v < n_views; ++v) check_cam(&cams[v]);
    DCGS_CHECK(n_chunks >= 0 && chunk_size > 0 && out_count &&
                   (n_chunks == 0 || (ids && out_ids && out_mask)),
               DCGS_E_INVALID, "select_chunks_noalloc: bad buffers");
    DCGS_CHECK(n_chunks <= DCGS_NOALLOC_MAX_CHUNKS, DCGS_E_CAPACITY,
               "select_chunks_noalloc: " + std::to_string(n_chunks) +
                   " chunks exceed its scratch of " + std::to_string(DCGS_NOALLOC_MAX_CHUNKS) +
                   " (use dcgs_select_chunks)");
    DCGS_CHECK(ctx->noalloc_scratch != nullptr, DCGS_E_INVALID,
               "select_chunks_noalloc: context without scratch");
    // the same kernels as dcgs_select_chunks; every mask entry the compaction
    // reads is written first, so nothing needs clearing.  No stage timer (its
    // events may be created on first use).
    dcgs::launch_select(cams, n_views, ids, n_chunks, chunk_size, ctx->noalloc_scratch, out_ids,
                        out_mask, out_count, S(stream));
  });
}

int dcgs_pool_create(dcgs_ctx *ctx, int sh_degree, int64_t budget, dcgs_pool **out) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] { dcgs::pool_create(ctx, sh_degree, budget, out); });
}

void dcgs_pool_destroy(dcgs_pool *pool) { dcgs::pool_destroy(pool); }

int dcgs_pool_ingest(dcgs_pool *pool, const float *params, int64_t n, double chunk_size,
                     void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] { dcgs::pool_ingest(pool, params, n, chunk_size, S(stream)); });
}

int dcgs_pool_chunks(dcgs_pool *pool, uint64_t *ids, int64_t *counts, int capacity, int *n_out) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] {
    DCGS_CHECK(n_out, DCGS_E_INVALID, "pool_chunks: null n_out");
    *n_out = (int)pool->chunks.size();
    DCGS_CHECK((int)pool->chunks.size() <= capacity, DCGS_E_CAPACITY, "pool_chunks: capacity");
    for (size_t c = 0; c < pool->chunks.size(); ++c) {
      if (ids) ids[c] = pool->chunks[c].id;
      if (counts) counts[c] = pool->chunks[c].n;
    }
  });
}

const uint64_t *dcgs_pool_device_ids(dcgs_pool *pool, int *n_out) {
  if (!pool) return nullptr;
  if (n_out) *n_out = (int)pool->chunks.size();
  return pool->d_ids.p;
}

int dcgs_pool_require(dcgs_pool *pool, const uint64_t *ids, int n, int64_t now, int *loaded,
                      int *evicted, void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx,
                 [&] { dcgs::pool_require(pool, ids, n, now, loaded, evicted, S(stream)); });
}

int dcgs_pool_prefetch(dcgs_pool *pool, const uint64_t *ids, int n, int64_t now, int *staged,
                       void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx,
                 [&] { dcgs::pool_prefetch(pool, ids, n, now, staged, S(stream)); });
}

int dcgs_pool_stats(dcgs_pool *pool, int64_t *out, int n_out) {
  if (!pool || !out) return DCGS_E_INVALID;
  const int64_t v[8] = {pool->n_loads,  pool->n_evictions, pool->n_prefetched, pool->n_misses,
                        pool->n_hits,   pool->bytes_h2d,   pool->bytes_d2h,    pool->resident_g};
  for (int k = 0; k < n_out && k < 8; ++k) out[k] = v[k];
  return DCGS_OK;
}

int dcgs_pool_read_chunk(dcgs_pool *pool, uint64_t id, float *params, float *m, float *v,
                         int32_t *step) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] { dcgs::pool_read_chunk(pool, id, params, m, v, step); });
}

int dcgs_pool_resident(dcgs_pool *pool, uint64_t *ids, int capacity, int *n_out,
                       int64_t *gaussians_out) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] {
    int k = 0;
    for (auto &c : pool->chunks)
      if (c.resident) {
        if (ids && k < capacity) ids[k] = c.id;
        ++k;
      }
    if (n_out) *n_out = k;
    if (gaussians_out) *gaussians_out = pool->resident_g;
    DCGS_CHECK(!ids || k <= capacity, DCGS_E_CAPACITY, "pool_resident: capacity");
  });
}

int dcgs_pool_loop_closure(dcgs_pool *pool, const dcgs_camera *keyframes,
                           const double *corrections, int n_keyframes,
                           const dcgs_camera *junctions, int n_junctions, int64_t *stats,
                           int n_stats, void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] {
    dcgs::pool_loop_closure(pool, keyframes, corrections, n_keyframes, junctions, n_junctions,
                            stats, n_stats, S(stream));
  });
}

int dcgs_compact(dcgs_pool *pool, const uint64_t *ids, const uint16_t *masks, int n_ids,
                 float *out, int64_t out_stride, int32_t *out_src, uint16_t *out_gmask,
                 int64_t capacity, int64_t *n_out, void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] {
    dcgs::pool_compact(pool, ids, masks, n_ids, out, out_stride, out_src, out_gmask, capacity,
                       n_out, S(stream));
  });
}

int dcgs_state_create(dcgs_ctx *ctx, dcgs_state **out) {
  if (!ctx || !out) return DCGS_E_INVALID;
  auto *s = new dcgs_state();
  s->ctx = ctx;
  *out = s;
  return DCGS_OK;
}

void dcgs_state_destroy(dcgs_state *st) {
  if (!st) return;
  if (st->cam_pinned) (void)hipHostFree(st->cam_pinned);
  delete st;
}

int dcgs_render_fwd(dcgs_ctx *ctx, dcgs_state *st, const float *params, int64_t n,
                    int64_t stride, int sh_degree, const uint16_t *gmask, int mask_shift,
                    const dcgs_camera *cams, int n_views, const float *bg, int tile_w,
                    int tile_h, int pixels_per_lane, float *rgb, float *depth, float *T,
                    void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(st && st->ctx == ctx, DCGS_E_INVALID, "render_fwd: state of another context");
    DCGS_CHECK(n_views >= 1 && n_views <= dcgs::kMaxViews && cams, DCGS_E_INVALID,
               "render_fwd: 1..16 views required");
    DCGS_CHECK(n >= 0 && n * n_views < (int64_t(1) << 31) && stride >= n && (n == 0 || params),
               DCGS_E_INVALID, "render_fwd: bad parameter block (n * n_views must be < 2^31)");
    DCGS_CHECK(sh_degree >= 0 && sh_degree <= 3, DCGS_E_INVALID, "render_fwd: sh_degree 0..3");
    DCGS_CHECK(mask_shift >= 0 && mask_shift + n_views <= 16, DCGS_E_INVALID,
               "render_fwd: mask_shift + n_views must be <= 16");
    DCGS_CHECK(pixels_per_lane >= 0 && pixels_per_lane < 256, DCGS_E_INVALID,
               "render_fwd: pixels_per_lane out of range");
    int ppt = pixels_per_lane & 15, ppt_bwd = pixels_per_lane >> 4;
    if (ppt == 0) ppt = tile_w == 8 ? 1 : tile_w == 16 ? 2 : 4;
    if (ppt_bwd == 0) ppt_bwd = ppt;
    DCGS_CHECK(dcgs::raster_shape_supported(tile_w, tile_h, ppt) &&
                   dcgs::raster_shape_supported(tile_w, tile_h, ppt_bwd),
               DCGS_E_INVALID,
               "render_fwd: raster shape must be 16x16x{1,2,4}, 8x8x1 or 32x16x{2,4,8}");
    for (int v = 0; v < n_views; ++v) {
      check_cam(&cams[v]);
      DCGS_CHECK(cams[v].width == cams[0].width && cams[v].height == cams[0].height,
                 DCGS_E_INVALID, "render_fwd: all views must share width and height");
      st->cams[v] = cams[v];
    }
    DCGS_CHECK(bg && rgb && depth, DCGS_E_INVALID, "render_fwd: null output");
    st->V = n_views;
    st->ppt = ppt;
    st->ppt_bwd = ppt_bwd;
    st->W = cams[0].width;
    st->H = cams[0].height;
    st->TW = tile_w;
    st->TH = tile_h;
    st->tiles_x = (st->W + tile_w - 1) / tile_w;
    st->tiles_y = (st->H + tile_h - 1) / tile_h;
    DCGS_CHECK((int64_t)st->tiles_x * st->tiles_y * n_views < (int64_t(1) << 24), DCGS_E_INVALID,
               "render_fwd: too many tiles");
    st->sh_degree = sh_degree;
    std::memcpy(st->bg, bg, 3 * sizeof(float));
    dcgs::render_forward(st, params, n, stride, gmask, mask_shift, S(stream), rgb, depth, T);
  });
}

int dcgs_render_bwd(dcgs_ctx *ctx, dcgs_state *st, const float *params, int64_t n,
                    int64_t stride, const float *dl_drgb, const float *dl_ddepth, float *grad,
                    int64_t grad_stride, int accumulate, float *grad2d, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(st && st->ctx == ctx, DCGS_E_INVALID, "render_bwd: state of another context");
    DCGS_CHECK(n == st->n && st->W > 0 && st->cam_dev.p, DCGS_E_INVALID,
               "render_bwd: n differs from the last forward on this state");
    DCGS_CHECK(st->fwd_ok, DCGS_E_INVALID, "render_bwd: the last forward on this state failed");
    DCGS_CHECK(dl_drgb && (n == 0 || (params && grad && grad_stride >= n && stride >= n)),
               DCGS_E_INVALID, "render_bwd: bad buffers");
    dcgs::render_backward(st, params, n, stride, dl_drgb, dl_ddepth, grad, grad_stride,
                          accumulate, grad2d, S(stream));
  });
}

int dcgs_loss_l1(dcgs_ctx *ctx, const float *rgb, const float *target, int64_t count,
                 double norm, float *dl_drgb, double *stats, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(rgb && target && dl_drgb && stats && count > 0 && norm > 0, DCGS_E_INVALID,
               "loss_l1: bad args");
    float *part = ctx->loss_part.need(2 * 1024);
    dcgs::StageTimer tm(ctx, DCGS_STAGE_LOSS, S(stream));
    dcgs::launch_loss_l1(rgb, target, count, norm, dl_drgb, stats, part, S(stream));
  });
}

int dcgs_loss_mapping(dcgs_ctx *ctx, const float *rgb, const float *target, const float *depth,
                      const float *depth_target, int n_views, int height, int width,
                      double lambda_s, double lambda_depth, float *dl_drgb, float *dl_ddepth,
                      double *stats, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::StageTimer tm(ctx, DCGS_STAGE_LOSS, S(stream));
    dcgs::mapping_loss(ctx, rgb, target, depth, depth_target, n_views, height, width, lambda_s,
                       lambda_depth, dl_drgb, dl_ddepth, stats, ctx->loss_maps, S(stream));
  });
}

int dcgs_sample_pixels(dcgs_ctx *ctx, const float *image, const float *render, const float *u,
                       int height, int width, double beta, double sigma, float *ps,
                       int32_t *out_idx, int32_t *out_count, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::sample_pixels(ctx, image, render, u, height, width, beta, sigma, ps, out_idx,
                        out_count, S(stream));
  });
}

int dcgs_adam_step(dcgs_pool *pool, const int32_t *src, const float *grad, int64_t n,
                   int64_t grad_stride, const dcgs_adam_config *cfg, void *stream) {
  if (!pool) return DCGS_E_INVALID;
  return guarded(pool->ctx, [&] {
    DCGS_CHECK(cfg && n >= 0 && (n == 0 || (src && grad && grad_stride >= n)), DCGS_E_INVALID,
               "adam_step: bad args");
    DCGS_CHECK(pool->d_params, DCGS_E_INVALID, "adam_step: pool holds no scene");
    dcgs::StageTimer tm(pool->ctx, DCGS_STAGE_ADAM, S(stream));
    dcgs::launch_adam(pool->d_params, pool->d_m, pool->d_v, pool->d_step, pool->R, src, grad, n,
                      grad_stride, *cfg, S(stream));
  });
}

int dcgs_autotune(dcgs_ctx *ctx, dcgs_state *st, const float *params, int64_t n, int64_t stride,
                  int sh_degree, const uint16_t *gmask, const dcgs_camera *cams, int n_views,
                  int force, int *out_shape, double *times_ms, int *n_shapes, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  static const int kShapes[][3] = {{16, 16, 1}, {16, 16, 2}, {16, 16, 4}, {8, 8, 1},
                                   {32, 16, 2}, {32, 16, 4}, {32, 16, 8}};
  constexpr int kN = sizeof(kShapes) / sizeof(kShapes[0]);
  if (n_shapes) *n_shapes = kN;
  return guarded(ctx, [&] {
    DCGS_CHECK(st && st->ctx == ctx && out_shape && cams && n_views >= 1 &&
                   n_views <= dcgs::kMaxViews && n >= 0,
               DCGS_E_INVALID, "autotune: bad args");
    int lg = 0;
    while ((int64_t(1) << lg) < n) ++lg;
    const uint64_t key = (uint64_t)cams[0].width << 40 | (uint64_t)cams[0].height << 24 |
                         (uint64_t)n_views << 8 | (uint64_t)lg;
    auto it = ctx->tune_cache.find(key);
    if (it != ctx->tune_cache.end() && !force) {
      for (int k = 0; k < 3; ++k) out_shape[k] = it->second[k];
      return;
    }
    const int W = cams[0].width, H = cams[0].height;
    const int64_t HW = (int64_t)W * H;
    const int R = dcgs::n_rows(sh_degree);
    float *img = ctx->tune_img.need(n_views * HW * 8 + 1);
    float *rgb = img, *depth = img + 3 * n_views * HW, *dl = img + 4 * n_views * HW;
    float *grad = ctx->tune_grad.need((size_t)R * (n > 0 ? n : 1));
    DCGS_HIP(hipMemsetAsync(dl, 0, 3 * n_views * HW * sizeof(float), S(stream)));
    const float bg[3] = {0, 0, 0};
    hipEvent_t e0, e1, e2;
    DCGS_HIP(hipEventCreate(&e0));
    DCGS_HIP(hipEventCreate(&e1));
    DCGS_HIP(hipEventCreate(&e2));
    struct Free {
      hipEvent_t a, b, c;
      ~Free() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        (void)hipEventDestroy(c);
      }
    } fr{e0, e1, e2};
    // forward and backward timed apart: the forward and the backward of one
    // tile size may take different pixels per lane (the pairs, the images
    // and the per-pixel state do not depend on it)
    float tf[kN], tb[kN];
    for (int k = 0; k < kN; ++k) {
      const int *sh = kShapes[k];
      auto fwd = [&] {
        const int rc = dcgs_render_fwd(ctx, st, params, n, stride, sh_degree, gmask, 0, cams,
                                       n_views, bg, sh[0], sh[1], sh[2], rgb, depth, nullptr,
                                       stream);
        DCGS_CHECK(rc == DCGS_OK, rc, "autotune: forward failed: " + ctx->err);
      };
      auto bwd = [&] {
        const int rc = dcgs_render_bwd(ctx, st, params, n, stride, dl, nullptr, grad, n, 0,
                                       nullptr, stream);
        DCGS_CHECK(rc == DCGS_OK, rc, "autotune: backward failed: " + ctx->err);
      };
      fwd();  // warm: buffers sized, code loaded
      bwd();
      tf[k] = tb[k] = 1e30f;
      for (int rep = 0; rep < 3; ++rep) {  // the fastest of three passes
        DCGS_HIP(hipEventRecord(e0, S(stream)));
        fwd();
        DCGS_HIP(hipEventRecord(e1, S(stream)));
        bwd();
        DCGS_HIP(hipEventRecord(e2, S(stream)));
        DCGS_HIP(hipEventSynchronize(e2));
        float a = 0.0f, b = 0.0f;
        DCGS_HIP(hipEventElapsedTime(&a, e0, e1));
        DCGS_HIP(hipEventElapsedTime(&b, e1, e2));
        tf[k] = std::min(tf[k], a);
        tb[k] = std::min(tb[k], b);
      }
      if (times_ms) times_ms[k] = tf[k] + tb[k];
    }
    // per tile size the fastest forward and the fastest backward
    double best = 1e300;
    int bf = 1, bb = 1;
    for (int k = 0; k < kN; ++k) {
      for (int j = 0; j < kN; ++j) {
        if (kShapes[j][0] != kShapes[k][0] || kShapes[j][1] != kShapes[k][1]) continue;
        if (tf[k] + tb[j] < best) {
          best = tf[k] + tb[j];
          bf = k;
          bb = j;
        }
      }
    }
    const int packed = kShapes[bf][2] | (kShapes[bb][2] == kShapes[bf][2] ? 0 : kShapes[bb][2] << 4);
    std::array<int, 3> a{kShapes[bf][0], kShapes[bf][1], packed};
    ctx->tune_cache[key] = a;
    for (int k = 0; k < 3; ++k) out_shape[k] = a[k];
  });
}

int dcgs_window_create(dcgs_ctx *ctx, dcgs_pool *pool, const dcgs_window_config *cfg,
                       dcgs_window **out) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] { dcgs::window_create(ctx, pool, cfg, out); });
}

void dcgs_window_destroy(dcgs_window *win) { dcgs::window_destroy(win); }

int dcgs_window_launch(dcgs_window *win, const uint64_t *ids, const uint16_t *masks, int n_ids,
                       const dcgs_camera *cams, int64_t *n_active, void *stream) {
  if (!win) return DCGS_E_INVALID;
  return guarded(dcgs::window_ctx(win), [&] {
    dcgs::window_launch(win, ids, masks, n_ids, cams, n_active, S(stream));
  });
}

int dcgs_window_sync(dcgs_window *win, int64_t *pairs_required, int *skipped) {
  if (!win) return DCGS_E_INVALID;
  return guarded(dcgs::window_ctx(win),
                 [&] { dcgs::window_sync(win, pairs_required, skipped); });
}

int dcgs_window_pairs(dcgs_window *win, int64_t *n_pairs) {
  if (!win || !n_pairs) return DCGS_E_INVALID;
  return guarded(dcgs::window_ctx(win), [&] { dcgs::window_pairs(win, n_pairs); });
}

int dcgs_prefetch_labels(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames, int horizon,
                         double chunk_size, uint8_t *labels, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::prefetch_labels(ctx, cams, n_frames, horizon, chunk_size, labels, S(stream));
  });
}

int dcgs_prefetch_features(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames,
                           const int32_t *frames, int n_sel, double chunk_size, double pos_unit,
                           const uint8_t *labels, float *X, uint64_t *cell_ids, uint8_t *y,
                           void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::prefetch_features(ctx, cams, n_frames, frames, n_sel, chunk_size, pos_unit, labels, X,
                            cell_ids, y, S(stream));
  });
}

int dcgs_mlp_forward(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16, const float *X,
                     int64_t n, float *z1, float *h1, float *z2, float *h2, float *logit,
                     void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::mlp_forward(ctx, theta, wbf16, X, n, z1, h1, z2, h2, logit, S(stream));
  });
}

int dcgs_mlp_backward(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16, const float *X,
                      const float *z1, const float *h1, const float *z2, const float *h2,
                      const float *logit, const uint8_t *y, int64_t n, float pos_weight,
                      float *grad, double *loss, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::mlp_backward(ctx, theta, wbf16, X, z1, h1, z2, h2, logit, y, n, pos_weight, grad, loss,
                       S(stream));
  });
}

int dcgs_mlp_adam(dcgs_ctx *ctx, float *theta, uint16_t *wbf16, float *m, float *v,
                  const float *grad, int64_t step, double lr, double beta1, double beta2,
                  double eps, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::mlp_adam(ctx, theta, wbf16, m, v, grad, step, lr, beta1, beta2, eps, S(stream));
  });
}

int dcgs_mlp_round(dcgs_ctx *ctx, const float *theta, uint16_t *wbf16, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] { dcgs::mlp_round(ctx, theta, wbf16, S(stream)); });
}

int dcgs_prefetch_predict(dcgs_ctx *ctx, const float *theta, const uint16_t *wbf16,
                          const dcgs_camera *history, double chunk_size, double pos_unit,
                          float threshold_logit, uint64_t *out_ids, int32_t *out_count,
                          float *out_logit, void *stream) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    dcgs::prefetch_predict(ctx, theta, wbf16, history, chunk_size, pos_unit, threshold_logit,
                           out_ids, out_count, out_logit, S(stream));
  });
}

int dcgs_profile_enable(dcgs_ctx *ctx, int enable) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    for (auto &m : ctx->marks) {
      ctx->spare_events.push_back(m.a);
      ctx->spare_events.push_back(m.b);
    }
    ctx->marks.clear();
    ctx->prof = enable != 0;
  });
}

int dcgs_profile_read(dcgs_ctx *ctx, double *ms, int64_t *calls, int n_stages) {
  if (!ctx) return DCGS_E_INVALID;
  return guarded(ctx, [&] {
    DCGS_CHECK(n_stages >= 0 && n_stages <= DCGS_STAGE_COUNT, DCGS_E_INVALID,
               "profile_read: n_stages out of range");
    for (int k = 0; k < n_stages; ++k) {
      if (ms) ms[k] = 0.0;
      if (calls) calls[k] = 0;
    }
    for (auto &m : ctx->marks) {
      DCGS_HIP(hipEventSynchronize(m.b));
      float t = 0.0f;
      DCGS_HIP(hipEventElapsedTime(&t, m.a, m.b));
      if (m.stage < n_stages) {
        if (ms) ms[m.stage] += t;
        if (calls) calls[m.stage] += 1;
      }
      ctx->spare_events.push_back(m.a);
      ctx->spare_events.push_back(m.b);
    }
    ctx->marks.clear();
  });
}

int dcgs_pairs_fit(int64_t n_pairs, int64_t pair_capacity) {
  return dcgs::pairs_overflow(n_pairs, pair_capacity, 0) ? DCGS_E_CAPACITY : DCGS_OK;
}

int dcgs_state_info(const dcgs_state *st, int64_t *n, int64_t *n_pairs, int32_t *tiles_x,
                    int32_t *tiles_y) {
  if (!st) return DCGS_E_INVALID;
  if (n) *n = st->n;
  if (n_pairs) *n_pairs = st->n_pairs;
  if (tiles_x) *tiles_x = st->tiles_x;
  if (tiles_y) *tiles_y = st->tiles_y;
  return DCGS_OK;
}

int dcgs_state_work(const dcgs_state *st, int64_t *walk, int64_t *inbox, void *stream) {
  if (!st || !walk || !inbox) return DCGS_E_INVALID;
  return guarded(st->ctx, [&] { dcgs::state_work(st, walk, inbox, S(stream)); });
}

int dcgs_state_export(const dcgs_state *st, uint64_t *keys, int32_t *values, int32_t *ranges,
                      int32_t *counts, float *records, int32_t *box, int32_t *last,
                      void *stream) {
  if (!st) return DCGS_E_INVALID;
  return guarded(st->ctx, [&] {
    dcgs::export_state(st, keys, values, ranges, counts, records, box, last, S(stream));
  });
}

}  // extern "C"
