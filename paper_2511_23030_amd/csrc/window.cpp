// Graph-captured mapping window: the batched forward, L1 loss, backward and
// Adam step of one window of keyframes (Sec. III-E "Optimization", the
// per-keyframe step batched over views) recorded once into a HIP graph and
// replayed for every window.
//
// Everything that varies from window to window without changing the work's
// shape lives in device memory the graph reads: the compacted Gaussians
// (written by the compaction kernel, launched before the graph), the
// cameras and the two counts n and n * views (one copy node from pinned
// staging), the targets (a caller buffer).  Grids are sized for the
// capacities; kernels read the counts on the device.  The pair count is
// only known on the device: when it exceeds the pair capacity the window
// draws nothing and skips its Adam step, and a sticky device flag makes
// every later replay do the same until the window is rebuilt, so the
// caller can redo the skipped windows in order with a larger capacity.
//
// Two graph instances alternate, each with its own staging block, so the
// host prepares window w+1 while window w runs.
#include <cstring>

#include "internal.h"

struct dcgs_window {
  dcgs_ctx *ctx = nullptr;
  dcgs_pool *pool = nullptr;
  dcgs_state *state = nullptr;
  dcgs_window_config cfg{};
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  void *staging[2] = {nullptr, nullptr};   // cameras + counts, then the overflow readback
  hipEvent_t done[2] = {nullptr, nullptr};
  bool launched[2] = {false, false};
  int next = 0;
  int64_t overflow = 0;
  dcgs::DevBuf<float> loss_part;
  dcgs::DevBuf<float> loss_maps;  // the full loss's SSIM maps and partial sums
};

namespace dcgs {

namespace {

int64_t *flag_of(dcgs_window *w, int x) {
  return (int64_t *)((char *)w->staging[x] + ((render_stage_bytes() + 63) / 64) * 64);
}

void capture(dcgs_window *w, int x) {
  const dcgs_window_config &c = w->cfg;
  dcgs_state *s = w->state;
  hipStream_t cs = w->cap_stream;
  const int64_t HW = (int64_t)c.width * c.height;
  const bool prof = w->ctx->prof;
  w->ctx->prof = false;  // no timing events inside the graph
  struct Restore {
    dcgs_ctx *ctx;
    bool prof;
    ~Restore() { ctx->prof = prof; }
  } restore{w->ctx, prof};
  int64_t *cnt = render_counters(s, cs);
  DCGS_HIP(hipStreamSynchronize(cs));  // the counters' first zeroing is not part of the graph
  hipGraph_t g = nullptr;
  DCGS_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  try {
    DCGS_HIP(hipMemcpyAsync(s->cam_dev.p, w->staging[x], render_stage_bytes(),
                            hipMemcpyHostToDevice, cs));
    render_forward_planned(s, c.params, c.capacity, c.gmask, cs, c.rgb, c.depth, nullptr);
    const bool full = c.lambda_s > 0.0 || c.lambda_depth > 0.0;
    const bool with_depth = c.lambda_depth > 0.0;
    if (full)  // its scratch was sized at creation: no allocation under capture
      mapping_loss(w->ctx, c.rgb, c.targets, with_depth ? c.depth : nullptr,
                   with_depth ? c.depth_targets : nullptr, c.n_views, c.height, c.width,
                   c.lambda_s, c.lambda_depth, c.dl_drgb, with_depth ? c.dl_ddepth : nullptr,
                   c.stats, w->loss_maps, cs);
    else
      launch_loss_l1(c.rgb, c.targets, (int64_t)c.n_views * 3 * HW, c.loss_norm, c.dl_drgb,
                     c.stats, w->loss_part.p, cs);
    render_backward(s, c.params, 0, c.capacity, c.dl_drgb, with_depth ? c.dl_ddepth : nullptr,
                    c.grad, c.capacity, 0, nullptr, cs);
    dcgs_pool *p = w->pool;
    launch_adam(p->d_params, p->d_m, p->d_v, p->d_step, p->R, c.src, c.grad, c.capacity,
                c.capacity, c.adam, cs, cnt);
    DCGS_HIP(hipMemcpyAsync(flag_of(w, x), cnt + 3, sizeof(int64_t), hipMemcpyDeviceToHost, cs));
  } catch (...) {
    hipGraph_t dropped = nullptr;
    (void)hipStreamEndCapture(cs, &dropped);
    if (dropped) (void)hipGraphDestroy(dropped);
    throw;
  }
  DCGS_HIP(hipStreamEndCapture(cs, &g));
  hipError_t e = hipGraphInstantiate(&w->exec[x], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  DCGS_HIP(e);
}

}  // namespace

void window_create(dcgs_ctx *ctx, dcgs_pool *pool, const dcgs_window_config *cfg,
                   dcgs_window **out) {
  DCGS_CHECK(ctx && pool && cfg && out, DCGS_E_INVALID, "window_create: bad args");
  const dcgs_window_config &c = *cfg;
  DCGS_CHECK(c.n_views >= 1 && c.n_views <= kMaxViews && c.width > 0 && c.height > 0 &&
                 c.width < 65536 && c.height < 65536 && c.capacity > 0 &&
                 c.pair_capacity > 0 && c.pair_capacity < (int64_t(1) << 31) &&
                 c.sh_degree == pool->deg && c.loss_norm > 0 && c.lambda_s >= 0 &&
                 c.lambda_s <= 1 && c.lambda_depth >= 0 &&
                 (c.lambda_depth == 0 || (c.depth_targets && c.dl_ddepth)),
             DCGS_E_INVALID, "window_create: bad configuration");
  DCGS_CHECK(c.params && c.grad && c.src && c.gmask && c.rgb && c.depth && c.dl_drgb &&
                 c.targets && c.stats,
             DCGS_E_INVALID, "window_create: null buffer");
  DCGS_CHECK(pool->d_params, DCGS_E_INVALID, "window_create: pool holds no scene");
  DCGS_CHECK(c.capacity * c.n_views < (int64_t(1) << 31), DCGS_E_INVALID,
             "window_create: capacity x views must stay below 2^31 records");
  DCGS_CHECK((int64_t)((c.width + c.tile_w - 1) / std::max(c.tile_w, 1)) *
                     ((c.height + c.tile_h - 1) / std::max(c.tile_h, 1)) * c.n_views <
                 (int64_t(1) << 24),
             DCGS_E_INVALID, "window_create: too many tiles");
  auto *w = new dcgs_window();
  struct Guard {
    dcgs_window *w;
    ~Guard() {
      if (w) window_destroy(w);
    }
  } guard{w};
  w->ctx = ctx;
  w->pool = pool;
  w->cfg = c;
  w->state = new dcgs_state();
  dcgs_state *s = w->state;
  s->ctx = ctx;
  s->W = c.width;
  s->H = c.height;
  s->TW = c.tile_w;
  s->TH = c.tile_h;
  s->ppt = c.pixels_per_lane & 15;
  s->ppt_bwd = (c.pixels_per_lane >> 4) ? (c.pixels_per_lane >> 4) : s->ppt;
  s->tiles_x = (c.width + c.tile_w - 1) / c.tile_w;
  s->tiles_y = (c.height + c.tile_h - 1) / c.tile_h;
  s->sh_degree = c.sh_degree;
  s->V = c.n_views;
  for (int k = 0; k < 3; ++k) s->bg[k] = c.bg[k];
  DCGS_CHECK(c.pixels_per_lane >= 0 && c.pixels_per_lane < 256 &&
                 raster_shape_supported(c.tile_w, c.tile_h, s->ppt) &&
                 raster_shape_supported(c.tile_w, c.tile_h, s->ppt_bwd),
             DCGS_E_INVALID, "window_create: unsupported raster shape");
  render_plan(s, c.capacity, c.pair_capacity);
  s->grad2d.need(10 * (size_t)s->rs + 1);
  w->loss_part.need(2 * 1024);
  if (c.lambda_s > 0.0 || c.lambda_depth > 0.0)
    mapping_loss_reserve(c.n_views, c.height, c.width, w->loss_maps);
  DCGS_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
  const size_t sb = ((render_stage_bytes() + 63) / 64) * 64 + 64;
  for (int x = 0; x < 2; ++x) {
    DCGS_HIP(hipHostMalloc(&w->staging[x], sb, hipHostMallocDefault));
    std::memset(w->staging[x], 0, sb);
    DCGS_HIP(hipEventCreateWithFlags(&w->done[x], hipEventDisableTiming));
  }
  for (int x = 0; x < 2; ++x) capture(w, x);
  guard.w = nullptr;
  *out = w;
}

void window_destroy(dcgs_window *w) {
  if (!w) return;
  for (int x = 0; x < 2; ++x)
    if (w->launched[x] && w->done[x]) (void)hipEventSynchronize(w->done[x]);
  if (w->cap_stream) (void)hipStreamSynchronize(w->cap_stream);
  for (int x = 0; x < 2; ++x) {
    if (w->exec[x]) (void)hipGraphExecDestroy(w->exec[x]);
    if (w->done[x]) (void)hipEventDestroy(w->done[x]);
    if (w->staging[x]) (void)hipHostFree(w->staging[x]);
  }
  if (w->cap_stream) (void)hipStreamDestroy(w->cap_stream);
  if (w->state) {
    if (w->state->cam_pinned) (void)hipHostFree(w->state->cam_pinned);
    delete w->state;
  }
  delete w;
}

void window_launch(dcgs_window *w, const uint64_t *ids, const uint16_t *masks, int n_ids,
                   const dcgs_camera *cams, int64_t *n_active, hipStream_t st) {
  DCGS_CHECK(cams && (ids || n_ids == 0), DCGS_E_INVALID, "window_launch: bad args");
  DCGS_CHECK(w->overflow == 0, DCGS_E_CAPACITY,
             "window_launch: an earlier window overflowed the pair capacity; rebuild the window");
  const dcgs_window_config &c = w->cfg;
  const int x = w->next;
  if (w->launched[x]) {
    DCGS_HIP(hipEventSynchronize(w->done[x]));
    const int64_t f = *flag_of(w, x);
    if (f != 0) {
      w->overflow = f;
      throw Error{DCGS_E_CAPACITY, "window_launch: an earlier window overflowed the pair capacity"};
    }
  }
  for (int v = 0; v < c.n_views; ++v) {
    DCGS_CHECK(cams[v].width == c.width && cams[v].height == c.height && cams[v].fx > 0 &&
                   cams[v].fy > 0 && cams[v].z_near > 0 && cams[v].z_far > cams[v].z_near,
               DCGS_E_INVALID, "window_launch: camera does not match the window");
    w->state->cams[v] = cams[v];
  }
  int64_t n = 0;
  pool_compact(w->pool, ids, masks, n_ids, c.params, c.capacity, c.src, c.gmask, c.capacity, &n,
               st);
  render_stage(w->state, w->staging[x], n);
  w->state->n = n;
  DCGS_HIP(hipGraphLaunch(w->exec[x], st));
  DCGS_HIP(hipEventRecord(w->done[x], st));
  w->launched[x] = true;
  w->next = x ^ 1;
  if (n_active) *n_active = n;
}

void window_sync(dcgs_window *w, int64_t *pairs_required, int *skipped) {
  // launch order: buffer next^1 is the most recent, next the one before
  const int recent = w->next ^ 1, before = w->next;
  int64_t f_recent = 0, f_before = 0;
  if (w->launched[recent]) {
    DCGS_HIP(hipEventSynchronize(w->done[recent]));
    f_recent = *flag_of(w, recent);
  }
  if (w->launched[before]) {
    DCGS_HIP(hipEventSynchronize(w->done[before]));
    f_before = *flag_of(w, before);
  }
  // the overflow flag is sticky: a skipped launch makes every later one skip
  const int n_skip = f_before != 0 ? 2 : (f_recent != 0 ? 1 : 0);
  const int64_t need = std::max(w->overflow, std::max(f_recent, f_before));
  if (pairs_required) *pairs_required = need;
  if (skipped) *skipped = n_skip;
  if (need != 0) {
    w->overflow = need;
    throw Error{DCGS_E_CAPACITY, "window_sync: a window overflowed the pair capacity"};
  }
}

dcgs_ctx *window_ctx(dcgs_window *w) { return w->ctx; }

void window_pairs(dcgs_window *w, int64_t *n_pairs) {
  // the pair count of the last completed launch (device counter)
  for (int x = 0; x < 2; ++x)
    if (w->launched[x]) DCGS_HIP(hipEventSynchronize(w->done[x]));
  int64_t v = 0;
  DCGS_HIP(hipMemcpy(&v, render_counters(w->state, nullptr) + 2, sizeof(int64_t),
                     hipMemcpyDeviceToHost));
  *n_pairs = v;
}

}  // namespace dcgs
