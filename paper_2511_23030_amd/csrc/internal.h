// Internal declarations of libdcgs: context, render state, pool, device
// helpers and the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/dcgs.h"

namespace dcgs {

constexpr int kWave = 64;
constexpr int kMaxViews = 16;
constexpr int kRecFloats = 16;  // four float4 per projection record

// Largest pair count one forward handles: pair offsets, gradient slots and
// list positions are 32-bit, per-tile ranges int32.
constexpr int64_t kMaxPairs = (int64_t(1) << 31) - 1;

// The overflow decision on a forward's (tile, Gaussian) pair count, taken
// in 64-bit: more pairs than the pair buffers hold, more than 32-bit
// indexing allows, or an earlier overflow of the same graph-replayed state
// (sticky) -- the window then draws nothing.
__host__ __device__ inline bool pairs_overflow(int64_t total, int64_t pcap, int64_t sticky) {
  return total > pcap || total > kMaxPairs || sticky != 0;
}

// Thrown inside the library only; every C entry point converts it to a status.
struct Error {
  int status;
  std::string msg;
};

#define DCGS_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                     \
      throw ::dcgs::Error{DCGS_E_HIP, std::string(#call) + ": " +             \
                                          hipGetErrorString(e_)};             \
  } while (0)

#define DCGS_CHECK(cond, status, msg)                                         \
  do {                                                                        \
    if (!(cond)) throw ::dcgs::Error{(status), (msg)};                        \
  } while (0)

#define DCGS_LAUNCH_CHECK() DCGS_HIP(hipGetLastError())

// Growable device buffer (never shrinks).
template <typename T>
struct DevBuf {
  T *p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  T *need(size_t n) {
    if (n > cap) {
      if (p) DCGS_HIP(hipFree(p));
      p = nullptr;
      size_t c = n + n / 8 + 64;
      DCGS_HIP(hipMalloc(&p, c * sizeof(T)));
      cap = c;
    }
    return p;
  }
};

inline int n_rows(int deg) { return 11 + 3 * (deg + 1) * (deg + 1); }

// Number of radix passes / digit width for a key of `bits` significant bits.
inline void digit_plan(int bits, int *passes, int *width) {
  if (bits <= 0) {
    *passes = 0;
    *width = 0;
    return;
  }
  *passes = (bits + 8) / 9;  // digits of at most 9 bits (16 bits: two of 8; 17: 9 + 8)
  *width = (bits + *passes - 1) / *passes;
}

}  // namespace dcgs

struct dcgs_ctx {
  int device = 0;
  std::string err;
  // stage timers
  bool prof = false;
  struct Mark {
    int stage;
    hipEvent_t a, b;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> spare_events;
  // chunk selection's per-chunk masks, one buffer per stream (selections on
  // different streams may run at once)
  std::mutex sel_mu;
  std::unordered_map<void *, std::unique_ptr<dcgs::DevBuf<uint16_t>>> sel_mask;
  dcgs::DevBuf<uint8_t> kf_buf;   // keyframe selection: cameras, active ids, outputs
  uint16_t *noalloc_scratch = nullptr;  // this device's copy of the static selection scratch
  dcgs::DevBuf<int> flag;
  dcgs::DevBuf<float> loss_part;
  dcgs::DevBuf<float> loss_maps;  // SSIM derivative maps and partial sums
  dcgs::DevBuf<uint32_t> samp;    // sampling flags and their scan
  dcgs::DevBuf<uint32_t> scan_part;
  int n_cu = 256;
  // autotuner: scratch outputs and the cache (key -> tile_w, tile_h, ppt)
  dcgs::DevBuf<float> tune_img, tune_grad;
  std::unordered_map<uint64_t, std::array<int, 3>> tune_cache;
  // learned prefetch: camera staging and MLP scratch
  struct Prefetch {
    void *pinned = nullptr;
    size_t pinned_cap = 0;
    hipEvent_t staged = nullptr;  // last camera upload's copy
    dcgs::DevBuf<uint8_t> cams;
    dcgs::DevBuf<float> dz1, dz2, part, split, colpart, X, act;
    dcgs::DevBuf<double> part_loss;
    dcgs::DevBuf<uint64_t> ids;
  } pf;
};

struct dcgs_state {
  dcgs_ctx *ctx = nullptr;
  // shape of the last forward
  int64_t n = 0, n_pairs = 0;
  int W = 0, H = 0, TW = 16, TH = 16, ppt = 2, tiles_x = 0, tiles_y = 0, sh_degree = 0;
  int ppt_bwd = 2;  // pixels per lane of the backward raster
  float bg[3] = {0, 0, 0};
  int V = 1;                              // views rendered together
  dcgs_camera cams[dcgs::kMaxViews]{};
  dcgs::DevBuf<uint8_t> cam_dev;          // projection constants per view
  void *cam_pinned = nullptr;             // host staging for cam_dev
  // per Gaussian
  dcgs::DevBuf<float4> rec;        // [3][n] float4 (A, B, C planes)
  dcgs::DevBuf<uint32_t> zkey;     // [n]
  dcgs::DevBuf<uint32_t> count;    // [n]
  dcgs::DevBuf<uint32_t> order;    // [n] depth order -> Gaussian
  dcgs::DevBuf<uint32_t> key_tmp, val_tmp;
  dcgs::DevBuf<uint32_t> scan;      // [n + 1] pair offsets in depth order
  dcgs::DevBuf<uint32_t> seg_tot;   // pair count per projection segment (view, workgroup)
  dcgs::DevBuf<uint32_t> seg_off;   // their exclusive scan: gradient slot bases
  dcgs::DevBuf<uint64_t> tmask;     // [n] kept tiles of the record's tile rectangle
  // per pair
  dcgs::DevBuf<uint64_t> pairs, pairs_tmp;
  dcgs::DevBuf<float2> partial;  // [5 * P] per-pair gradient partials (ten floats)
  // launch plan: grids sized for n_grid Gaussians, record planes rs apart,
  // pcap pair slots (planned windows; eager forwards size them exactly).
  // The device counters [n, nr, pairs, overflow, sticky overflow, 64-bit
  // pair total] follow the camera constants in cam_dev.
  bool fwd_ok = false;  // the last forward completed (a backward may follow)
  int64_t n_grid = 0, rs = 0, pcap = 0;
  // per tile
  dcgs::DevBuf<int2> ranges;
  dcgs::DevBuf<uint64_t> frontier;
  dcgs::DevBuf<uint32_t> torder;  // raster launch order (tile per workgroup), longest lists first
  // backward work list: long lists split into segments (render.hip)
  dcgs::DevBuf<uint32_t> segc, segs, segpart;  // per-order counts, their scans, scan partials
  dcgs::DevBuf<int2> witem;        // (tile, segment) per backward workgroup
  dcgs::DevBuf<int> bslot;         // per tile: first boundary-state slot, -1 if not split
  dcgs::DevBuf<float> bound;       // per slot: T, colour, depth of every pixel of the tile
  dcgs::DevBuf<float> fseg;        // per slot of a forward-split tile: product, last, how it ended
  int64_t wcap = 0;                // work items the backward grid is sized for
  int64_t fcap = 0;                // work items of forward-split tiles the forward grids cover
  // per pixel
  dcgs::DevBuf<float> T_final;
  dcgs::DevBuf<int> last;
  // radix sort histograms
  dcgs::DevBuf<uint32_t> hist;
  dcgs::DevBuf<float> grad2d;  // [10][n] when the caller passes none
  dcgs::DevBuf<uint32_t> scan_part;  // block totals of the pair-count scan
  dcgs::DevBuf<unsigned long long> count_part;  // 64-bit pair-count sums per k_depth_counts workgroup
};

struct HostChunk {
  uint64_t id = 0;
  int64_t n = 0;
  int64_t pages = 0;
  int block = -1;           // host block holding the chunk's pages
  float *params = nullptr;  // [pages][R][PG] inside the block
  float *m = nullptr;
  float *v = nullptr;
  int32_t *step = nullptr;  // [pages][PG]
  // residency
  bool resident = false;
  int64_t last_access = -1;
  std::vector<int32_t> dev_pages;
  hipEvent_t ready = nullptr;  // recorded on the copy stream after the last load
  bool staged = false;         // loaded by a prefetch, not yet required
};

struct dcgs_pool {
  dcgs_ctx *ctx = nullptr;
  int deg = 0, R = 0;
  int64_t budget = 0;        // Gaussians
  double s = 0;              // chunk side (metres), fixed at ingest
  int64_t page_cap = 0;      // device pages
  int64_t resident_g = 0;    // Gaussians resident
  static constexpr int PG_LOG2 = 12;
  static constexpr int PG = 1 << PG_LOG2;
  // device pool, page-major: [page][R][PG] floats, step [page][PG]
  float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr;
  int32_t *d_step = nullptr;
  std::vector<int32_t> free_pages;  // kept sorted descending (pop_back = lowest)
  // host store: pinned blocks, each holding whole chunks (params, m, v and
  // step pages back to back); a block is freed when no chunk lives in it
  struct HostBlock {
    char *base = nullptr;
    int64_t live = 0;  // chunks stored in the block
  };
  std::vector<HostBlock> blocks;
  std::vector<HostChunk> chunks;               // ascending id
  std::unordered_map<uint64_t, int> index;     // id -> position in chunks
  dcgs::DevBuf<uint64_t> d_ids;                // ascending ids on device
  // compaction segment upload
  dcgs::DevBuf<int4> d_seg;
  int4 *h_seg = nullptr;
  size_t h_seg_cap = 0;
  hipEvent_t seg_done = nullptr;
  hipEvent_t cut = nullptr;  // compute-stream point an eviction's copy waits for
  // staging: every host<->device chunk copy runs on this stream
  hipStream_t copy = nullptr;
  // frame_event[f]: recorded on the compute stream at the first require of
  // frame f, i.e. after all work of frames < f was enqueued there
  std::unordered_map<int64_t, hipEvent_t> frame_event;
  // counters
  int64_t n_loads = 0, n_evictions = 0, n_prefetched = 0, n_misses = 0, n_hits = 0;
  int64_t bytes_h2d = 0, bytes_d2h = 0;
};

namespace dcgs {

// A timing event from the context's free list (nullptr if none can be made).
hipEvent_t take_event(dcgs_ctx *ctx) noexcept;

// Records start/stop events around a stage on `st` when ctx->prof is set.
// Never throws: a failed record only drops that sample.
struct StageTimer {
  dcgs_ctx *ctx;
  hipStream_t st;
  int stage;
  hipEvent_t a = nullptr;
  StageTimer(dcgs_ctx *c, int s, hipStream_t stream) noexcept : ctx(c), st(stream), stage(s) {
    if (ctx && ctx->prof) {
      a = take_event(ctx);
      if (a && hipEventRecord(a, st) != hipSuccess) a = nullptr;
    }
  }
  ~StageTimer() {
    if (!a) return;
    hipEvent_t b = take_event(ctx);
    if (b && hipEventRecord(b, st) == hipSuccess) ctx->marks.push_back({stage, a, b});
  }
};

// ---- launchers (one translation unit each) ----
void launch_chunk_ids(const float *mean, int64_t n, int64_t stride, double s,
                      uint64_t *out, int *flag, hipStream_t st);
void launch_select(const dcgs_camera *cams, int n_views, const uint64_t *ids,
                   int n_chunks, double s, uint16_t *mask_tmp,
                   uint64_t *out_ids, uint16_t *out_mask, int32_t *out_count,
                   hipStream_t st);
// Keyframe selection, Sec. III-F (chunks.hip): Eq. (8) membership, Eq. (7)
// overlap counts, and the window (host outputs; synchronises st).
void keyframe_overlap(dcgs_ctx *ctx, const dcgs_camera *kf, int n_kf, int latest, double g,
                      const uint64_t *ids, int n, double s, const uint64_t *act, int n_act,
                      uint8_t *in_set, int32_t *n_visible, int32_t *n_overlap, double *overlap,
                      int n_window, int32_t *window, int32_t *n_window_out, hipStream_t st);
// Per-chunk view mask only (bit v: view v sees the chunk), 1..16 views.
void launch_select_mask(const dcgs_camera *cams, int n_views, const uint64_t *ids,
                        int n_chunks, double s, uint16_t *mask, hipStream_t st);
void launch_compact(const float *pool, int R, const int4 *seg, int n_seg,
                    const uint16_t *seg_mask, float *out, int64_t out_stride,
                    int32_t *out_src, uint16_t *out_gmask, hipStream_t st);
// With cnt non-null, n is a capacity and the count is cnt[0]; nothing is
// updated when cnt[3] != 0 (the window's pair capacity overflowed).
void launch_adam(float *params, float *m, float *v, int32_t *step, int R,
                 const int32_t *src, const float *grad, int64_t n,
                 int64_t grad_stride, const dcgs_adam_config &cfg,
                 hipStream_t st, const int64_t *cnt = nullptr);
void launch_loss_l1(const float *rgb, const float *target, int64_t count,
                    double norm, float *dl, double *stats, float *part,
                    hipStream_t st);

// mapping loss of Eqs. (2)-(4) (loss.hip)
void mapping_loss(dcgs_ctx *ctx, const float *rgb, const float *target, const float *depth,
                  const float *depth_target, int n_views, int H, int W, double lambda_s,
                  double lambda_depth, float *dl_drgb, float *dl_ddepth, double *stats,
                  DevBuf<float> &scratch, hipStream_t st);

void mapping_loss_reserve(int n_views, int H, int W, DevBuf<float> &scratch);

// LoG sampling map (sampling.hip)
void sample_pixels(dcgs_ctx *ctx, const float *image, const float *render, const float *u,
                   int H, int W, double beta, double sigma, float *ps, int32_t *out_idx,
                   int32_t *out_count, hipStream_t st);

// learned prefetch (prefetch.hip)
void prefetch_labels(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames, int horizon,
                     double s, uint8_t *labels, hipStream_t st);
void prefetch_features(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames,
                       const int32_t *frames, int n_sel, double s, double pos_unit,
                       const uint8_t *labels, float *X, uint64_t *ids, uint8_t *y,
                       hipStream_t st);
void mlp_forward(dcgs_ctx *ctx, const float *theta, const uint16_t *wb, const float *X,
                 int64_t n, float *z1, float *h1, float *z2, float *h2, float *logit,
                 hipStream_t st);
void mlp_backward(dcgs_ctx *ctx, const float *theta, const uint16_t *wb, const float *X,
                  const float *z1, const float *h1, const float *z2, const float *h2,
                  const float *logit, const uint8_t *y, int64_t n, float pos_weight,
                  float *grad, double *loss, hipStream_t st);
void mlp_adam(dcgs_ctx *ctx, float *theta, uint16_t *wb, float *m, float *v, const float *grad,
              int64_t step, double lr, double beta1, double beta2, double eps, hipStream_t st);
void mlp_round(dcgs_ctx *ctx, const float *theta, uint16_t *wb, hipStream_t st);
void prefetch_predict(dcgs_ctx *ctx, const float *theta, const uint16_t *wb,
                      const dcgs_camera *hist, double s, double pos_unit, float threshold,
                      uint64_t *out_ids, int32_t *out_count, float *out_logit, hipStream_t st);

// exclusive scan of in (or of in[gather[i]] when gather != null), n
// elements; out has n + 1 entries (out[n] = total).
// With n_dev non-null, n is a capacity (grids are sized for it) and the
// element count is min(*n_dev, n), read on the device (graph capture).
void scan_u32(const uint32_t *in, const uint32_t *gather, uint32_t *out,
              int64_t n, uint32_t *part, hipStream_t st, const int64_t *n_dev = nullptr);
size_t scan_part_size(int64_t n);

// stable LSD radix sort of (key, value) u32 pairs over key bits [0, bits).
// Result ends in keys/vals; tmp buffers are n entries each.
void sort_u32_pairs(uint32_t *keys, uint32_t *vals, uint32_t *ktmp,
                    uint32_t *vtmp, int64_t n, int bits, DevBuf<uint32_t> &hist,
                    hipStream_t st, const int64_t *n_dev = nullptr);
// stable LSD radix sort of u64 words by bits [lo, lo + bits).
void sort_u64_bits(uint64_t *a, uint64_t *tmp, int64_t n, int lo, int bits,
                   DevBuf<uint32_t> &hist, hipStream_t st, const int64_t *n_dev = nullptr);

void render_forward(dcgs_state *s, const float *params, int64_t n,
                    int64_t stride, const uint16_t *gmask, int mask_shift, hipStream_t st,
                    float *rgb, float *depth, float *T);
void render_backward(dcgs_state *s, const float *params, int64_t n,
                     int64_t stride, const float *dl_drgb,
                     const float *dl_ddepth, float *grad, int64_t grad_stride,
                     int accumulate, float *grad2d, hipStream_t st);
// Planned (graph-capturable) rendering: buffers for n_cap Gaussians and
// pcap pairs are allocated by render_plan; the per-window counts and
// cameras come from the staging block (render_stage writes it, the caller
// copies it to the device block at state->cam_dev); render_forward_planned
// and render_backward then enqueue work with no host synchronisation.
void render_plan(dcgs_state *s, int64_t n_cap, int64_t pcap);
size_t render_stage_bytes();
void render_stage(const dcgs_state *s, void *pinned, int64_t n);
void render_forward_planned(dcgs_state *s, const float *params, int64_t stride,
                            const uint16_t *gmask, hipStream_t st, float *rgb, float *depth,
                            float *T);
int64_t *render_counters(dcgs_state *s, hipStream_t st);
bool raster_shape_supported(int tw, int th, int ppt);
// Scratch (32-bit words) of one radix pass over n keys with 8-bit digits.
size_t radix_scratch(int64_t n);

// graph-captured mapping windows (window.cpp)
void window_create(dcgs_ctx *ctx, dcgs_pool *pool, const dcgs_window_config *cfg,
                   dcgs_window **out);
void window_destroy(dcgs_window *w);
void window_launch(dcgs_window *w, const uint64_t *ids, const uint16_t *masks, int n_ids,
                   const dcgs_camera *cams, int64_t *n_active, hipStream_t st);
void window_sync(dcgs_window *w, int64_t *pairs_required, int *skipped);
void window_pairs(dcgs_window *w, int64_t *n_pairs);
dcgs_ctx *window_ctx(dcgs_window *w);
void pool_loop_closure(dcgs_pool *p, const dcgs_camera *keyframes, const double *corr, int n_kf,
                       const dcgs_camera *junctions, int n_junctions, int64_t *stats,
                       int n_stats, hipStream_t st);
void pool_release_chunk(dcgs_pool *p, HostChunk &h);
void pool_index(dcgs_pool *p, hipStream_t st);
void pool_compact(dcgs_pool *p, const uint64_t *ids, const uint16_t *masks, int n_ids,
                  float *out, int64_t out_stride, int32_t *out_src, uint16_t *out_gmask,
                  int64_t capacity, int64_t *n_out, hipStream_t st);
void state_work(const dcgs_state *s, int64_t *walk, int64_t *inbox, hipStream_t st);
void export_state(const dcgs_state *s, uint64_t *keys, int32_t *values,
                  int32_t *ranges, int32_t *counts, float *records,
                  int32_t *box, int32_t *last, hipStream_t st);

}  // namespace dcgs
