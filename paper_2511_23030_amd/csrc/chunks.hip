// Chunk IDs (Sec. III-D, Eqs. 5-6) and visible-chunk selection
// (Sec. III-D "Frustum Culling") for gfx950.
#include <algorithm>
#include <vector>

#include "frustum.h"

namespace dcgs {
namespace {

using namespace frustum;

__global__ void k_chunk_ids(const float *__restrict__ mean, int64_t n,
                            int64_t stride, double s, uint64_t *__restrict__ out,
                            int *__restrict__ flag) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double half = 0.5 * s;
  int64_t c[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double p = (double)mean[a * stride + i];
    c[a] = (int64_t)floor((p + half) / s);  // Eq. (5)
  }
  const int64_t lo = -(int64_t(1) << 20), hi = (int64_t(1) << 20) - 1;
  bool ok = c[0] >= lo && c[0] <= hi && c[1] >= lo && c[1] <= hi &&
            c[2] >= lo && c[2] <= hi;
  if (!ok) {
    out[i] = ~uint64_t(0);
    *flag = 1;
    return;
  }
  // Eq. (6): 21 bits per axis after adding 2^20.
  out[i] = (uint64_t(c[0] - lo) << 42) | (uint64_t(c[1] - lo) << 21) |
           uint64_t(c[2] - lo);
}

__global__ void k_select_mask(CamSet cs, int n_views,
                              const uint64_t *__restrict__ ids, int n,
                              double s, uint16_t *__restrict__ mask) {
  __shared__ ViewAxes va[kMaxViews];
  for (int t = threadIdx.x; t < n_views * kAxes; t += blockDim.x)
    build_axes(cs.c[t / kAxes], t % kAxes, va[t / kAxes]);
  __syncthreads();
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t id = ids[i];
  const int64_t off = int64_t(1) << 20, m21 = (int64_t(1) << 21) - 1;
  const double cc[3] = {double(int64_t((id >> 42) & m21) - off) * s,
                        double(int64_t((id >> 21) & m21) - off) * s,
                        double(int64_t(id & m21) - off) * s};
  const double h = 0.5 * s;
  unsigned m = 0;
  for (int v = 0; v < n_views; ++v)
    if (box_meets(va[v], cc, h)) m |= 1u << v;
  mask[i] = (uint16_t)m;
}

// Single-workgroup stable compaction of the chunks with a non-zero mask.
__global__ void __launch_bounds__(1024)
    k_select_compact(const uint64_t *__restrict__ ids,
                     const uint16_t *__restrict__ mask, int n,
                     uint64_t *__restrict__ out_ids,
                     uint16_t *__restrict__ out_mask, int32_t *out_count) {
  __shared__ int wave_sum[1024 / kWave];
  __shared__ int base_s;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int r = 0; r < n; r += 1024) {
    int i = r + threadIdx.x;
    uint16_t m = i < n ? mask[i] : 0;
    uint64_t b = __ballot(m != 0);
    int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(b >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)b, 0));
    if (lane == 0) wave_sum[wv] = __popcll(b);
    __syncthreads();
    int off = base_s;
    for (int w = 0; w < wv; ++w) off += wave_sum[w];
    if (m != 0) {
      out_ids[off + pre] = ids[i];
      out_mask[off + pre] = m;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w = 0; w < 1024 / kWave; ++w) t += wave_sum[w];
      base_s += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out_count = base_s;
}

// ---- keyframe selection (Sec. III-F, Eqs. 7-8) ----

// floor(p / g) exactly: the rounded quotient can reach an integer when p is
// just below a cell face, so the estimate is corrected until k g <= p <
// (k + 1) g (k g is exact for the cell numbers that occur).
__device__ inline int64_t cell_floor(double p, double g) {
#pragma clang fp contract(off)
  double k = floor(p / g);
  if (k * g > p) k -= 1.0;
  if ((k + 1.0) * g <= p) k += 1.0;
  return (int64_t)k;
}

// Camera centre -R^T t (each product and sum rounded in order).
__device__ inline void centre_of(const Cam &c, double C[3]) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) C[i] = -((c.R[i] * c.t[0] + c.R[3 + i] * c.t[1]) + c.R[6 + i] * c.t[2]);
}

// One workgroup per keyframe: the 26 separating axes of its frustum, then
// every chunk of the grid against them (the visibility test of the chunk
// selection); visible chunks are looked up in the ascending active ids by
// binary search.  Counts are integers reduced over the workgroup (exact).
constexpr int kKfThreads = 256;
__global__ void __launch_bounds__(kKfThreads)
    k_keyframe_overlap(const Cam *__restrict__ cams, int latest, double g,
                       const uint64_t *__restrict__ ids, int n, double s,
                       const uint64_t *__restrict__ act, int n_act, uint8_t *__restrict__ in_set,
                       int32_t *__restrict__ n_vis, int32_t *__restrict__ n_ov,
                       double *__restrict__ ov) {
  __shared__ ViewAxes va;
  __shared__ int red[2][kKfThreads / kWave];
  const int k = blockIdx.x;
  for (int t = threadIdx.x; t < kAxes; t += blockDim.x) build_axes(cams[k], t, va);
  __syncthreads();
  const int64_t off = int64_t(1) << 20, m21 = (int64_t(1) << 21) - 1;
  const double h = 0.5 * s;
  int nv = 0, no = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const uint64_t id = ids[i];
    const double cc[3] = {double(int64_t((id >> 42) & m21) - off) * s,
                          double(int64_t((id >> 21) & m21) - off) * s,
                          double(int64_t(id & m21) - off) * s};
    if (!box_meets(va, cc, h)) continue;
    ++nv;
    int lo = 0, hi = n_act;  // first active id >= id
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (act[mid] < id) lo = mid + 1;
      else hi = mid;
    }
    no += (lo < n_act && act[lo] == id) ? 1 : 0;
  }
  for (int o = kWave / 2; o > 0; o >>= 1) {
    nv += __shfl_xor(nv, o);
    no += __shfl_xor(no, o);
  }
  if ((threadIdx.x & (kWave - 1)) == 0) {
    red[0][threadIdx.x / kWave] = nv;
    red[1][threadIdx.x / kWave] = no;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  int tv = 0, to = 0;
  for (int w = 0; w < kKfThreads / kWave; ++w) {
    tv += red[0][w];
    to += red[1][w];
  }
  n_vis[k] = tv;
  n_ov[k] = to;
  ov[k] = tv > 0 ? (double)to / (double)tv : 1.0;  // Eq. (7); nothing to load when nothing is seen
  double ck[3], cl[3];
  centre_of(cams[k], ck);
  centre_of(cams[latest], cl);
  bool same = true;
  for (int a = 0; a < 3; ++a) same = same && cell_floor(ck[a], g) == cell_floor(cl[a], g);
  in_set[k] = same ? 1 : 0;  // Eq. (8): k in K(p_latest)
}

}  // namespace

void keyframe_overlap(dcgs_ctx *ctx, const dcgs_camera *kf, int n_kf, int latest, double g,
                      const uint64_t *ids, int n, double s, const uint64_t *act, int n_act,
                      uint8_t *in_set, int32_t *n_visible, int32_t *n_overlap, double *overlap,
                      int n_window, int32_t *window, int32_t *n_window_out, hipStream_t st) {
  // device block: cameras, active ids, then the outputs (8-byte aligned parts)
  const size_t cam_b = (size_t)n_kf * sizeof(Cam), act_b = (size_t)n_act * sizeof(uint64_t);
  const size_t out_b = (size_t)n_kf * (sizeof(double) + 2 * sizeof(int32_t) + 8);
  uint8_t *d = ctx->kf_buf.need(cam_b + act_b + out_b + 64);
  Cam *d_cam = reinterpret_cast<Cam *>(d);
  uint64_t *d_act = reinterpret_cast<uint64_t *>(d + cam_b);
  double *d_ov = reinterpret_cast<double *>(d + cam_b + act_b);
  int32_t *d_nv = reinterpret_cast<int32_t *>(d_ov + n_kf);
  int32_t *d_no = d_nv + n_kf;
  uint8_t *d_in = reinterpret_cast<uint8_t *>(d_no + n_kf);
  std::vector<Cam> hc((size_t)n_kf);
  for (int k = 0; k < n_kf; ++k) hc[k] = to_cam(kf[k]);
  DCGS_HIP(hipMemcpyAsync(d_cam, hc.data(), cam_b, hipMemcpyHostToDevice, st));
  if (n_act > 0) DCGS_HIP(hipMemcpyAsync(d_act, act, act_b, hipMemcpyHostToDevice, st));
  hipLaunchKernelGGL(k_keyframe_overlap, dim3((unsigned)n_kf), dim3(kKfThreads), 0, st, d_cam,
                     latest, g, ids, n, s, d_act, n_act, d_in, d_nv, d_no, d_ov);
  DCGS_LAUNCH_CHECK();
  std::vector<double> h_ov((size_t)n_kf);
  std::vector<int32_t> h_nv((size_t)n_kf), h_no((size_t)n_kf);
  std::vector<uint8_t> h_in((size_t)n_kf);
  DCGS_HIP(hipMemcpyAsync(h_ov.data(), d_ov, n_kf * sizeof(double), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipMemcpyAsync(h_nv.data(), d_nv, n_kf * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipMemcpyAsync(h_no.data(), d_no, n_kf * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipMemcpyAsync(h_in.data(), d_in, (size_t)n_kf, hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  if (in_set) std::copy(h_in.begin(), h_in.end(), in_set);
  if (n_visible) std::copy(h_nv.begin(), h_nv.end(), n_visible);
  if (n_overlap) std::copy(h_no.begin(), h_no.end(), n_overlap);
  if (overlap) std::copy(h_ov.begin(), h_ov.end(), overlap);
  if (window) {
    // the window: candidates of K(p_latest), highest overlap first, ties to
    // the more recent (higher) keyframe
    std::vector<int32_t> cand;
    for (int k = 0; k < n_kf; ++k)
      if (h_in[k]) cand.push_back(k);
    std::stable_sort(cand.begin(), cand.end(), [&](int32_t a, int32_t b) {
      return h_ov[a] != h_ov[b] ? h_ov[a] > h_ov[b] : a > b;
    });
    const int m = std::min<int>(n_window, (int)cand.size());
    for (int i = 0; i < m; ++i) window[i] = cand[i];
    if (n_window_out) *n_window_out = m;
  }
}

void launch_chunk_ids(const float *mean, int64_t n, int64_t stride, double s,
                      uint64_t *out, int *flag, hipStream_t st) {
  if (n == 0) return;
  int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_chunk_ids, dim3((unsigned)blocks), dim3(256), 0, st,
                     mean, n, stride, s, out, flag);
  DCGS_LAUNCH_CHECK();
}

void launch_select_mask(const dcgs_camera *cams, int n_views, const uint64_t *ids,
                        int n_chunks, double s, uint16_t *mask, hipStream_t st) {
  if (n_chunks <= 0) return;
  DCGS_CHECK(n_views >= 1 && n_views <= kMaxViews, DCGS_E_INVALID, "select: 1..16 views");
  CamSet args{};
  for (int v = 0; v < n_views; ++v) args.c[v] = to_cam(cams[v]);
  const int blocks = (n_chunks + 255) / 256;
  hipLaunchKernelGGL(k_select_mask, dim3(blocks), dim3(256), 0, st, args, n_views, ids,
                     n_chunks, s, mask);
  DCGS_LAUNCH_CHECK();
}

void launch_select(const dcgs_camera *cams, int n_views, const uint64_t *ids,
                   int n_chunks, double s, uint16_t *mask_tmp,
                   uint64_t *out_ids, uint16_t *out_mask, int32_t *out_count,
                   hipStream_t st) {
  launch_select_mask(cams, n_views, ids, n_chunks, s, mask_tmp, st);
  hipLaunchKernelGGL(k_select_compact, dim3(1), dim3(1024), 0, st, ids,
                     mask_tmp, n_chunks, out_ids, out_mask, out_count);
  DCGS_LAUNCH_CHECK();
}

}  // namespace dcgs
