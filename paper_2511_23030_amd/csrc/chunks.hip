// Chunk IDs (Sec. III-D, Eqs. 5-6) and visible-chunk selection
// (Sec. III-D "Frustum Culling") for gfx950.
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

}  // namespace

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
