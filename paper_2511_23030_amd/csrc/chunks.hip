// Chunk IDs (Sec. III-D, Eqs. 5-6) and visible-chunk selection
// (Sec. III-D "Frustum Culling") for gfx950.
#include "internal.h"

namespace dcgs {
namespace {

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

struct Cam {
  double R[9], t[3], fx, fy, cx, cy, W, H, zn, zf;
};

constexpr int kAxes = 26;

struct CamSet {
  Cam c[kMaxViews];
};

struct ViewAxes {
  double a[kAxes][3];
  double lo[kAxes], hi[kAxes];
};

__device__ inline void corner(const Cam &c, int k, double P[3]) {
  const double Z = (k & 4) ? c.zf : c.zn;
  const double u = (k & 1) ? c.W : 0.0, v = (k & 2) ? c.H : 0.0;
  const double X = (u - c.cx) * Z / c.fx, Y = (v - c.cy) * Z / c.fy;
  const double d0 = X - c.t[0], d1 = Y - c.t[1], d2 = Z - c.t[2];
  // world = R^T (Xc - t)
  P[0] = c.R[0] * d0 + c.R[3] * d1 + c.R[6] * d2;
  P[1] = c.R[1] * d0 + c.R[4] * d1 + c.R[7] * d2;
  P[2] = c.R[2] * d0 + c.R[5] * d1 + c.R[8] * d2;
}

__device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

// Candidate separating axes of an axis-aligned box and a frustum: the box
// face normals, the frustum face normals, and the cross products of the box
// edge directions with the frustum edge directions.
__device__ void make_axis(const Cam &c, int ax, double out[3]) {
  double P[8][3];
  for (int k = 0; k < 8; ++k) corner(c, k, P[k]);
  auto edge = [&](int xy, double e[3]) {  // side edge through image corner xy
    e[0] = P[4 + xy][0] - P[xy][0];
    e[1] = P[4 + xy][1] - P[xy][1];
    e[2] = P[4 + xy][2] - P[xy][2];
  };
  double fe[6][3];
  for (int k = 0; k < 4; ++k) edge(k, fe[k]);
  for (int j = 0; j < 3; ++j) {
    fe[4][j] = c.R[j];      // camera x axis (world)
    fe[5][j] = c.R[3 + j];  // camera y axis (world)
  }
  if (ax < 3) {
    out[0] = ax == 0;
    out[1] = ax == 1;
    out[2] = ax == 2;
  } else if (ax == 3) {
    for (int j = 0; j < 3; ++j) out[j] = c.R[6 + j];
  } else if (ax < 8) {
    // side planes u=0 (corners 0,2), u=W (1,3), v=0 (0,1), v=H (2,3)
    const int pa[4] = {0, 1, 0, 2}, pb[4] = {2, 3, 1, 3};
    cross3(fe[pa[ax - 4]], fe[pb[ax - 4]], out);
  } else {
    int k = ax - 8;
    double b[3] = {double((k / 6) == 0), double((k / 6) == 1), double((k / 6) == 2)};
    cross3(b, fe[k % 6], out);
  }
}

__global__ void k_select_mask(CamSet cs, int n_views,
                              const uint64_t *__restrict__ ids, int n,
                              double s, uint16_t *__restrict__ mask) {
  __shared__ ViewAxes va[kMaxViews];
  const Cam *cams = cs.c;
  for (int t = threadIdx.x; t < n_views * kAxes; t += blockDim.x) {
    int v = t / kAxes, ax = t % kAxes;
    double a[3];
    make_axis(cams[v], ax, a);
    double lo = 1e300, hi = -1e300;
    for (int k = 0; k < 8; ++k) {
      double P[3];
      corner(cams[v], k, P);
      double d = a[0] * P[0] + a[1] * P[1] + a[2] * P[2];
      lo = fmin(lo, d);
      hi = fmax(hi, d);
    }
    va[v].a[ax][0] = a[0];
    va[v].a[ax][1] = a[1];
    va[v].a[ax][2] = a[2];
    va[v].lo[ax] = lo;
    va[v].hi[ax] = hi;
  }
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
  for (int v = 0; v < n_views; ++v) {
    bool sep = false;
    for (int ax = 0; ax < kAxes && !sep; ++ax) {
      const double *a = va[v].a[ax];
      double c = a[0] * cc[0] + a[1] * cc[1] + a[2] * cc[2];
      double r = h * (fabs(a[0]) + fabs(a[1]) + fabs(a[2]));
      sep = (c + r < va[v].lo[ax]) || (c - r > va[v].hi[ax]);
    }
    if (!sep) m |= 1u << v;
  }
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

void launch_select(const dcgs_camera *cams, int n_views, const uint64_t *ids,
                   int n_chunks, double s, uint16_t *mask_tmp,
                   uint64_t *out_ids, uint16_t *out_mask, int32_t *out_count,
                   hipStream_t st) {
  CamSet args{};
  for (int v = 0; v < n_views; ++v) {
    Cam &c = args.c[v];
    for (int j = 0; j < 9; ++j) c.R[j] = cams[v].R[j];
    for (int j = 0; j < 3; ++j) c.t[j] = cams[v].t[j];
    c.fx = cams[v].fx;
    c.fy = cams[v].fy;
    c.cx = cams[v].cx;
    c.cy = cams[v].cy;
    c.W = cams[v].width;
    c.H = cams[v].height;
    c.zn = cams[v].z_near;
    c.zf = cams[v].z_far;
  }
  if (n_chunks > 0) {
    int blocks = (n_chunks + 255) / 256;
    hipLaunchKernelGGL(k_select_mask, dim3(blocks), dim3(256), 0, st, args,
                       n_views, ids, n_chunks, s, mask_tmp);
    DCGS_LAUNCH_CHECK();
  }
  hipLaunchKernelGGL(k_select_compact, dim3(1), dim3(1024), 0, st, ids,
                     mask_tmp, n_chunks, out_ids, out_mask, out_count);
  DCGS_LAUNCH_CHECK();
}

}  // namespace dcgs
