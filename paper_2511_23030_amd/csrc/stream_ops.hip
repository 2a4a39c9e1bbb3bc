// Streaming kernels of the mapping step for gfx950: compaction of resident
// chunks into one SoA buffer (Sec. III-E), the per-Gaussian Adam update with
// scatter back into the resident pool (float64 arithmetic, one rounding per
// stored value), and the L1 image loss (Eqs. 2-4 without SSIM).  All three
// are HBM-bound: coalesced row-wise access, enough workgroups to fill 256
// CUs, no atomics.
#include "internal.h"

namespace dcgs {
namespace {

constexpr int kRowsPerBlock = 8;

// seg = (device page, count in page, destination offset, view mask)
__global__ void __launch_bounds__(256)
    k_compact(const float *__restrict__ pool, int R, const int4 *__restrict__ seg,
              float *__restrict__ out, int64_t out_stride, int32_t *__restrict__ out_src,
              uint16_t *__restrict__ out_gmask) {
  constexpr int PG = dcgs_pool::PG;
  const int4 sg = seg[blockIdx.x];
  const int r0 = blockIdx.y * kRowsPerBlock;
  const float *src = pool + ((int64_t)sg.x * R) * PG;
  for (int r = r0; r < min(R, r0 + kRowsPerBlock); ++r) {
    const float *s = src + (int64_t)r * PG;
    float *d = out + (int64_t)r * out_stride + sg.z;
    for (int k = threadIdx.x; k < sg.y; k += blockDim.x) d[k] = s[k];
  }
  if (blockIdx.y == 0) {
    for (int k = threadIdx.x; k < sg.y; k += blockDim.x) {
      if (out_src) out_src[sg.z + k] = sg.x * PG + k;
      if (out_gmask) out_gmask[sg.z + k] = (uint16_t)sg.w;
    }
  }
}

__device__ inline int group_of_row(int r) {
  return r < 3 ? 0 : r < 6 ? 1 : r < 10 ? 2 : r == 10 ? 3 : r < 14 ? 4 : 5;
}

struct AdamArgs {
  float lr[6];
  float b1, b2, eps;
};

__global__ void __launch_bounds__(256)
    k_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V,
           int32_t *__restrict__ step, int R, const int32_t *__restrict__ src,
           const float *__restrict__ grad, int64_t n, int64_t gs, AdamArgs a,
           const int64_t *__restrict__ cnt) {
  constexpr int PG = dcgs_pool::PG, L2 = dcgs_pool::PG_LOG2;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (cnt) {
    if (cnt[3] != 0) return;  // the window overflowed its pair capacity
    n = min(n, cnt[0]);
  }
  if (i >= n) return;
  const int32_t slot = src[i];
  const int64_t page = slot >> L2, k = slot & (PG - 1);
  const int t = step[page * PG + k] + 1;
  step[page * PG + k] = t;
  // float64 arithmetic from the float32 state and gradient, each result
  // rounded once to float32 (the kernel is bound by its 1.6 KB of traffic
  // per Gaussian, not by these operations)
  const double b1 = a.b1, b2 = a.b2, eps = a.eps;
  const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
  const int64_t base = page * R * PG + k;
  for (int r = 0; r < R; ++r) {
    const double g = grad[r * gs + i];
    const int64_t idx = base + (int64_t)r * PG;
    const double m = b1 * (double)M[idx] + (1.0 - b1) * g;
    const double v = b2 * (double)V[idx] + (1.0 - b2) * (g * g);
    M[idx] = (float)m;
    V[idx] = (float)v;
    const double lr = a.lr[group_of_row(r)];
    P[idx] = (float)((double)P[idx] - lr * (m / bc1) / (sqrt(v / bc2) + eps));
  }
}

constexpr int kLossBlocks = 1024;

__global__ void __launch_bounds__(256)
    k_loss(const float *__restrict__ x, const float *__restrict__ y, int64_t count,
           float inv, float *__restrict__ dl, float *__restrict__ part) {
  __shared__ float s1[256], s2[256];
  float a1 = 0.0f, a2 = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = x[i] - y[i];
    dl[i] = d > 0.0f ? inv : (d < 0.0f ? -inv : 0.0f);
    a1 += fabsf(d);
    const float e = fminf(fmaxf(x[i], 0.0f), 1.0f) - y[i];
    a2 += e * e;
  }
  s1[threadIdx.x] = a1;
  s2[threadIdx.x] = a2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ void __launch_bounds__(256)
    k_loss_final(const float *__restrict__ part, int nb, double *__restrict__ stats) {
  __shared__ double s1[256], s2[256];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  s1[threadIdx.x] = a;
  s2[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      s1[threadIdx.x] += s1[threadIdx.x + h];
      s2[threadIdx.x] += s2[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    stats[0] = s1[0];
    stats[1] = s2[0];
  }
}

}  // namespace

void launch_compact(const float *pool, int R, const int4 *seg, int n_seg, const uint16_t *,
                    float *out, int64_t out_stride, int32_t *out_src, uint16_t *out_gmask,
                    hipStream_t st) {
  if (n_seg == 0) return;
  dim3 grid((unsigned)n_seg, (unsigned)((R + kRowsPerBlock - 1) / kRowsPerBlock));
  hipLaunchKernelGGL(k_compact, grid, dim3(256), 0, st, pool, R, seg, out, out_stride, out_src,
                     out_gmask);
  DCGS_LAUNCH_CHECK();
}

void launch_adam(float *params, float *m, float *v, int32_t *step, int R, const int32_t *src,
                 const float *grad, int64_t n, int64_t grad_stride, const dcgs_adam_config &cfg,
                 hipStream_t st, const int64_t *cnt) {
  if (n == 0) return;
  AdamArgs a{};
  for (int k = 0; k < 6; ++k) a.lr[k] = cfg.lr[k];
  a.b1 = cfg.beta1;
  a.b2 = cfg.beta2;
  a.eps = cfg.eps;
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, m, v,
                     step, R, src, grad, n, grad_stride, a, cnt);
  DCGS_LAUNCH_CHECK();
}

void launch_loss_l1(const float *rgb, const float *target, int64_t count, double norm,
                    float *dl, double *stats, float *part, hipStream_t st) {
  hipLaunchKernelGGL(k_loss, dim3(kLossBlocks), dim3(256), 0, st, rgb, target, count,
                     (float)(1.0 / norm), dl, part);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, part, kLossBlocks, stats);
  DCGS_LAUNCH_CHECK();
}

}  // namespace dcgs
