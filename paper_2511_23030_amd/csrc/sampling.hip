// The LoG sampling map of the Sampling section for gfx950: where the input
// image has Laplacian-of-Gaussian detail that the current render lacks,
// P_s = max(P_L - P~, 0), and the pixels a per-pixel uniform draw selects.
//
// P_L = min(1, beta |LoG(image)|), P~ = min(1, beta |LoG(render)|), |.| the
// Euclidean norm over the three colour channels of the per-channel LoG; the
// LoG is the sum of the second-derivative Gaussian filter along rows (with
// the Gaussian along columns) and along columns (with the Gaussian along
// rows), mirror boundary with the edge sample repeated.  One 256-thread
// workgroup per 16 x 16 tile stages each channel with its halo in LDS and
// runs the two separable passes; selected pixels are listed in raster order
// by a scan of per-pixel flags.
#include <cmath>

#include "internal.h"

namespace dcgs {
namespace {

constexpr int kT = 16;
constexpr int kMaxR = 12;                 // sigma <= 3
constexpr int kMaxS = kT + 2 * kMaxR;

struct LogTaps {
  float g[2 * kMaxR + 1], d2[2 * kMaxR + 1];
  int r;
};

__device__ inline int mirror(int i, int n) {
  // "d c b a | a b c d": -1 -> 0, n -> n - 1 (valid for |overhang| <= n)
  if (i < 0) i = -i - 1;
  if (i >= n) i = 2 * n - 1 - i;
  return i < 0 ? 0 : (i >= n ? n - 1 : i);
}

__global__ void __launch_bounds__(256)
    k_log_map(const float *__restrict__ image, const float *__restrict__ render,
              const float *__restrict__ u, int W, int H, LogTaps taps, float beta,
              float *__restrict__ ps, uint32_t *__restrict__ flag) {
  __shared__ float s[kMaxS][kMaxS + 1];
  __shared__ float hg[kMaxS][kT + 1], hd[kMaxS][kT + 1];
  const int r = taps.r, S = kT + 2 * r;
  const int x0 = blockIdx.x * kT - r, y0 = blockIdx.y * kT - r;
  const int tr = threadIdx.x / kT, tc = threadIdx.x % kT;
  const int64_t HW = (int64_t)W * H;
  float ss[2] = {0.f, 0.f};  // sum of squares over channels: image, render
  for (int src = 0; src < 2; ++src) {
    const float *img = src == 0 ? image : render;
    for (int c = 0; c < 3; ++c) {
      __syncthreads();
      for (int e = threadIdx.x; e < S * S; e += blockDim.x) {
        const int rr = e / S, cc = e - rr * S;
        s[rr][cc] = img[c * HW + (int64_t)mirror(y0 + rr, H) * W + mirror(x0 + cc, W)];
      }
      __syncthreads();
      for (int e = threadIdx.x; e < S * kT; e += blockDim.x) {
        const int rr = e / kT, cc = e - rr * kT;
        float a = 0.f, b = 0.f;
        for (int k = 0; k <= 2 * r; ++k) {
          const float v = s[rr][cc + k];
          a = fmaf(taps.g[k], v, a);
          b = fmaf(taps.d2[k], v, b);
        }
        hg[rr][cc] = a;
        hd[rr][cc] = b;
      }
      __syncthreads();
      float lap = 0.f;
      for (int k = 0; k <= 2 * r; ++k) {
        lap = fmaf(taps.g[k], hd[tr + k][tc], lap);   // d2 along rows, g along columns
        lap = fmaf(taps.d2[k], hg[tr + k][tc], lap);  // g along rows, d2 along columns
      }
      ss[src] = fmaf(lap, lap, ss[src]);
    }
  }
  const int px = blockIdx.x * kT + tc, py = blockIdx.y * kT + tr;
  if (px >= W || py >= H) return;
  const float pl = fminf(1.0f, beta * sqrtf(ss[0]));
  const float pt = fminf(1.0f, beta * sqrtf(ss[1]));
  const float p = fmaxf(pl - pt, 0.0f);
  const int64_t o = (int64_t)py * W + px;
  if (ps) ps[o] = p;
  flag[o] = u[o] < p ? 1u : 0u;
}

__global__ void k_list_flags(const uint32_t *__restrict__ flag, const uint32_t *__restrict__ pos,
                             int64_t n, int32_t *__restrict__ out, int32_t *__restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && flag[i]) out[pos[i]] = (int32_t)i;
  if (i == 0) *count = (int32_t)pos[n];
}

LogTaps make_taps(double sigma) {
  LogTaps t{};
  t.r = (int)std::ceil(4.0 * sigma);
  double g[2 * kMaxR + 1], sum = 0.0;
  for (int k = -t.r; k <= t.r; ++k) {
    g[k + t.r] = std::exp(-0.5 * k * k / (sigma * sigma));
    sum += g[k + t.r];
  }
  for (int k = -t.r; k <= t.r; ++k) {
    const double gn = g[k + t.r] / sum;
    t.g[k + t.r] = (float)gn;
    t.d2[k + t.r] = (float)((k * k / std::pow(sigma, 4) - 1.0 / (sigma * sigma)) * gn);
  }
  return t;
}

}  // namespace

void sample_pixels(dcgs_ctx *ctx, const float *image, const float *render, const float *u,
                   int H, int W, double beta, double sigma, float *ps, int32_t *out_idx,
                   int32_t *out_count, hipStream_t st) {
  DCGS_CHECK(image && render && u && out_idx && out_count && H > 0 && W > 0 && beta > 0 &&
                 sigma > 0 && std::ceil(4.0 * sigma) <= kMaxR,
             DCGS_E_INVALID, "sample_pixels: bad args (sigma at most 3)");
  DCGS_CHECK((int64_t)std::ceil(4.0 * sigma) < std::min(H, W), DCGS_E_INVALID,
             "sample_pixels: image smaller than the filter");
  const int64_t n = (int64_t)W * H;
  DCGS_CHECK(n < (int64_t(1) << 31), DCGS_E_INVALID, "sample_pixels: image too large");
  uint32_t *flag = ctx->samp.need(2 * (size_t)n + 2);
  uint32_t *pos = flag + n;
  uint32_t *part = ctx->scan_part.need(scan_part_size(n) + 2);
  const dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT);
  hipLaunchKernelGGL(k_log_map, grid, dim3(256), 0, st, image, render, u, W, H,
                     make_taps(sigma), (float)beta, ps, flag);
  DCGS_LAUNCH_CHECK();
  scan_u32(flag, nullptr, pos, n, part, st);
  hipLaunchKernelGGL(k_list_flags, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, flag,
                     pos, n, out_idx, out_count);
  DCGS_LAUNCH_CHECK();
}

}  // namespace dcgs
