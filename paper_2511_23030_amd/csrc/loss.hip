// The mapping loss of Eqs. (2)-(4) with its gradient for gfx950:
// (1 - lambda_s) L1 + lambda_s (1 - SSIM) on colour plus lambda_depth L1 on
// depth, each view's terms averaged over its own pixels and summed over the
// views of a window.
//
// SSIM uses the 11-tap Gaussian window (sigma 1.5) applied separably with
// zero padding, C1 = 0.01^2, C2 = 0.03^2.  Forward and backward are image
// stencils: one 256-thread workgroup per 32 x 32 output tile of one colour
// plane stages the tile plus a 5-pixel halo in LDS (1.7 reads per pixel),
// blurs rows, then columns, each thread finishing four vertically adjacent
// pixels from one sweep of 14 staged rows.  The forward writes, per pixel, the derivatives of that pixel's
// SSIM with respect to the three local moments (mean, mean of squares, mean
// of products); the backward blurs those maps again (the window is
// symmetric, so the adjoint of the blur is the blur) and combines them with
// the pixel values.  Sums run in a fixed order (block partials, then one
// float64 pass), so losses and gradients are deterministic.
#include "internal.h"

namespace dcgs {
namespace {

constexpr int kT = 32;           // output tile side
constexpr int kPP = kT * kT / 256;  // output pixels per thread (a column run)
constexpr int kR = 5;            // window radius
constexpr int kS = kT + 2 * kR;  // staged side
constexpr float kC1 = 0.01f * 0.01f;
constexpr float kC2 = 0.03f * 0.03f;

struct Window11 {
  float g[11];
};

// Sum of one float per thread over a 256-thread workgroup in a fixed order
// (wavefront butterflies, then the four wavefront totals in order); every
// thread gets the total.  red: kWave-strided scratch of 4 floats.
__device__ inline float block_sum(float v, float *red) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v += __shfl_xor(v, off);
  __syncthreads();  // red may still be read by an earlier call's threads
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}

// Stage an (kS x kS) region of a plane (zero outside) for up to 3 inputs.
template <int NIN>
__device__ inline void stage(const float *const (&in)[NIN], int W, int H, int x0, int y0,
                             float (&s)[NIN][kS][kS + 1]) {
  for (int e = threadIdx.x; e < kS * kS; e += blockDim.x) {
    const int r = e / kS, c = e - r * kS;
    const int px = x0 + c, py = y0 + r;
    const bool in_img = px >= 0 && px < W && py >= 0 && py < H;
#pragma unroll
    for (int q = 0; q < NIN; ++q) s[q][r][c] = in_img ? in[q][(int64_t)py * W + px] : 0.0f;
  }
}

// Forward: SSIM of every pixel of one colour plane and its derivatives with
// respect to the local moments m_x = G*x, m_xx = G*(x x), m_xy = G*(x y):
// a = dS/dm_x, b = dS/dm_xx, c = dS/dm_xy.  part[block] = sum of S.
__global__ void __launch_bounds__(256)
    k_ssim_fwd(const float *__restrict__ x, const float *__restrict__ y, int W, int H,
               Window11 win, float *__restrict__ amap, float *__restrict__ bmap,
               float *__restrict__ cmap, float *__restrict__ part) {
  __shared__ float s[2][kS][kS + 1];
  __shared__ float h[5][kS][kT + 1];
  __shared__ float red[256 / kWave];
  const int64_t HW = (int64_t)W * H;
  const int64_t plane = blockIdx.z;
  x += plane * HW;
  y += plane * HW;
  const int x0 = blockIdx.x * kT - kR, y0 = blockIdx.y * kT - kR;
  const float *const in[2] = {x, y};
  stage<2>(in, W, H, x0, y0, s);
  __syncthreads();
  // rows: 5 moments of the staged rows at the tile's columns
  for (int e = threadIdx.x; e < kS * kT; e += blockDim.x) {
    const int r = e / kT, c = e - r * kT;
    float mx = 0.f, my = 0.f, mxx = 0.f, myy = 0.f, mxy = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float a = s[0][r][c + k], b = s[1][r][c + k], g = win.g[k];
      mx = fmaf(g, a, mx);
      my = fmaf(g, b, my);
      mxx = fmaf(g, a * a, mxx);
      myy = fmaf(g, b * b, myy);
      mxy = fmaf(g, a * b, mxy);
    }
    h[0][r][c] = mx;
    h[1][r][c] = my;
    h[2][r][c] = mxx;
    h[3][r][c] = myy;
    h[4][r][c] = mxy;
  }
  __syncthreads();
  // columns: thread (c, r0) finishes rows r0 .. r0 + kPP - 1 of column c;
  // every output sums its 11 taps in order
  const int c = threadIdx.x % kT, r0 = (threadIdx.x / kT) * kPP;
  float m[kPP][5];
#pragma unroll
  for (int p = 0; p < kPP; ++p)
#pragma unroll
    for (int q = 0; q < 5; ++q) m[p][q] = 0.0f;
#pragma unroll
  for (int k = 0; k < 11 + kPP - 1; ++k) {
    float hv[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) hv[q] = h[q][r0 + k][c];
#pragma unroll
    for (int p = 0; p < kPP; ++p)
      if (k - p >= 0 && k - p < 11) {
        const float g = win.g[k - p];
#pragma unroll
        for (int q = 0; q < 5; ++q) m[p][q] = fmaf(g, hv[q], m[p][q]);
      }
  }
  float S_sum = 0.0f;
#pragma unroll
  for (int p = 0; p < kPP; ++p) {
    const int px = blockIdx.x * kT + c, py = blockIdx.y * kT + r0 + p;
    if (px < W && py < H) {
      const float mx = m[p][0], my = m[p][1];
      const float sx = m[p][2] - mx * mx, sy = m[p][3] - my * my, sxy = m[p][4] - mx * my;
      const float A1 = 2.0f * mx * my + kC1, A2 = 2.0f * sxy + kC2;
      const float B1 = mx * mx + my * my + kC1, B2 = sx + sy + kC2;
      const float iB = 1.0f / (B1 * B2);
      const float S = A1 * A2 * iB;
      const int64_t o = plane * HW + (int64_t)py * W + px;
      // S(m_x, m_xx, m_xy) with sx = m_xx - m_x^2 and sxy = m_xy - m_x m_y
      amap[o] = 2.0f * my * (A2 - A1) * iB - 2.0f * mx * S * (1.0f / B1 - 1.0f / B2);
      bmap[o] = -S / B2;
      cmap[o] = 2.0f * A1 * iB;
      S_sum += S;
    }
  }
  const float tot = block_sum(S_sum, red);
  if (threadIdx.x == 0)
    part[(plane * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = tot;
}

// Backward: dl/dx = w1 sign(x - y) - ws ((G*a) + 2 x (G*b) + y (G*c)) with
// w1 = (1 - lambda_s) / (3HW), ws = lambda_s / (3HW).  Also per-block sums
// of |x - y| and of the squared error with x clipped to [0, 1].
__global__ void __launch_bounds__(256)
    k_ssim_bwd(const float *__restrict__ x, const float *__restrict__ y,
               const float *__restrict__ amap, const float *__restrict__ bmap,
               const float *__restrict__ cmap, int W, int H, Window11 win, float w1, float ws,
               float *__restrict__ dl, float *__restrict__ part) {
  __shared__ float s[3][kS][kS + 1];
  __shared__ float h[3][kS][kT + 1];
  __shared__ float red[2][256 / kWave];
  const int64_t HW = (int64_t)W * H;
  const int64_t plane = blockIdx.z;
  const int x0 = blockIdx.x * kT - kR, y0 = blockIdx.y * kT - kR;
  const float *const in[3] = {amap + plane * HW, bmap + plane * HW, cmap + plane * HW};
  stage<3>(in, W, H, x0, y0, s);
  __syncthreads();
  for (int e = threadIdx.x; e < kS * kT; e += blockDim.x) {
    const int r = e / kT, c = e - r * kT;
    float v0 = 0.f, v1 = 0.f, v2 = 0.f;
#pragma unroll
    for (int k = 0; k < 11; ++k) {
      const float g = win.g[k];
      v0 = fmaf(g, s[0][r][c + k], v0);
      v1 = fmaf(g, s[1][r][c + k], v1);
      v2 = fmaf(g, s[2][r][c + k], v2);
    }
    h[0][r][c] = v0;
    h[1][r][c] = v1;
    h[2][r][c] = v2;
  }
  __syncthreads();
  const int c = threadIdx.x % kT, r0 = (threadIdx.x / kT) * kPP;
  float gsum[kPP][3];
#pragma unroll
  for (int p = 0; p < kPP; ++p) gsum[p][0] = gsum[p][1] = gsum[p][2] = 0.0f;
#pragma unroll
  for (int k = 0; k < 11 + kPP - 1; ++k) {
    const float h0 = h[0][r0 + k][c], h1 = h[1][r0 + k][c], h2 = h[2][r0 + k][c];
#pragma unroll
    for (int p = 0; p < kPP; ++p)
      if (k - p >= 0 && k - p < 11) {
        const float g = win.g[k - p];
        gsum[p][0] = fmaf(g, h0, gsum[p][0]);
        gsum[p][1] = fmaf(g, h1, gsum[p][1]);
        gsum[p][2] = fmaf(g, h2, gsum[p][2]);
      }
  }
  float a1 = 0.0f, a2 = 0.0f;
#pragma unroll
  for (int p = 0; p < kPP; ++p) {
    const int px = blockIdx.x * kT + c, py = blockIdx.y * kT + r0 + p;
    if (px < W && py < H) {
      const int64_t o = plane * HW + (int64_t)py * W + px;
      const float xv = x[o], yv = y[o], d = xv - yv;
      const float sg = d > 0.0f ? 1.0f : (d < 0.0f ? -1.0f : 0.0f);
      dl[o] = w1 * sg - ws * (gsum[p][0] + 2.0f * xv * gsum[p][1] + yv * gsum[p][2]);
      a1 += fabsf(d);
      const float e = fminf(fmaxf(xv, 0.0f), 1.0f) - yv;
      a2 += e * e;
    }
  }
  const float t1 = block_sum(a1, red[0]);
  const float t2 = block_sum(a2, red[1]);
  if (threadIdx.x == 0) {
    const int64_t b = (plane * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    part[2 * b] = t1;
    part[2 * b + 1] = t2;
  }
}

// Depth term: dl = wd sign(D - D_gt), wd = lambda_depth / (HW); per-block
// sums of |D - D_gt| (grid-stride, fixed order).
__global__ void __launch_bounds__(256)
    k_depth_l1(const float *__restrict__ d, const float *__restrict__ t, int64_t count, float wd,
               float *__restrict__ dl, float *__restrict__ part) {
  __shared__ float red[256];
  float a = 0.0f;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float e = d[i] - t[i];
    if (dl) dl[i] = e > 0.0f ? wd : (e < 0.0f ? -wd : 0.0f);
    a += fabsf(e);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out = sum of n partials (stride `step`, offset `off`) in float64, one block.
__global__ void __launch_bounds__(1024)
    k_sum_parts(const float *__restrict__ part, int64_t n, int step, int off,
                double *__restrict__ out) {
  // thread t sums elements t, t + 1024, ... (eight loads in flight per
  // step), then a fixed tree over the 1024 threads
  __shared__ double red[1024];
  double a = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 7 * 1024 < n; i += 8 * 1024) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[(i + u * 1024) * step + off];
#pragma unroll
    for (int u = 0; u < 8; ++u) a += v[u];
  }
  for (; i < n; i += 1024) a += part[i * step + off];
  red[threadIdx.x] = a;
  __syncthreads();
  for (int k = 512; k > 0; k >>= 1) {
    if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

Window11 make_window() {
  Window11 w{};
  double g[11], s = 0.0;
  for (int k = 0; k < 11; ++k) {
    const double d = k - 5.0;
    g[k] = std::exp(-d * d / (2.0 * 1.5 * 1.5));
    s += g[k];
  }
  for (int k = 0; k < 11; ++k) w.g[k] = (float)(g[k] / s);
  return w;
}

constexpr int kDepthBlocks = 512;

}  // namespace

// Scratch of mapping_loss for n_views images of H x W (sized ahead of a
// graph capture, where nothing may allocate).
size_t mapping_loss_scratch(int n_views, int H, int W) {
  const int64_t HW = (int64_t)W * H;
  const int planes = 3 * n_views;
  const int64_t nb = (int64_t)((W + kT - 1) / kT) * ((H + kT - 1) / kT) * planes;
  return 3 * (size_t)planes * HW + 3 * nb + kDepthBlocks + 16;
}

void mapping_loss_reserve(int n_views, int H, int W, DevBuf<float> &scratch) {
  scratch.need(mapping_loss_scratch(n_views, H, W));
}

void mapping_loss(dcgs_ctx *ctx, const float *rgb, const float *target, const float *depth,
                  const float *depth_target, int n_views, int H, int W, double lambda_s,
                  double lambda_depth, float *dl_drgb, float *dl_ddepth, double *stats,
                  DevBuf<float> &scratch, hipStream_t st) {
  DCGS_CHECK(rgb && target && dl_drgb && stats && n_views >= 1 && H > 0 && W > 0 &&
                 lambda_s >= 0 && lambda_s <= 1 && lambda_depth >= 0,
             DCGS_E_INVALID, "loss_mapping: bad args");
  DCGS_CHECK(lambda_depth == 0 || (depth && depth_target), DCGS_E_INVALID,
             "loss_mapping: the depth term needs depth and depth_target");
  (void)ctx;
  const int64_t HW = (int64_t)W * H;
  const int planes = 3 * n_views;
  const dim3 grid((W + kT - 1) / kT, (H + kT - 1) / kT, planes);
  const int64_t nb = (int64_t)grid.x * grid.y * grid.z;
  float *maps = scratch.need(mapping_loss_scratch(n_views, H, W));
  float *amap = maps, *bmap = amap + planes * HW, *cmap = bmap + planes * HW;
  float *pS = cmap + planes * HW, *pL = pS + nb, *pD = pL + 2 * nb;
  const Window11 win = make_window();
  const float norm = (float)(1.0 / (3.0 * (double)HW));
  hipLaunchKernelGGL(k_ssim_fwd, grid, dim3(256), 0, st, rgb, target, W, H, win, amap, bmap,
                     cmap, pS);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_ssim_bwd, grid, dim3(256), 0, st, rgb, target, amap, bmap, cmap, W, H,
                     win, (float)(1.0 - lambda_s) * norm, (float)lambda_s * norm, dl_drgb, pL);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, pL, nb, 2, 0, stats);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, pL, nb, 2, 1, stats + 1);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, pS, nb, 1, 0, stats + 2);
  DCGS_LAUNCH_CHECK();
  if (depth && depth_target) {
    hipLaunchKernelGGL(k_depth_l1, dim3(kDepthBlocks), dim3(256), 0, st, depth, depth_target,
                       (int64_t)n_views * HW, (float)(lambda_depth / (double)HW), dl_ddepth, pD);
    DCGS_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, pD, (int64_t)kDepthBlocks, 1, 0,
                       stats + 3);
    DCGS_LAUNCH_CHECK();
  } else {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, st, pD, (int64_t)0, 1, 0, stats + 3);
    DCGS_LAUNCH_CHECK();
  }
}

}  // namespace dcgs
