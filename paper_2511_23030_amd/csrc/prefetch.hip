// Learned chunk prefetch for gfx950: candidate-cell features, exact
// visibility labels (the frustum test of Sec. III-D applied to the next
// frames), and the prefetch MLP 59 -> 256 -> 256 -> 1 (GELU, sigmoid) with
// its backward, loss and Adam.  The dense layers run on the fp32 matrix
// cores (v_mfma_f32_16x16x4_f32); weights are bfloat16 (exact in fp32),
// every accumulation is fp32, and every reduction has a fixed order, so
// results are deterministic.
#include <cmath>

#include "frustum.h"

namespace dcgs {
namespace {

using namespace frustum;

constexpr int kHist = 8;
constexpr int kGX = 64, kGY = 64;
constexpr int kCand = kGX * kGY;  // one horizontal layer of cells
constexpr int kIn = kHist * 7 + 3;
constexpr int kHid = 256;
constexpr double kOffsetUnit = 8.0;
constexpr int kOffW1 = 0, kOffB1 = kHid * kIn, kOffW2 = kOffB1 + kHid,
              kOffB2 = kOffW2 + kHid * kHid, kOffW3 = kOffB2 + kHid, kOffB3 = kOffW3 + kHid,
              kParams = kOffB3 + 1;
constexpr int kBfW1 = 0, kBfW2 = kHid * kIn, kBfW3 = kBfW2 + kHid * kHid,
              kBfTotal = kBfW3 + kHid;
static_assert(kParams == DCGS_MLP_PARAMS, "parameter count");
static_assert(kBfTotal == DCGS_MLP_BF16, "bfloat16 weight count");

__device__ inline float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// float32 -> bfloat16, round to nearest, ties to even (finite inputs).
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ---------------------------------------------------------------------------
// Features and labels
// ---------------------------------------------------------------------------
__device__ inline void centre_of(const Cam &c, double o[3]) {
  for (int j = 0; j < 3; ++j)
    o[j] = -(c.R[j] * c.t[0] + c.R[3 + j] * c.t[1] + c.R[6 + j] * c.t[2]);
}

__device__ inline void base_cell(const Cam &c, double s, int64_t b[3]) {
  double o[3];
  centre_of(c, o);
  for (int a = 0; a < 3; ++a) b[a] = (int64_t)floor((o[a] + 0.5 * s) / s);  // Eq. (5)
}

__device__ inline void cell_of(const int64_t b[3], int q, int64_t c[3]) {
  c[0] = b[0] + (q % kGX) - kGX / 2;
  c[1] = b[1] + (q / kGX) % kGY - kGY / 2;
  c[2] = b[2];
}

__device__ inline uint64_t encode_cell(const int64_t c[3]) {
  const int64_t lo = -(int64_t(1) << 20), hi = (int64_t(1) << 20) - 1;
  if (c[0] < lo || c[0] > hi || c[1] < lo || c[1] > hi || c[2] < lo || c[2] > hi)
    return ~uint64_t(0);
  return (uint64_t(c[0] - lo) << 42) | (uint64_t(c[1] - lo) << 21) | uint64_t(c[2] - lo);
}

// Unit quaternion (w, x, y, z), w >= 0, of a rotation matrix (Shepperd's
// method: divide by the largest of the four diagonal combinations).
__device__ inline void quat_of(const double M[9], double q[4]) {
  const double m00 = M[0], m11 = M[4], m22 = M[8], tr = m00 + m11 + m22;
  double w, x, y, z;
  if (tr >= m00 && tr >= m11 && tr >= m22) {
    w = 0.5 * sqrt(1.0 + tr);
    const double f = 0.25 / w;
    x = (M[7] - M[5]) * f;
    y = (M[2] - M[6]) * f;
    z = (M[3] - M[1]) * f;
  } else if (m00 >= m11 && m00 >= m22) {
    x = 0.5 * sqrt(1.0 + m00 - m11 - m22);
    const double f = 0.25 / x;
    w = (M[7] - M[5]) * f;
    y = (M[1] + M[3]) * f;
    z = (M[2] + M[6]) * f;
  } else if (m11 >= m22) {
    y = 0.5 * sqrt(1.0 - m00 + m11 - m22);
    const double f = 0.25 / y;
    w = (M[2] - M[6]) * f;
    x = (M[1] + M[3]) * f;
    z = (M[5] + M[7]) * f;
  } else {
    z = 0.5 * sqrt(1.0 - m00 - m11 + m22);
    const double f = 0.25 / z;
    w = (M[3] - M[1]) * f;
    x = (M[2] + M[6]) * f;
    y = (M[5] + M[7]) * f;
  }
  const double sg = w < 0 ? -1.0 : 1.0;
  q[0] = sg * w;
  q[1] = sg * x;
  q[2] = sg * y;
  q[3] = sg * z;
}

// One block = 256 candidates of one batch row (frame).  Rows of X are
// [56 pose values | 3 offset values]; the block's 256 rows are contiguous
// and written cooperatively.
__global__ void __launch_bounds__(256)
    k_features(const Cam *__restrict__ cams, const int32_t *__restrict__ frames, double s,
               double pos_unit, const uint8_t *__restrict__ labels, float *__restrict__ X,
               uint64_t *__restrict__ ids, uint8_t *__restrict__ y) {
  __shared__ float pose[kHist * 7];
  __shared__ float offs[256][3];
  const int f = blockIdx.y;
  const int t = frames[f];
  const Cam &c0 = cams[t];
  double o0[3];
  centre_of(c0, o0);
  if (threadIdx.x < kHist) {
    const int k = threadIdx.x;
    const Cam &ck = cams[t - k < 0 ? 0 : t - k];
    double ok[3], d[3];
    centre_of(ck, ok);
    for (int j = 0; j < 3; ++j) d[j] = ok[j] - o0[j];
    for (int i = 0; i < 3; ++i)
      pose[k * 7 + i] =
          (float)((c0.R[3 * i] * d[0] + c0.R[3 * i + 1] * d[1] + c0.R[3 * i + 2] * d[2]) /
                  pos_unit);
    double M[9], q[4];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        M[3 * i + j] = c0.R[3 * i] * ck.R[3 * j] + c0.R[3 * i + 1] * ck.R[3 * j + 1] +
                       c0.R[3 * i + 2] * ck.R[3 * j + 2];
    quat_of(M, q);
    for (int j = 0; j < 4; ++j) pose[k * 7 + 3 + j] = (float)q[j];
  }
  const int q = blockIdx.x * 256 + threadIdx.x;
  int64_t b[3], c[3];
  base_cell(c0, s, b);
  cell_of(b, q, c);
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = (double)c[a] * s - o0[a];
  for (int i = 0; i < 3; ++i)
    offs[threadIdx.x][i] =
        (float)((c0.R[3 * i] * d[0] + c0.R[3 * i + 1] * d[1] + c0.R[3 * i + 2] * d[2]) /
                (kOffsetUnit * s));
  const int64_t row = (int64_t)f * kCand + q;
  if (ids) ids[row] = encode_cell(c);
  if (y) y[row] = labels[(int64_t)t * kCand + q];
  __syncthreads();
  float *Xb = X + ((int64_t)f * kCand + blockIdx.x * 256) * kIn;
  for (int e = threadIdx.x; e < 256 * kIn; e += 256) {
    const int r = e / kIn, col = e - r * kIn;
    Xb[e] = col < kHist * 7 ? pose[col] : offs[r][col - kHist * 7];
  }
}

// labels[t][q] = 1 when candidate q of frame t meets the frustum of one of
// frames t+1 .. t+horizon.  Block = 256 candidates of frame t0 + blockIdx.y.
__global__ void __launch_bounds__(256)
    k_labels(const Cam *__restrict__ cams, int n_frames, int t0, int horizon, double s,
             uint8_t *__restrict__ labels) {
  __shared__ ViewAxes va[kMaxViews];
  const int t = t0 + blockIdx.y;
  const int nv = min(horizon, n_frames - 1 - t);
  for (int e = threadIdx.x; e < nv * kAxes; e += blockDim.x)
    build_axes(cams[t + 1 + e / kAxes], e % kAxes, va[e / kAxes]);
  __syncthreads();
  const int q = blockIdx.x * 256 + threadIdx.x;
  int64_t b[3], c[3];
  base_cell(cams[t], s, b);
  cell_of(b, q, c);
  const double cc[3] = {(double)c[0] * s, (double)c[1] * s, (double)c[2] * s};
  bool vis = false;
  for (int v = 0; v < nv && !vis; ++v) vis = box_meets(va[v], cc, 0.5 * s);
  labels[(int64_t)t * kCand + q] = vis ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Dense layers on the fp32 matrix cores
// ---------------------------------------------------------------------------
typedef float f32x4 __attribute__((ext_vector_type(4)));

enum { EPI_STORE = 0, EPI_BIAS_GELU = 1, EPI_GELU_GRAD = 2 };

template <typename TB>
__device__ inline float load_b(const TB *p);
template <>
__device__ inline float load_b<float>(const float *p) { return *p; }
template <>
__device__ inline float load_b<uint16_t>(const uint16_t *p) { return bf16_to_f32(*p); }

// C[M][N] (row stride ldc) = A[M][K] * B[K][N] with element (m, k) of A at
// A[m*sam + k*sak] and (k, n) of B at B[k*sbk + n*sbn].  64 x 64 tile per
// 256-thread block (2 x 2 waves of 32 x 32, each 2 x 2 MFMA 16x16x4 tiles),
// K staged through LDS 16 at a time.  blockIdx.z splits K into slices of
// k_slice; slice z writes C + z * M * ldc (partials, summed later in order).
// Epilogues: EPI_STORE writes the sum; EPI_BIAS_GELU writes z = sum + bias[n]
// to C and GELU(z) to C2; EPI_GELU_GRAD writes sum * GELU'(aux[m][n]).
template <typename TB, int EPI>
__global__ void __launch_bounds__(256)
    k_gemm(const float *__restrict__ A, int64_t sam, int64_t sak, const TB *__restrict__ B,
           int64_t sbk, int64_t sbn, int M, int N, int K, int k_slice, float *__restrict__ C,
           int64_t ldc, const float *__restrict__ bias, const float *__restrict__ aux,
           float *__restrict__ C2) {
  __shared__ float As[16][64 + 4];
  __shared__ float Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * k_slice, ke = min(K, kb + k_slice);
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const bool a_k_fast = sak == 1, b_n_fast = sbn == 1;
  for (int k0 = kb; k0 < ke; k0 += 16) {
    float ra[4], rb[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int am = a_k_fast ? e >> 4 : e & 63, ak = a_k_fast ? e & 15 : e >> 6;
      const int gm = m0 + am, gk = k0 + ak;
      ra[u] = (gm < M && gk < ke) ? A[(int64_t)gm * sam + (int64_t)gk * sak] : 0.f;
      const int bn = b_n_fast ? e & 63 : e >> 4, bk = b_n_fast ? e >> 6 : e & 15;
      const int gn = n0 + bn, gk2 = k0 + bk;
      rb[u] = (gn < N && gk2 < ke) ? load_b<TB>(B + (int64_t)gk2 * sbk + (int64_t)gn * sbn) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      const int am = a_k_fast ? e >> 4 : e & 63, ak = a_k_fast ? e & 15 : e >> 6;
      As[ak][am] = ra[u];
      const int bn = b_n_fast ? e & 63 : e >> 4, bk = b_n_fast ? e >> 6 : e & 15;
      Bs[bk][bn] = rb[u];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; kk += 4) {
      float a[2], b[2];
      for (int i = 0; i < 2; ++i) a[i] = As[kk + (lane >> 4)][wm + i * 16 + (lane & 15)];
      for (int j = 0; j < 2; ++j) b[j] = Bs[kk + (lane >> 4)][wn + j * 16 + (lane & 15)];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  float *Cz = C + (int64_t)blockIdx.z * M * ldc;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const float v = acc[i][j][r];
        const int64_t o = (int64_t)m * ldc + n;
        if (EPI == EPI_STORE) {
          Cz[o] = v;
        } else if (EPI == EPI_BIAS_GELU) {
          const float z = v + bias[n];
          C[o] = z;
          C2[o] = gelu(z);
        } else {
          C[o] = v * gelu_grad(aux[o]);
        }
      }
}

// out[i] = sum over s of part[s][i] (s ascending), i < n.
__global__ void k_sum_slices(const float *__restrict__ part, int S, int64_t n,
                             float *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int s = 0; s < S; ++s) acc += part[(int64_t)s * n + i];
  out[i] = acc;
}

// Column sums of X[n][256] over row blocks of 256: part[blk][j].
__global__ void __launch_bounds__(256)
    k_colsum(const float *__restrict__ X, int64_t n, float *__restrict__ part) {
  const int j = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 256, r1 = min(n, r0 + 256);
  float acc = 0.f;
  for (int64_t r = r0; r < r1; ++r) acc += X[r * kHid + j];
  part[(int64_t)blockIdx.x * kHid + j] = acc;
}

__device__ inline float wave_sum(float v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// logit[b] = w3 . h2[b] + b3, one wave per sample.
__global__ void __launch_bounds__(256)
    k_head_fwd(const float *__restrict__ h2, int64_t n, const uint16_t *__restrict__ w3,
               const float *__restrict__ b3, float *__restrict__ logit) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= n) return;
  float acc = 0.f;
  for (int u = 0; u < 4; ++u) {
    const int j = lane + 64 * u;
    acc = fmaf(bf16_to_f32(w3[j]), h2[b * kHid + j], acc);
  }
  acc = wave_sum(acc);
  if (lane == 0) logit[b] = acc + b3[0];
}

// Loss gradient at the head.  A block takes 64 samples (16 per wave, one
// at a time): dlogit = (wp y (sigmoid - 1) + (1 - y) sigmoid) / n and
// dz2[b][j] = dlogit w3[j] GELU'(z2[b][j]).  Per block: partial sums of
// dlogit * h2[b][j] (-> dw3), of dlogit (-> db3) and of the loss (float64).
constexpr int kHeadRows = 64;

__global__ void __launch_bounds__(256)
    k_head_bwd(const float *__restrict__ z2, const float *__restrict__ h2,
               const float *__restrict__ logit, const uint8_t *__restrict__ y, int64_t n,
               float pos_weight, const uint16_t *__restrict__ w3, float *__restrict__ dz2,
               float *__restrict__ part_w3, double *__restrict__ part_loss) {
  __shared__ float dl_s[kHeadRows];
  __shared__ double loss_s[kHeadRows];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t b0 = (int64_t)blockIdx.x * kHeadRows;
  const float inv_n = 1.0f / (float)n;
  float w3v[4];
  for (int u = 0; u < 4; ++u) w3v[u] = bf16_to_f32(w3[lane + 64 * u]);
  for (int i = 0; i < kHeadRows / 4; ++i) {
    const int r = wv * (kHeadRows / 4) + i;
    const int64_t b = b0 + r;
    float dl = 0.f;
    double ls = 0.0;
    if (b < n) {
      const float x = logit[b];
      const float yy = y[b] ? 1.0f : 0.0f;
      const float sg = 1.0f / (1.0f + expf(-x));
      dl = (pos_weight * yy * (sg - 1.0f) + (1.0f - yy) * sg) * inv_n;
      // softplus(-x) for positives, softplus(x) for negatives
      const double xd = x;
      const double sp_pos = xd > 0 ? log1p(exp(-xd)) : -xd + log1p(exp(xd));
      const double sp_neg = xd > 0 ? xd + log1p(exp(-xd)) : log1p(exp(xd));
      ls = yy > 0 ? (double)pos_weight * sp_pos : sp_neg;
      for (int u = 0; u < 4; ++u) {
        const int j = lane + 64 * u;
        dz2[b * kHid + j] = dl * w3v[u] * gelu_grad(z2[b * kHid + j]);
      }
    }
    if (lane == 0) {
      dl_s[r] = dl;
      loss_s[r] = ls;
    }
  }
  __syncthreads();
  // dw3 partial: thread j sums dlogit * h2[b][j] over the block's samples
  const int j = threadIdx.x;
  float acc = 0.f;
  for (int r = 0; r < kHeadRows; ++r) {
    const int64_t b = b0 + r;
    if (b < n) acc = fmaf(dl_s[r], h2[b * kHid + j], acc);
  }
  part_w3[(int64_t)blockIdx.x * (kHid + 1) + j] = acc;
  if (threadIdx.x == 0) {
    float sd = 0.f;
    double sl = 0.0;
    for (int r = 0; r < kHeadRows; ++r) {
      sd += dl_s[r];
      sl += loss_s[r];
    }
    part_w3[(int64_t)blockIdx.x * (kHid + 1) + kHid] = sd;
    part_loss[blockIdx.x] = sl;
  }
}

// Fixed-order sum of float64 partials; out = sum / n.
__global__ void __launch_bounds__(256)
    k_loss_final(const double *__restrict__ part, int64_t np, int64_t n, double *__restrict__ out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0] / (double)n;
}

// Adam on the float32 master vector, arithmetic in float64, then the
// bfloat16 copy of the weights.
__global__ void k_mlp_adam(float *__restrict__ theta, uint16_t *__restrict__ wb,
                           float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, double lr, double b1, double b2,
                           double bc1, double bc2, double eps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kParams) return;
  const double gi = g[i];
  const double mi = b1 * (double)m[i] + (1.0 - b1) * gi;
  const double vi = b2 * (double)v[i] + (1.0 - b2) * gi * gi;
  const double th = (double)theta[i] - lr * (mi / bc1) / (sqrt(vi / bc2) + eps);
  m[i] = (float)mi;
  v[i] = (float)vi;
  const float t32 = (float)th;
  theta[i] = t32;
  int o = -1;
  if (i < kOffB1) o = kBfW1 + i;
  else if (i >= kOffW2 && i < kOffB2) o = kBfW2 + (i - kOffW2);
  else if (i >= kOffW3 && i < kOffB3) o = kBfW3 + (i - kOffW3);
  if (o >= 0) wb[o] = f32_to_bf16(t32);
}

// wb = theta's weights rounded to bfloat16.
__global__ void k_mlp_round(const float *__restrict__ theta, uint16_t *__restrict__ wb) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= kBfTotal) return;
  int i;
  if (o < kBfW2) i = kOffW1 + o;
  else if (o < kBfW3) i = kOffW2 + (o - kBfW2);
  else i = kOffW3 + (o - kBfW3);
  wb[o] = f32_to_bf16(theta[i]);
}

// Ids of the candidates whose logit >= thr, in candidate order (one block).
__global__ void __launch_bounds__(1024)
    k_pick(const float *__restrict__ logit, const uint64_t *__restrict__ ids, int n, float thr,
           uint64_t *__restrict__ out, int32_t *__restrict__ count) {
  __shared__ int wave_sum_s[16];
  __shared__ int base_s;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) base_s = 0;
  __syncthreads();
  for (int r = 0; r < n; r += 1024) {
    const int i = r + threadIdx.x;
    const bool keep = i < n && logit[i] >= thr && ids[i] != ~uint64_t(0);
    const uint64_t bal = __ballot(keep);
    const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(bal >> 32),
                                              __builtin_amdgcn_mbcnt_lo((unsigned)bal, 0));
    if (lane == 0) wave_sum_s[wv] = __popcll(bal);
    __syncthreads();
    int off = base_s;
    for (int w = 0; w < wv; ++w) off += wave_sum_s[w];
    if (keep) out[off + pre] = ids[i];
    __syncthreads();
    if (threadIdx.x == 0) {
      int t = 0;
      for (int w = 0; w < 16; ++w) t += wave_sum_s[w];
      base_s += t;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = base_s;
}

unsigned blocks_of(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

// Cameras (and optional frame list) to the device through pinned staging;
// the previous upload's copy must be complete before the staging is reused.
const Cam *upload_cams(dcgs_ctx *ctx, const dcgs_camera *cams, int n, const int32_t *frames,
                       int nf, const int32_t **frames_dev, hipStream_t st) {
  auto &P = ctx->pf;
  const size_t cbytes = (size_t)n * sizeof(Cam), fbytes = (size_t)nf * sizeof(int32_t);
  const size_t bytes = cbytes + fbytes + 16;
  if (P.staged) DCGS_HIP(hipEventSynchronize(P.staged));
  if (bytes > P.pinned_cap) {
    if (P.pinned) DCGS_HIP(hipHostFree(P.pinned));
    P.pinned = nullptr;
    P.pinned_cap = 0;
    DCGS_HIP(hipHostMalloc(&P.pinned, bytes, hipHostMallocDefault));
    P.pinned_cap = bytes;
  }
  if (!P.staged) DCGS_HIP(hipEventCreateWithFlags(&P.staged, hipEventDisableTiming));
  Cam *hc = (Cam *)P.pinned;
  for (int k = 0; k < n; ++k) hc[k] = to_cam(cams[k]);
  int32_t *hf = (int32_t *)((char *)P.pinned + cbytes);
  for (int k = 0; k < nf; ++k) hf[k] = frames[k];
  uint8_t *d = P.cams.need(bytes);
  DCGS_HIP(hipMemcpyAsync(d, P.pinned, cbytes + fbytes, hipMemcpyHostToDevice, st));
  DCGS_HIP(hipEventRecord(P.staged, st));
  if (frames_dev) *frames_dev = (const int32_t *)(d + cbytes);
  return (const Cam *)d;
}

}  // namespace

void prefetch_labels(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames, int horizon,
                     double s, uint8_t *labels, hipStream_t st) {
  DCGS_CHECK(cams && labels && n_frames > 0 && horizon >= 1 && horizon <= kMaxViews && s > 0,
             DCGS_E_INVALID, "prefetch_labels: bad args");
  const Cam *dc = upload_cams(ctx, cams, n_frames, nullptr, 0, nullptr, st);
  for (int t0 = 0; t0 < n_frames; t0 += 32768) {
    const int nt = std::min(32768, n_frames - t0);
    hipLaunchKernelGGL(k_labels, dim3(kCand / 256, nt), dim3(256), 0, st, dc, n_frames, t0,
                       horizon, s, labels);
    DCGS_LAUNCH_CHECK();
  }
}

void prefetch_features(dcgs_ctx *ctx, const dcgs_camera *cams, int n_frames,
                       const int32_t *frames, int n_sel, double s, double pos_unit,
                       const uint8_t *labels, float *X, uint64_t *ids, uint8_t *y,
                       hipStream_t st) {
  DCGS_CHECK(cams && frames && X && n_frames > 0 && n_sel > 0 && n_sel <= 65535 && s > 0 &&
                 pos_unit > 0 && (!y || labels),
             DCGS_E_INVALID, "prefetch_features: bad args");
  for (int k = 0; k < n_sel; ++k)
    DCGS_CHECK(frames[k] >= 0 && frames[k] < n_frames, DCGS_E_INVALID,
               "prefetch_features: frame index out of range");
  const int32_t *fd = nullptr;
  const Cam *dc = upload_cams(ctx, cams, n_frames, frames, n_sel, &fd, st);
  hipLaunchKernelGGL(k_features, dim3(kCand / 256, n_sel), dim3(256), 0, st, dc, fd, s, pos_unit,
                     labels, X, ids, y);
  DCGS_LAUNCH_CHECK();
}

void mlp_forward(dcgs_ctx *, const float *theta, const uint16_t *wb, const float *X, int64_t n,
                 float *z1, float *h1, float *z2, float *h2, float *logit, hipStream_t st) {
  DCGS_CHECK(theta && wb && X && z1 && h1 && z2 && h2 && logit && n >= 0, DCGS_E_INVALID,
             "mlp_forward: bad args");
  if (n == 0) return;
  DCGS_CHECK(n <= (int64_t)65535 * 64, DCGS_E_INVALID, "mlp_forward: batch too large");
  const dim3 g(kHid / 64, blocks_of(n, 64), 1);
  hipLaunchKernelGGL((k_gemm<uint16_t, EPI_BIAS_GELU>), g, dim3(256), 0, st, X, (int64_t)kIn,
                     (int64_t)1, wb + kBfW1, (int64_t)1, (int64_t)kIn, (int)n, kHid, kIn, kIn,
                     z1, (int64_t)kHid, theta + kOffB1, nullptr, h1);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL((k_gemm<uint16_t, EPI_BIAS_GELU>), g, dim3(256), 0, st, h1, (int64_t)kHid,
                     (int64_t)1, wb + kBfW2, (int64_t)1, (int64_t)kHid, (int)n, kHid, kHid, kHid,
                     z2, (int64_t)kHid, theta + kOffB2, nullptr, h2);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_head_fwd, dim3(blocks_of(n, 4)), dim3(256), 0, st, h2, n, wb + kBfW3,
                     theta + kOffB3, logit);
  DCGS_LAUNCH_CHECK();
}

void mlp_backward(dcgs_ctx *ctx, const float *theta, const uint16_t *wb, const float *X,
                  const float *z1, const float *h1, const float *z2, const float *h2,
                  const float *logit, const uint8_t *y, int64_t n, float pos_weight,
                  float *grad, double *loss, hipStream_t st) {
  DCGS_CHECK(theta && wb && X && z1 && h1 && z2 && h2 && logit && y && grad && n > 0 &&
                 pos_weight > 0,
             DCGS_E_INVALID, "mlp_backward: bad args");
  DCGS_CHECK(n <= (int64_t)65535 * 64, DCGS_E_INVALID, "mlp_backward: batch too large");
  auto &P = ctx->pf;
  float *dz2 = P.dz2.need((size_t)n * kHid), *dz1 = P.dz1.need((size_t)n * kHid);
  const int64_t nb4 = blocks_of(n, kHeadRows);
  float *pw3 = P.part.need((size_t)nb4 * (kHid + 1));
  double *pl = P.part_loss.need((size_t)nb4 + 1);
  hipLaunchKernelGGL(k_head_bwd, dim3((unsigned)nb4), dim3(256), 0, st, z2, h2, logit, y, n,
                     pos_weight, wb + kBfW3, dz2, pw3, pl);
  DCGS_LAUNCH_CHECK();
  // dw3 and db3: the block partials summed in block order (w3 and b3 are
  // adjacent in the master vector)
  hipLaunchKernelGGL(k_sum_slices, dim3(blocks_of(kHid + 1, 256)), dim3(256), 0, st, pw3,
                     (int)nb4, (int64_t)(kHid + 1), grad + kOffW3);
  DCGS_LAUNCH_CHECK();
  if (loss) {
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, st, pl, nb4, n, loss);
    DCGS_LAUNCH_CHECK();
  }
  // split-K weight gradients: S slices of the batch, summed in slice order
  const int S = (int)std::min<int64_t>(64, std::max<int64_t>(1, n / 1024));
  const int ks = (int)((n + S - 1) / S);
  const int ks16 = (ks + 15) / 16 * 16;
  float *pw = P.split.need((size_t)S * kHid * kHid);
  // dW2[j][i] = sum_b dz2[b][j] h1[b][i]
  hipLaunchKernelGGL((k_gemm<float, EPI_STORE>), dim3(kHid / 64, kHid / 64, S), dim3(256), 0, st,
                     dz2, (int64_t)1, (int64_t)kHid, h1, (int64_t)kHid, (int64_t)1, kHid, kHid,
                     (int)n, ks16, pw, (int64_t)kHid, nullptr, nullptr, nullptr);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_slices, dim3(blocks_of(kHid * kHid, 256)), dim3(256), 0, st, pw, S,
                     (int64_t)kHid * kHid, grad + kOffW2);
  DCGS_LAUNCH_CHECK();
  // db2
  const int64_t nb256 = blocks_of(n, 256);
  float *pc = P.colpart.need((size_t)nb256 * kHid);
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)nb256), dim3(256), 0, st, dz2, n, pc);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_slices, dim3(1), dim3(256), 0, st, pc, (int)nb256, (int64_t)kHid,
                     grad + kOffB2);
  DCGS_LAUNCH_CHECK();
  // dz1 = (dz2 W2) * GELU'(z1)
  hipLaunchKernelGGL((k_gemm<uint16_t, EPI_GELU_GRAD>), dim3(kHid / 64, blocks_of(n, 64), 1),
                     dim3(256), 0, st, dz2, (int64_t)kHid, (int64_t)1, wb + kBfW2,
                     (int64_t)kHid, (int64_t)1, (int)n, kHid, kHid, kHid, dz1, (int64_t)kHid,
                     nullptr, z1, nullptr);
  DCGS_LAUNCH_CHECK();
  // dW1[j][i] = sum_b dz1[b][j] x[b][i]
  hipLaunchKernelGGL((k_gemm<float, EPI_STORE>), dim3(1, kHid / 64, S), dim3(256), 0, st, dz1,
                     (int64_t)1, (int64_t)kHid, X, (int64_t)kIn, (int64_t)1, kHid, kIn, (int)n,
                     ks16, pw, (int64_t)kIn, nullptr, nullptr, nullptr);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_slices, dim3(blocks_of(kHid * kIn, 256)), dim3(256), 0, st, pw, S,
                     (int64_t)kHid * kIn, grad + kOffW1);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)nb256), dim3(256), 0, st, dz1, n, pc);
  DCGS_LAUNCH_CHECK();
  hipLaunchKernelGGL(k_sum_slices, dim3(1), dim3(256), 0, st, pc, (int)nb256, (int64_t)kHid,
                     grad + kOffB1);
  DCGS_LAUNCH_CHECK();
}

void mlp_adam(dcgs_ctx *, float *theta, uint16_t *wb, float *m, float *v, const float *grad,
              int64_t step, double lr, double beta1, double beta2, double eps, hipStream_t st) {
  DCGS_CHECK(theta && wb && m && v && grad && step >= 1 && lr > 0 && beta1 >= 0 && beta1 < 1 &&
                 beta2 >= 0 && beta2 < 1 && eps > 0,
             DCGS_E_INVALID, "mlp_adam: bad args");
  const double bc1 = 1.0 - std::pow(beta1, (double)step), bc2 = 1.0 - std::pow(beta2, (double)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3(blocks_of(kParams, 256)), dim3(256), 0, st, theta, wb, m,
                     v, grad, lr, beta1, beta2, bc1, bc2, eps);
  DCGS_LAUNCH_CHECK();
}

void mlp_round(dcgs_ctx *, const float *theta, uint16_t *wb, hipStream_t st) {
  DCGS_CHECK(theta && wb, DCGS_E_INVALID, "mlp_round: bad args");
  hipLaunchKernelGGL(k_mlp_round, dim3(blocks_of(kBfTotal, 256)), dim3(256), 0, st, theta, wb);
  DCGS_LAUNCH_CHECK();
}

void prefetch_predict(dcgs_ctx *ctx, const float *theta, const uint16_t *wb,
                      const dcgs_camera *hist, double s, double pos_unit, float threshold,
                      uint64_t *out_ids, int32_t *out_count, float *out_logit,
                      hipStream_t st) {
  DCGS_CHECK(theta && wb && hist && out_ids && out_count && s > 0 && pos_unit > 0,
             DCGS_E_INVALID, "prefetch_predict: bad args");
  auto &P = ctx->pf;
  // history order: entry k is frame t-k; as a trajectory the current frame is last
  dcgs_camera traj[kHist];
  for (int k = 0; k < kHist; ++k) traj[kHist - 1 - k] = hist[k];
  const int32_t frame = kHist - 1;
  float *X = P.X.need((size_t)kCand * kIn);
  uint64_t *ids = P.ids.need(kCand);
  float *act = P.act.need((size_t)4 * kCand * kHid + kCand);
  prefetch_features(ctx, traj, kHist, &frame, 1, s, pos_unit, nullptr, X, ids, nullptr, st);
  float *lg = out_logit ? out_logit : act + (size_t)4 * kCand * kHid;
  mlp_forward(ctx, theta, wb, X, kCand, act, act + (size_t)kCand * kHid,
              act + (size_t)2 * kCand * kHid, act + (size_t)3 * kCand * kHid, lg, st);
  hipLaunchKernelGGL(k_pick, dim3(1), dim3(1024), 0, st, lg, ids, kCand, threshold, out_ids,
                     out_count);
  DCGS_LAUNCH_CHECK();
}

}  // namespace dcgs
