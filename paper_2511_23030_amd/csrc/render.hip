// Differentiable Gaussian rasterization for gfx950: projection (float64
// geometry), depth order, (tile, Gaussian) pair emission, stable tile sort,
// per-tile ranges, front-to-back compositing, and its adjoint.
//
// The paper's optimisation step renders RGB and depth of the visible
// Gaussians for a keyframe and differentiates the losses of Eqs. (2)-(4)
// (Sec. III-C, Sec. III-E).  The rendering model is stated in dcgs.h.
//
// Layout decisions (gfx950):
//  * Parameters are SoA rows, so every per-Gaussian kernel reads coalesced.
//  * Geometry (covariance, EWA, conic, pixel box, depth) is computed in
//    float64: every integer decision (culling, pixel box, tile rect, the
//    float32 depth key) then agrees with a float64 reference except within
//    ~1e-15 of a boundary.  The cost is hidden under the 236-byte parameter
//    read per Gaussian.
//  * A projection record is four float4 (64 B, one aligned segment): u and
//    v relative to the pixel box corner (small magnitudes keep float32
//    offsets exact to ~1e-7 px), conic, opacity, colour, depth and the
//    packed pixel box, then where the record's gradient slots start and its
//    kept-tile mask (read by the backward with the record); the projection
//    writes all 64 bytes at once.
//  * The depth digits of the (tile, depth) keys are the same for all pairs of
//    a Gaussian, so the LSD passes over them run on the N Gaussians before
//    pair expansion; pairs are then emitted in depth order and stably sorted
//    on the tile digits only.  The result is the order of a full LSD radix
//    sort of the 64-bit (tile, float32 depth bits) keys, ties by index.
//  * Rasterization: one workgroup per tile, one pixel per lane, records
//    staged in LDS in batches, workgroups mapped to XCDs in contiguous bands
//    of tiles so neighbouring tiles share an L2.
//  * Backward: each tile walks its list back to front from the deepest
//    composited position, recovers T_k = T_{k+1}/(1-alpha_k), reduces each
//    Gaussian's ten screen-space gradient terms across the tile (wavefront
//    butterfly, then a fixed-order sum over waves) and writes them to a
//    per-pair slot.  A per-Gaussian pass sums its slots in a fixed order:
//    gradients are bit-reproducible and use no float atomics.
#include <algorithm>

#include "internal.h"

namespace dcgs {
namespace {

constexpr float kAlphaMin = 1.0f / 255.0f;
constexpr float kAlphaMax = 0.99f;
constexpr float kTMin = 1e-4f;
constexpr double kDilation = 0.3;
// Records store the conic Q (Q00, Q01, Q11) as log2(e) (-Q00/2, -Q01,
// -Q11/2); kQ converts a stored diagonal entry back (x -2/log2(e)).
constexpr double kLog2e = 1.4426950408889634;
constexpr float kQ = (float)(-2.0 / kLog2e);
constexpr uint32_t kCulledKey = 0xFFFFFFFFu;

struct CamD {
  double R[9], t[3], fx, fy, cx, cy, zn, zf, C[3], limx, limy;
  int W, H;
};

CamD make_cam(const dcgs_camera &c) {
  CamD d{};
  for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
  d.fx = c.fx;
  d.fy = c.fy;
  d.cx = c.cx;
  d.cy = c.cy;
  d.zn = c.z_near;
  d.zf = c.z_far;
  d.W = c.width;
  d.H = c.height;
  for (int i = 0; i < 3; ++i)  // camera centre C = -R^T t
    d.C[i] = -(c.R[i] * c.t[0] + c.R[3 + i] * c.t[1] + c.R[6 + i] * c.t[2]);
  d.limx = ((1.3 * 0.5) * c.width) / c.fx;
  d.limy = ((1.3 * 0.5) * c.height) / c.fy;
  return d;
}

// Real orthonormal SH basis (no Condon-Shortley phase), k = l*l + l + m.
template <typename T>
__device__ inline void sh_eval(int deg, T x, T y, T z, T *Y) {
  constexpr double kPi = 3.14159265358979323846;
  Y[0] = T(0.5 / sqrt(kPi));
  if (deg < 1) return;
  const T c1 = T(sqrt(3.0 / (4.0 * kPi)));
  Y[1] = c1 * y;
  Y[2] = c1 * z;
  Y[3] = c1 * x;
  if (deg < 2) return;
  const T c2a = T(0.5 * sqrt(15.0 / kPi)), c20 = T(0.25 * sqrt(5.0 / kPi)),
          c22 = T(0.25 * sqrt(15.0 / kPi));
  Y[4] = c2a * x * y;
  Y[5] = c2a * y * z;
  Y[6] = c20 * (3.0 * z * z - 1.0);
  Y[7] = c2a * x * z;
  Y[8] = c22 * (x * x - y * y);
  if (deg < 3) return;
  const T c33 = T(0.25 * sqrt(35.0 / (2.0 * kPi))), c32 = T(0.5 * sqrt(105.0 / kPi)),
          c31 = T(0.25 * sqrt(21.0 / (2.0 * kPi))), c30 = T(0.25 * sqrt(7.0 / kPi)),
          c32b = T(0.25 * sqrt(105.0 / kPi));
  Y[9] = c33 * y * (3.0 * x * x - y * y);
  Y[10] = c32 * x * y * z;
  Y[11] = c31 * y * (5.0 * z * z - 1.0);
  Y[12] = c30 * z * (5.0 * z * z - 3.0);
  Y[13] = c31 * x * (5.0 * z * z - 1.0);
  Y[14] = c32b * z * (x * x - y * y);
  Y[15] = c33 * x * (x * x - 3.0 * y * y);
}

// gd = sum_k f[k] grad Y_k(x, y, z), with (x, y, z) treated as independent
// (the caller projects onto the sphere's tangent plane); k >= 1.
template <typename T>
__device__ inline void sh_grad_dot(int deg, T x, T y, T z, const T *f, T gd[3]) {
  constexpr double kPi = 3.14159265358979323846;
  gd[0] = gd[1] = gd[2] = T(0);
  if (deg < 1) return;
  const T c1 = T(sqrt(3.0 / (4.0 * kPi)));
  gd[0] += c1 * f[3];
  gd[1] += c1 * f[1];
  gd[2] += c1 * f[2];
  if (deg < 2) return;
  const T c2a = T(0.5 * sqrt(15.0 / kPi)), c20 = T(0.25 * sqrt(5.0 / kPi)),
          c22 = T(0.25 * sqrt(15.0 / kPi));
  gd[0] += c2a * y * f[4] + c2a * z * f[7] + 2.0 * c22 * x * f[8];
  gd[1] += c2a * x * f[4] + c2a * z * f[5] - 2.0 * c22 * y * f[8];
  gd[2] += c2a * y * f[5] + 6.0 * c20 * z * f[6] + c2a * x * f[7];
  if (deg < 3) return;
  const T c33 = T(0.25 * sqrt(35.0 / (2.0 * kPi))), c32 = T(0.5 * sqrt(105.0 / kPi)),
          c31 = T(0.25 * sqrt(21.0 / (2.0 * kPi))), c30 = T(0.25 * sqrt(7.0 / kPi)),
          c32b = T(0.25 * sqrt(105.0 / kPi));
  gd[0] += 6.0 * c33 * x * y * f[9] + c32 * y * z * f[10] + c31 * (5.0 * z * z - 1.0) * f[13] +
           2.0 * c32b * x * z * f[14] + c33 * (3.0 * x * x - 3.0 * y * y) * f[15];
  gd[1] += c33 * (3.0 * x * x - 3.0 * y * y) * f[9] + c32 * x * z * f[10] +
           c31 * (5.0 * z * z - 1.0) * f[11] - 2.0 * c32b * y * z * f[14] - 6.0 * c33 * x * y * f[15];
  gd[2] += c32 * x * y * f[10] + 10.0 * c31 * y * z * f[11] + c30 * (15.0 * z * z - 3.0) * f[12] +
           10.0 * c31 * x * z * f[13] + c32b * (x * x - y * y) * f[14];
}

// Geometry of one Gaussian.  The forward projection runs in float64 (T =
// double) so every integer decision matches a float64 reference; the
// backward chain rule runs in float32 (T = float), which halves its
// registers.
template <typename T>
struct GeoT {
  T mu[3], s[3], qn[4], qnorm, o, Rg[9], M[9], Sig[6];
  T X, Y, Z, A0[3], A1[3], a, b, c, det;
  T u, v, r2;  // r2 = 2 ln(255 o): alpha >= 1/255 where d^T Q d <= r2
  bool culled;
  int i0, i1, j0, j1;
};
using Geo = GeoT<double>;

// a / b: IEEE division in float64 (the forward geometry, whose keys and
// boxes must match a float64 reference bit for bit); in float32 (the
// backward chain) the hardware reciprocal (about 1 ulp) times a.
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// Camera-independent part: activations, rotation, covariance.
template <typename T>
__device__ inline void load_gauss(const float *__restrict__ P, int64_t stride, int64_t i,
                                  GeoT<T> &g) {
  for (int k = 0; k < 3; ++k) g.mu[k] = (T)P[k * stride + i];
  for (int k = 0; k < 3; ++k) g.s[k] = exp((T)P[(3 + k) * stride + i]);
  T q[4];
  for (int k = 0; k < 4; ++k) q[k] = (T)P[(6 + k) * stride + i];
  g.o = qdiv(T(1), T(1) + exp(-(T)P[10 * stride + i]));
  g.qnorm = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int k = 0; k < 4; ++k) g.qn[k] = qdiv(q[k], g.qnorm);
  const T w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
  T *R = g.Rg;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) g.M[3 * r + c] = R[3 * r + c] * g.s[c];
  // Sigma = M M^T: xx, xy, xz, yy, yz, zz
  const T *M = g.M;
  g.Sig[0] = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  g.Sig[1] = M[0] * M[3] + M[1] * M[4] + M[2] * M[5];
  g.Sig[2] = M[0] * M[6] + M[1] * M[7] + M[2] * M[8];
  g.Sig[3] = M[3] * M[3] + M[4] * M[4] + M[5] * M[5];
  g.Sig[4] = M[3] * M[6] + M[4] * M[7] + M[5] * M[8];
  g.Sig[5] = M[6] * M[6] + M[7] * M[7] + M[8] * M[8];
}

// Camera-dependent part: camera coordinates, culling, EWA, conic, pixel box.
// With cull false (the backward of a record the forward drew) the culling
// tests and the box are skipped: the float32 chain must not take its own
// decisions near the float64 forward's thresholds.
template <typename T>
__device__ inline void project(const CamD &cam, GeoT<T> &g, bool cull = true) {
  T Rc[9];
  for (int k = 0; k < 9; ++k) Rc[k] = (T)cam.R[k];
  g.X = Rc[0] * g.mu[0] + Rc[1] * g.mu[1] + Rc[2] * g.mu[2] + (T)cam.t[0];
  g.Y = Rc[3] * g.mu[0] + Rc[4] * g.mu[1] + Rc[5] * g.mu[2] + (T)cam.t[1];
  g.Z = Rc[6] * g.mu[0] + Rc[7] * g.mu[1] + Rc[8] * g.mu[2] + (T)cam.t[2];
  g.culled = false;
  if (cull) {
    g.culled = !(g.Z > (T)cam.zn);
    if (!g.culled) {
      const T rx = fabs(qdiv(g.X, g.Z)), ry = fabs(qdiv(g.Y, g.Z));
      g.culled = (rx > (T)cam.limx) || (ry > (T)cam.limy) || (g.o < T(1.0 / 255.0));
    }
    if (g.culled) return;
  }
  const T fx = (T)cam.fx, fy = (T)cam.fy;
  const T iz = qdiv(T(1), g.Z);
  const T j00 = fx * iz, j02 = -fx * g.X * iz * iz;
  const T j11 = fy * iz, j12 = -fy * g.Y * iz * iz;
  for (int c = 0; c < 3; ++c) {
    g.A0[c] = j00 * Rc[c] + j02 * Rc[6 + c];
    g.A1[c] = j11 * Rc[3 + c] + j12 * Rc[6 + c];
  }
  const T *S = g.Sig;
  auto quad = [&](const T *p, const T *q) {
    const T sx = S[0] * q[0] + S[1] * q[1] + S[2] * q[2];
    const T sy = S[1] * q[0] + S[3] * q[1] + S[4] * q[2];
    const T sz = S[2] * q[0] + S[4] * q[1] + S[5] * q[2];
    return p[0] * sx + p[1] * sy + p[2] * sz;
  };
  g.a = quad(g.A0, g.A0) + T(kDilation);
  g.b = quad(g.A0, g.A1);
  g.c = quad(g.A1, g.A1) + T(kDilation);
  g.det = g.a * g.c - g.b * g.b;
  if (cull && !(g.det > T(0))) {
    g.culled = true;
    return;
  }
  g.u = qdiv(fx * g.X, g.Z) + (T)cam.cx;
  g.v = qdiv(fy * g.Y, g.Z) + (T)cam.cy;
  if (!cull) return;
  g.r2 = T(2) * log(T(255) * g.o);
  const T r2 = g.r2;
  const T ex = sqrt(r2 * g.a), ey = sqrt(r2 * g.c);
  const T big = T(1e9);
  const T e0 = fmin(fmax(g.u - ex - T(0.5), -big), big), e1 = fmin(fmax(g.u + ex - T(0.5), -big), big);
  const T f0 = fmin(fmax(g.v - ey - T(0.5), -big), big), f1 = fmin(fmax(g.v + ey - T(0.5), -big), big);
  g.i0 = (int)fmax(ceil(e0), T(0));
  g.i1 = (int)fmin(floor(e1), (T)(cam.W - 1));
  g.j0 = (int)fmax(ceil(f0), T(0));
  g.j1 = (int)fmin(floor(f1), (T)(cam.H - 1));
  if (g.i0 > g.i1 || g.j0 > g.j1) g.culled = true;
}

template <typename T>
__device__ inline void load_geo(const float *__restrict__ P, int64_t stride, int64_t i,
                                const CamD &cam, GeoT<T> &g) {
  load_gauss(P, stride, i, g);
  project(cam, g);
}

// Colour before the clamp (raw) for each channel.
template <typename T>
__device__ inline void color_raw(const float *__restrict__ coef, int64_t cstride,
                                 int deg, const GeoT<T> &g, const CamD &cam, T *dir, T &dnorm,
                                 T *Y, T raw[3]) {
  T d0 = g.mu[0] - (T)cam.C[0], d1 = g.mu[1] - (T)cam.C[1], d2 = g.mu[2] - (T)cam.C[2];
  dnorm = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
  dir[0] = qdiv(d0, dnorm);
  dir[1] = qdiv(d1, dnorm);
  dir[2] = qdiv(d2, dnorm);
  sh_eval(deg, dir[0], dir[1], dir[2], Y);
  const int K = (deg + 1) * (deg + 1);
  for (int ch = 0; ch < 3; ++ch) {
    T acc = T(0);
    if constexpr (sizeof(T) == 4) {
      // float (the projection backward): unrolled by 4, not fully, so four
      // coefficient loads are in flight per step without hoisting all 48
      // into registers (which would cap the kernel's occupancy)
#pragma unroll 4
      for (int k = 0; k < K; ++k) acc += (T)coef[(3 * k + ch) * cstride] * Y[k];
    } else {
      // double (the forward projection, held to 128 registers): rolled;
      // its coefficients come from LDS
#pragma unroll 1
      for (int k = 0; k < K; ++k) acc += (T)coef[(3 * k + ch) * cstride] * Y[k];
    }
    raw[ch] = acc + T(0.5);
  }
}

// Tiles of a record's tile rectangle that can hold a pixel it composites.
// Bit k (row-major in the rectangle) is set when the rectangle of pixel
// centres that tile k shares with the pixel box meets the ellipse
// f(d) = d^T Q d <= tau' (Q the conic, d relative to (u, v)): alpha >= 1/255
// exactly where f <= tau = 2 ln(255 o), and tau' = (tau + 1e-3 (1 + tau)) /
// (1 - 16 u kappa), u = 2^-24, kappa = 2 (Q00 + Q11) / lambda_min(Q), covers
// the float32 evaluation of a sample, so a tile that is dropped holds no
// pixel the float32 compositing would take.  The minimum of the convex f
// over a rectangle not holding the centre lies on an edge, at the clamped
// minimiser of f along it.  Every tile is kept when the rectangle has more
// than 64 tiles or 16 u kappa >= 1/2.  n_keep gets the number kept.
__device__ inline uint64_t tile_mask(const Geo &g, int TW, int TH, uint32_t &n_keep) {
  const int tx0 = g.i0 / TW, tx1 = g.i1 / TW, ty0 = g.j0 / TH, ty1 = g.j1 / TH;
  const int w = tx1 - tx0 + 1, n_rect = w * (ty1 - ty0 + 1);
  const double half = 0.5 * (g.a - g.c);
  const double lmax = 0.5 * (g.a + g.c) + sqrt(half * half + g.b * g.b);  // of Sigma2
  const double kappa = 2.0 * (g.a + g.c) / g.det * lmax;
  const double shrink = 1.0 - 16.0 * 0x1p-24 * kappa;
  if (n_rect > 64 || !(shrink > 0.5)) {
    n_keep = (uint32_t)n_rect;
    return n_rect >= 64 ? ~uint64_t(0) : ((uint64_t(1) << n_rect) - 1);
  }
  const double tau = g.r2;
  const double lim = (tau + 1e-3 * (1.0 + tau)) / shrink;
  // Per row of tiles: the row's band of pixel-centre rows meets the ellipse
  // {f <= lim} in an x-interval [xl, xr], and a tile is kept when its
  // pixel-centre columns meet that interval.  The right end of the ellipse
  // across y is concave, the left end convex, so over the band they are
  // reached at the ellipse's rightmost / leftmost point clamped into it.
  const double idet = 1.0 / g.det;
  const double q00 = g.c * idet, q01 = -g.b * idet, q11 = g.a * idet;
  const double dq = idet;                        // det Q = 1 / det Sigma2
  const double ymax = sqrt(q00 * lim / dq);      // half height of the ellipse
  const double yr = -q01 * sqrt(lim / (q11 * dq));  // y of its rightmost point
  const double uh = g.u - 0.5, vh = g.v - 0.5;
  uint32_t lo = 0, hi = 0;
  int k = 0;
  for (int ty = ty0; ty <= ty1; ++ty, k += w) {
    const double y0 = max(ty * TH, g.j0) - vh, y1 = min(ty * TH + TH - 1, g.j1) - vh;
    if (y1 < -ymax || y0 > ymax) continue;
    const double ya = fmax(y0, -ymax), yb = fmin(y1, ymax);
    const double y_r = fmin(fmax(yr, ya), yb), y_l = fmin(fmax(-yr, ya), yb);
    const double xr = (-q01 * y_r + sqrt(fmax(q00 * lim - dq * y_r * y_r, 0.0))) / q00;
    const double xl = (-q01 * y_l - sqrt(fmax(q00 * lim - dq * y_l * y_l, 0.0))) / q00;
    for (int tx = tx0, kk = k; tx <= tx1; ++tx, ++kk) {
      const double x0 = max(tx * TW, g.i0) - uh, x1 = min(tx * TW + TW - 1, g.i1) - uh;
      if (x1 >= xl && x0 <= xr) {
        if (kk < 32) lo |= 1u << kk; else hi |= 1u << (kk - 32);
      }
    }
  }
  n_keep = (uint32_t)(__popc(lo) + __popc(hi));
  return ((uint64_t)hi << 32) | lo;
}

// Slot of tile k of a record's rectangle among its kept tiles.
__device__ __forceinline__ uint32_t kept_rank(uint64_t m, int n_rect, int k) {
  return n_rect > 64 ? (uint32_t)k : (uint32_t)__popcll(m & ((uint64_t(1) << k) - 1));
}

__device__ __forceinline__ bool tile_kept(uint64_t m, int n_rect, int k) {
  return n_rect > 64 || ((m >> k) & 1);
}

// Per-pair gradient slots: record r's kept tiles take slots base(r) ..
// base(r) + count[r] - 1 (row-major), in record order.  The projection's
// workgroups cover 64 consecutive Gaussians, so within one view a
// workgroup's records form a segment v * gridDim + block of consecutive
// records; base(r) = seg_off[segment] + the record's prefix inside its
// segment, seg_off the exclusive scan of the segment totals.  The record
// carries its prefix and segment id, so it is written whole here, and the
// pass that sums a record's slots finds neighbouring records' slots side by
// side.
__device__ __forceinline__ uint32_t slot_base(const uint32_t *__restrict__ seg_off,
                                              const float4 &D) {
  return seg_off[__float_as_uint(D.w)] + __float_as_uint(D.x);
}

// A drawn record's place in the depth order as one 64-bit key: the depth
// sort is stable on the float32 depth bits with records in index order, so
// record a precedes record b exactly when (depth bits, index) of a is
// smaller.  Depths are positive, so every key exceeds 0 (0: nothing).
__device__ __forceinline__ uint64_t depth_order_key(const float4 *__restrict__ rec, uint32_t r) {
  return ((uint64_t)__float_as_uint(rec[4 * (int64_t)r + 2].y) << 32) | r;
}

// One thread per Gaussian; it projects the Gaussian into every view whose
// bit is set in its chunk's view mask.  Record r = v * n + g is the float4s
// rec[4 r .. 4 r + 3] (64 contiguous bytes, one gather per record: geometry,
// colour, depth and box, then the slot prefix, kept-tile mask and segment
// id; a culled record is not written).  seg_tot[v * gridDim + block] = the
// pair count of the workgroup's records of view v.  cnt[0] = n (device
// counter; the grid may be sized for a capacity).
// Four waves per SIMD: the float64 projection is latency-bound, and the
// compiler fits it in 128 registers without spilling.
constexpr int kPrepThreads = 64;
__global__ void __launch_bounds__(kPrepThreads) __attribute__((amdgpu_waves_per_eu(4, 8)))
    k_preprocess(const float *__restrict__ P, const int64_t *__restrict__ cnt, int64_t stride,
                 int deg, const CamD *__restrict__ cams, int V,
                 const uint16_t *__restrict__ gmask, int mask_shift, int TW, int TH,
                 float4 *__restrict__ rec, int64_t RS, uint32_t *__restrict__ zkey,
                 uint32_t *__restrict__ sortkey, uint32_t *__restrict__ order,
                 uint32_t *__restrict__ count, uint64_t *__restrict__ tmask,
                 uint32_t *__restrict__ seg_tot) {
  static_assert(kPrepThreads == kWave, "one wavefront per segment");
  // the Gaussian's colour coefficients, read once for all views into this
  // thread's LDS column (each thread reads back only its own column)
  __shared__ float shc[48][kPrepThreads];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = cnt[0];
  // every lane takes part in the segment prefix sums, past n too (with no
  // pairs); a workgroup wholly past n only writes zero segment totals
  const bool live = i < n;
  Geo g;
  unsigned m = 0;
  if (live) {
    load_gauss(P, stride, i, g);
    for (int r = 0; r < 3 * (deg + 1) * (deg + 1); ++r)
      shc[r][threadIdx.x] = P[(11 + r) * stride + i];
    m = gmask ? ((unsigned)gmask[i] >> mask_shift) : 0xFFFFu;
  }
  const int lane = threadIdx.x;
  for (int v = 0; v < V; ++v) {
    const int64_t r = v * n + i;
    uint32_t n_keep = 0;
    uint64_t tm = 0;
    bool drawn = false;
    float zf = 0.0f;
    if (live) {
      order[r] = (uint32_t)r;
      bool culled = !((m >> v) & 1u);
      if (!culled) {
        project(cams[v], g);
        culled = g.culled;
        zf = (float)g.Z;
      }
      zkey[r] = __float_as_uint(zf);
      if (culled) {  // its record is never read: no pairs, and exports zero it
        count[r] = 0;
        tmask[r] = 0;
        sortkey[r] = kCulledKey;
      } else {
        drawn = true;
        tm = tile_mask(g, TW, TH, n_keep);
        tmask[r] = tm;
        count[r] = n_keep;
        sortkey[r] = __float_as_uint(zf);
      }
    }
    // the segment's inclusive prefix of pair counts (lane order = record order)
    uint32_t incl = n_keep;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t t = __shfl_up(incl, off);
      if (lane >= off) incl += t;
    }
    const uint32_t segment = (uint32_t)v * gridDim.x + blockIdx.x;
    if (lane == kWave - 1) seg_tot[segment] = incl;
    if (drawn) {
      double dir[3], dn, Y[16], raw[3];
      color_raw(&shc[0][threadIdx.x], kPrepThreads, deg, g, cams[v], dir, dn, Y, raw);
      const double id = 1.0 / g.det;
      rec[4 * r] = make_float4((float)(g.u - g.i0), (float)(g.v - g.j0),
                               (float)(-0.5 * kLog2e * g.c * id), (float)(kLog2e * g.b * id));
      rec[4 * r + 1] = make_float4((float)(-0.5 * kLog2e * g.a * id), (float)g.o,
                                   (float)fmax(raw[0], 0.0), (float)fmax(raw[1], 0.0));
      rec[4 * r + 2] = make_float4((float)fmax(raw[2], 0.0), zf,
                                   __uint_as_float((uint32_t)g.i0 | ((uint32_t)g.i1 << 16)),
                                   __uint_as_float((uint32_t)g.j0 | ((uint32_t)g.j1 << 16)));
      rec[4 * r + 3] = make_float4(__uint_as_float(incl - n_keep), __uint_as_float((uint32_t)tm),
                                   __uint_as_float((uint32_t)(tm >> 32)), __uint_as_float(segment));
    }
  }
}

// The records' pair counts in depth order (what the pair-offset scan sums,
// gathered once here instead of by it).
// Each workgroup also writes the 64-bit sum of its counts; k_pairs_total
// adds those up: the 32-bit scan of the counts wraps beyond 2^32 pairs, and
// the overflow decision must see the true count.
constexpr int kCountThreads = 256;
__global__ void __launch_bounds__(kCountThreads)
    k_depth_counts(const uint32_t *__restrict__ order, const uint32_t *__restrict__ count,
           const int64_t *__restrict__ cnt, uint32_t *__restrict__ count_sorted,
           unsigned long long *__restrict__ part_sum) {
  __shared__ unsigned long long part[kCountThreads / kWave];
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long c = 0;
  if (j < cnt[1]) {
    const uint32_t k = count[order[j]];
    count_sorted[j] = k;
    c = k;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int w = 0; w < kCountThreads / kWave; ++w) s += part[w];
    part_sum[blockIdx.x] = s;
  }
}

// One workgroup: cnt[5] = the 64-bit pair total (the sum of k_depth_counts'
// per-workgroup sums, in a fixed order); cnt[2] = pairs to process; cnt[3] =
// the total when it overflows (pairs_overflow: beyond the pair capacity or
// 2^31 - 1, or any earlier window of this state overflowed, cnt[4] sticky),
// else 0.  Every later kernel of the window does nothing when cnt[3] != 0.
constexpr int kTotalThreads = 1024;
__global__ void __launch_bounds__(kTotalThreads)
    k_pairs_total(const unsigned long long *__restrict__ part_sum, int64_t *__restrict__ cnt,
                  int64_t pcap) {
  __shared__ unsigned long long wsum[kTotalThreads / kWave];
  const int64_t nb = (cnt[1] + kCountThreads - 1) / kCountThreads;
  unsigned long long s = 0;
  for (int64_t b = threadIdx.x; b < nb; b += kTotalThreads) s += part_sum[b];
  for (int off = kWave / 2; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & (kWave - 1)) == 0) wsum[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x != 0) return;
  unsigned long long t = 0;
  for (int w = 0; w < kTotalThreads / kWave; ++w) t += wsum[w];
  const int64_t total = (int64_t)t;
  cnt[5] = total;
  const bool over = pairs_overflow(total, pcap, cnt[4]);
  cnt[2] = over ? 0 : total;
  cnt[3] = over ? (total > 0 ? total : 1) : 0;
  if (over) cnt[4] = 1;
}

// Position of the k-th set bit (k from 0) of m, which has more than k set
// bits: six halving steps.
__device__ __forceinline__ int nth_set_bit(uint64_t m, int k) {
  int pos = 0;
#pragma unroll
  for (int w = 32; w >= 1; w >>= 1) {
    const uint64_t low = m & ((uint64_t(1) << w) - 1);
    const int c = __popcll(low);
    if (k >= c) {
      k -= c;
      pos += w;
      m >>= w;
    }
  }
  return pos;
}

// Pairs of record r = v n + g: (global tile v T + t) << 32 | r, in depth
// order (the run of the record of depth rank j starts at scan[j]), a
// record's kept tiles row-major.  A workgroup takes 256 consecutive depth
// ranks, whose runs are one contiguous stretch of the pair array: it stages
// their records' run starts, ids, tile rectangles and masks in LDS, and its
// threads then write the stretch position by position (coalesced stores, a
// long run spread over all lanes), each finding its record by binary search
// over the staged run starts.
constexpr int kEmitThreads = 256;
__global__ void __launch_bounds__(kEmitThreads)
    k_emit(const uint32_t *__restrict__ order, const uint32_t *__restrict__ count_sorted,
           const uint32_t *__restrict__ scan, const float4 *__restrict__ rec,
           const uint64_t *__restrict__ tmask, const int64_t *__restrict__ cnt, int TW, int TH,
           int tiles_x, int tiles_per_view, uint64_t *__restrict__ pairs) {
  __shared__ uint32_t s_start[kEmitThreads], s_g[kEmitThreads], s_row[kEmitThreads];
  __shared__ uint32_t s_wc[kEmitThreads];
  __shared__ uint64_t s_mask[kEmitThreads];
  const int64_t n = cnt[0], nr = cnt[1];
  if (cnt[3] != 0) return;
  const int64_t j0 = (int64_t)blockIdx.x * kEmitThreads;
  if (j0 >= nr) return;
  const int64_t j1 = min(j0 + (int64_t)kEmitThreads, nr);
  const uint32_t first = scan[j0], last = scan[j1];
  const int t = threadIdx.x;
  const int64_t j = j0 + t;
  // an empty or absent entry starts where the next one does; the search
  // below returns the last entry starting at or before a position, which
  // always has pairs (an empty one is followed by one of the same start)
  uint32_t start = last;
  if (j < j1) {
    start = scan[j];
    if (count_sorted[j] > 0) {
      const uint32_t g = order[j];
      const float4 C = rec[4 * (int64_t)g + 2];
      const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
      const int tx0 = (int)(bx & 0xFFFF) / TW, tx1 = (int)(bx >> 16) / TW;
      const int ty0 = (int)(by & 0xFFFF) / TH, ty1 = (int)(by >> 16) / TH;
      const int wc = tx1 - tx0 + 1, n_rect = wc * (ty1 - ty0 + 1);
      s_g[t] = g;
      // the global tile id of the rectangle's top-left tile, and its width
      // (top bit: every tile kept, the mask unused beyond 64 tiles)
      s_row[t] = (uint32_t)(g / n) * (uint32_t)tiles_per_view + (uint32_t)(ty0 * tiles_x + tx0);
      s_wc[t] = (uint32_t)wc | (n_rect > 64 ? 0x80000000u : 0u);
      s_mask[t] = tmask[g];
    }
  }
  s_start[t] = start;
  __syncthreads();
  for (uint32_t p = first + (uint32_t)t; p < last; p += kEmitThreads) {
    int lo = 0, hi = kEmitThreads;  // last entry with start <= p: in [lo, hi)
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_start[mid] <= p) lo = mid;
      else hi = mid;
    }
    const int k = (int)(p - s_start[lo]);
    const uint32_t wf = s_wc[lo];
    const int wc = (int)(wf & 0x7FFFFFFFu);
    const int pos = (wf >> 31) ? k : nth_set_bit(s_mask[lo], k);
    const int dy = pos / wc, dx = pos - dy * wc;
    const uint32_t tile = s_row[lo] + (uint32_t)(dy * tiles_x + dx);
    pairs[p] = ((uint64_t)tile << 32) | s_g[lo];
  }
}

__global__ void k_ranges(const uint64_t *__restrict__ pairs, const int64_t *__restrict__ cnt,
                         int n_tiles, int2 *__restrict__ ranges) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n_tiles) return;
  const int64_t P = cnt[3] != 0 ? 0 : cnt[2];  // an overflowed window draws nothing
  auto lower = [&](uint32_t key) {
    int64_t lo = 0, hi = P;
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if ((uint32_t)(pairs[mid] >> 32) < key) lo = mid + 1;
      else hi = mid;
    }
    return lo;
  };
  ranges[t] = make_int2((int)lower((uint32_t)t), (int)lower((uint32_t)t + 1));
}

// Raster launch order: workgroup b takes tile order[b].  The 8 XCDs receive
// workgroups round-robin (workgroup b runs on XCD b % 8), so the base order
// gives each XCD a contiguous band of tiles (neighbouring tiles share
// Gaussians in its L2).  That order is then sorted, stably, by the bit
// length of each tile's list, longest first: the few long lists (the
// vanishing point of a road holds 100 times the median) start at once
// instead of ending the launch alone, and within a length class the XCD
// bands are kept.  Tiles whose forward is split (more than
// (kFwdSplit - 1) S pairs, S the segment length) go before every other
// tile, so their segments head the work list.  Padding blocks get tile ids >= n_tiles and sort last.
constexpr int kOrderBits = 5;
constexpr int kFwdSplit = 4;  // segments from which a tile's forward is split too
__global__ void k_order_keys(const int2 *__restrict__ ranges, const int64_t *__restrict__ cnt,
                             int n_tiles, int grid, int S, uint32_t *__restrict__ key,
                             uint32_t *__restrict__ val) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= grid) return;
  const int per = (n_tiles + 7) >> 3;
  const int t = (b & 7) * per + (b >> 3);
  uint32_t k = 31;
  if (t < n_tiles && cnt[3] == 0) {
    const int2 r = ranges[t];
    const int L = r.y - r.x;
    k = 31u - (32u - (uint32_t)__clz(L));  // 31 - bit length
    // a forward-split list sorts before every list of at most
    // (kFwdSplit - 1) S pairs (whose keys are at least 31 - that bound's
    // bit length)
    if (L > (kFwdSplit - 1) * S) k = min(k, 30u - (32u - (uint32_t)__clz((kFwdSplit - 1) * S)));
  }
  key[b] = k;
  val[b] = (uint32_t)t;
}

struct Sample {
  bool ok;
  float power, G, alpha, dx, dy;  // power: the exponent in base 2
};

struct Box {
  int i0, i1, j0, j1;  // inclusive pixel columns i0..i1, rows j0..j1
};


// The one definition of a (pixel, Gaussian) sample, shared by forward and
// backward so that both take identical threshold decisions.
// The pixel is (X0 + lx, Y0 + ly): (X0, Y0) the origin of its 8x8 cell and
// (i0..i1, j0..j1) the record's pixel box, all wavefront-uniform; lxh, lyh
// = lx + 0.5, ly + 0.5.  The offset from the box corner, (X0 + lx + 0.5) -
// i0 = lxh + (X0 - i0), is exact in float32 (small half-integers), so dx is
// the rounding of (px - i0 + 0.5) - A.x.
__device__ __forceinline__ Sample sample(int lx, int ly, float lxh, float lyh, int X0, int Y0,
                                         const Box &b, const float4 &A, const float4 &B) {
  // No implicit FMA contraction here: every kernel that inlines this takes
  // the same roundings (HIP's __f*_rn helpers are plain operators).
#pragma clang fp contract(off)
  Sample s;
  // bitwise, not short-circuit: no lane-mask branch for a partial cell; one
  // unsigned range compare per axis (the box is never empty: i0 <= i1)
  s.ok = ((uint32_t)(lx - (b.i0 - X0)) <= (uint32_t)(b.i1 - b.i0)) &
         ((uint32_t)(ly - (b.j0 - Y0)) <= (uint32_t)(b.j1 - b.j0));
  s.dx = (lxh + (float)(X0 - b.i0)) - A.x;
  s.dy = (lyh + (float)(Y0 - b.j0)) - A.y;
  // the record holds the conic scaled by -log2(e) / 2 (off-diagonal by
  // -log2(e)), so the exponent comes out in base 2: power = log2(e) (-d^T Q d / 2)
  const float t = __builtin_fmaf(B.x, s.dy * s.dy, A.w * (s.dx * s.dy));
  s.power = __builtin_fmaf(A.z, s.dx * s.dx, t);
  s.G = __builtin_amdgcn_exp2f(s.power);  // e^(-d^T Q d / 2)
  const float oG = B.y * s.G;
  s.alpha = fminf(kAlphaMax, oG);
  s.ok = s.ok & !(s.power > 0.0f) & !(s.alpha < kAlphaMin);
  return s;
}

// Lane layout of the rasterizers.  A tile is a grid of 8x8-pixel cells,
// numbered row-major; cell j (0 <= j < PPT) of wavefront w is cell
// w * PPT + j, and lane l holds its pixel (l % 8, l / 8).  A cell is one
// wavefront-wide pixel set, so whether a record's box meets it, and whether
// any of its pixels still composites, are uniform branches that skip the
// cell's arithmetic for the whole wavefront.
template <int TW, int TH, int PPT>
struct CellLayout {
  static_assert(TW % 8 == 0 && TH % 8 == 0, "tiles are whole 8x8 cells");
  static_assert((TW * TH / PPT) % kWave == 0, "whole wavefronts per tile");
  static constexpr int kCells = TW * TH / 64;  // at most 32
  int w;                 // this wavefront (uniform)
  int X0[PPT], Y0[PPT];  // its cells' origins in pixels (uniform)
  __device__ __forceinline__ CellLayout(int tx, int ty) {
    w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int c = w * PPT + j;
      X0[j] = tx * TW + (c % (TW / 8)) * 8;
      Y0[j] = ty * TH + (c / (TW / 8)) * 8;
    }
  }
  // Bit c set: some pixel of cell c of tile (tx, ty) may take the record
  // (A, B, C): the cell meets the record's pixel box and, unless that cannot
  // be decided safely, the record's alpha >= 1/255 ellipse.  Computed once
  // per record and tile by the thread that stages the record; a cleared bit
  // only lets a wavefront skip a cell whose every pixel the sample test
  // would reject.
  static __device__ __forceinline__ uint32_t cell_mask(const float4 &A, const float4 &B,
                                                       const float4 &C, int tx, int ty) {
    const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
    const int i0 = bx & 0xFFFF, i1 = bx >> 16, j0 = by & 0xFFFF, j1 = by >> 16;
    // -power = P(d) = p00 dx^2 + 2 p01 dx dy + p11 dy^2 for d = pixel centre
    // - mean; a pixel passes only if P(d) <= log2(255 o) (alpha >= 1/255).
    // Float32 throughout (float64 here would cost the rasterizer registers).
    const float p00 = -A.z, p01 = -0.5f * A.w, p11 = -B.x;
    const bool exact = p00 > 0.0f && p11 > 0.0f && p00 * p11 > p01 * p01 && B.y > 0.0f;
    // threshold with room for the float32 exponent, opacity product and
    // constant roundings of the sample test (a few 1e-7 in log2 units)
    const float thr = exact ? __log2f(255.0f * B.y) + 1e-3f : 0.0f;
    uint32_t m = 0;
#pragma unroll
    for (int c = 0; c < kCells; ++c) {
      const int x0 = tx * TW + (c % (TW / 8)) * 8, y0 = ty * TH + (c / (TW / 8)) * 8;
      // the cell's pixels inside the box
      const int xa = max(x0, i0), xb = min(x0 + 7, i1), ya = max(y0, j0), yb = min(y0 + 7, j1);
      if (xa > xb || ya > yb) continue;
      if (!exact) {
        m |= 1u << c;
        continue;
      }
      // their centres relative to the mean, rounded as the sample test's
      // dx, dy are (the first operands are exact half-integers)
      const float ax = ((float)(xa - i0) + 0.5f) - A.x, bx = ((float)(xb - i0) + 0.5f) - A.x;
      const float ay = ((float)(ya - j0) + 0.5f) - A.y, by = ((float)(yb - j0) + 0.5f) - A.y;
      // minimum of P over that rectangle: 0 inside, else on an edge (any
      // point of an edge gives an upper bound; the clamped one is the minimum)
      float pmin = 0.0f;
      if (!(ax <= 0.0f && bx >= 0.0f && ay <= 0.0f && by >= 0.0f)) {
        const float ex[2] = {ax, bx}, ey[2] = {ay, by};
        // an approximate reciprocal moves the edge point by a few ulp,
        // which raises P by a second-order amount far below err
        const float r00 = __builtin_amdgcn_rcpf(p00), r11 = __builtin_amdgcn_rcpf(p11);
        pmin = 3.0e38f;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const float x = ex[e], yy = fminf(fmaxf(-p01 * x * r11, ay), by);
          pmin = fminf(pmin, p00 * x * x + 2.0f * p01 * x * yy + p11 * yy * yy);
          const float y = ey[e], xx = fminf(fmaxf(-p01 * y * r00, ax), bx);
          pmin = fminf(pmin, p00 * xx * xx + 2.0f * p01 * xx * y + p11 * y * y);
        }
      }
      // bound on the float32 rounding of P here and in the sample test at
      // any of the pixels: a handful of roundings each of terms no larger
      // than these
      const float X = fmaxf(fabsf(ax), fabsf(bx)), Y = fmaxf(fabsf(ay), fabsf(by));
      const float err = 32.0f * 0x1p-24f * (p00 * X * X + 2.0f * fabsf(p01) * X * Y + p11 * Y * Y);
      if (pmin - err <= thr) m |= 1u << c;
    }
    return m;
  }
  // this wavefront's PPT bits of a tile cell mask (uniform)
  __device__ __forceinline__ uint32_t mine(uint32_t m) const {
    return (m >> (w * PPT)) & ((1u << PPT) - 1u);
  }
};

// A record's packed pixel box, read once per wavefront into scalar registers.
__device__ __forceinline__ Box uniform_box(const float4 &C) {
  const uint32_t bx = __builtin_amdgcn_readfirstlane(__float_as_uint(C.z));
  const uint32_t by = __builtin_amdgcn_readfirstlane(__float_as_uint(C.w));
  Box b;
  b.i0 = bx & 0xFFFF;
  b.i1 = bx >> 16;
  b.j0 = by & 0xFFFF;
  b.j1 = by >> 16;
  return b;
}

// Long lists are split for the backward into segments of 64 list positions
// per pixel of the tile (4096 for 8x8 tiles, 16384 for 16x16; a multiple of
// every raster batch size): one workgroup per (tile, segment).  For a split
// tile the forward stores each pixel's compositing state (T, colour, depth)
// at every segment end (the list's end included), so a segment's backward
// starts where the reverse sweep of the whole list would be at that
// position: T from the stored state, and the colour and depth composited
// behind it as the final values minus those stored.  (A list of kFwdSplit
// or more segments is split in the forward as well; see k_raster_fwd.)
constexpr int kSegPerPixel = 64;
constexpr int kStateVals = 5;  // T, colour r, g, b, depth

__host__ __device__ constexpr int seg_len(int tw, int th) { return kSegPerPixel * tw * th; }
__device__ __forceinline__ int seg_count(int L, int S) { return L > S ? (L + S - 1) / S : 1; }

// Per position b of the launch order: work items (segments) of its tile,
// and boundary-state slots (one per segment of a split tile).
__global__ void k_seg_count(const uint32_t *__restrict__ order, const int2 *__restrict__ ranges,
                            int n_tiles, int grid, int S, uint32_t *__restrict__ cw,
                            uint32_t *__restrict__ cb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= grid) return;
  const int t = (int)order[b];
  uint32_t w = 0, bs = 0;
  if (t < n_tiles) {
    const int2 r = ranges[t];
    const int ns = seg_count(r.y - r.x, S);
    w = (uint32_t)ns;
    bs = ns > 1 ? (uint32_t)ns : 0u;
  }
  cw[b] = w;
  cb[b] = bs;
}

// The work list (tile, segment) in launch order, each tile's first
// boundary slot (-1: not split), the work-item count cnt[6] and cnt[7], the
// count of work items of forward-split tiles (the first ones of the list).
__global__ void k_seg_fill(const uint32_t *__restrict__ order, const int2 *__restrict__ ranges,
                           int n_tiles, int grid, int S, const uint32_t *__restrict__ cw,
                           const uint32_t *__restrict__ sw, const uint32_t *__restrict__ cb,
                           const uint32_t *__restrict__ sb, int2 *__restrict__ witem,
                           int *__restrict__ bslot, int64_t *__restrict__ cnt) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b == 0) cnt[6] = (int64_t)sw[grid];
  if (b >= grid) return;
  auto fwd_split = [&](const int q) {
    const int u = (int)order[q];
    if (u >= n_tiles) return false;
    const int2 r = ranges[u];
    return seg_count(r.y - r.x, S) >= kFwdSplit;
  };
  const bool fs = fwd_split(b);
  if (b == 0 && !fs) cnt[7] = 0;
  if (fs && (b + 1 == grid || !fwd_split(b + 1))) cnt[7] = (int64_t)sw[b + 1];
  const int t = (int)order[b];
  if (t >= n_tiles) return;
  const uint32_t w0 = sw[b];
  for (uint32_t i = 0; i < cw[b]; ++i) witem[w0 + i] = make_int2(t, (int)i);
  bslot[t] = cb[b] != 0 ? (int)sb[b] : -1;
}

// Records per straight-line group of the one-cell forward rasterizer.
constexpr int kFwdGroup = 4;

// A list of at least kFwdSplit segments is also split in the forward (a
// single wavefront walking it would end the launch alone): pass 1 takes,
// per segment and pixel, the product of (1 - alpha) over the segment's
// samples; pass 2 composites each segment from the transmittance the
// earlier segments' products leave (a pixel whose product chain falls
// below 1e-4 stopped in that segment), with colour and depth from zero;
// a combine kernel sums the segments in order into the pixel's outputs and
// rewrites the segment-end states as running totals for the backward.
// Pass 0 is the whole-list forward of every other tile.  Per segment slot
// the pass state holds 3 planes: the product, the last composited position
// and how the segment ended for the pixel.  These tiles' work items are the
// first cnt[7] of the work list: the three kernels' grids cover at most
// k pairs / ((k - 1) S) of them, k = kFwdSplit (a split list of
// L > (k - 1) S pairs has at most L / S + 1 < k L / ((k - 1) S) segments).
constexpr int kFsegVals = 3;
enum : int { kSegAlive = 0, kSegStopped = 1, kSegDead = 2 };

template <int TW, int TH, int PPT, int PASS>
__global__ void __launch_bounds__(TW * TH / PPT)
    k_raster_fwd(const uint64_t *__restrict__ pairs, const int2 *__restrict__ ranges,
                 const uint32_t *__restrict__ order,
                 const float4 *__restrict__ rec, int64_t RS, int W, int H, int tiles_x,
                 int n_tiles, int tiles_per_view, float bg0, float bg1, float bg2,
                 float *__restrict__ rgb, float *__restrict__ depth, float *__restrict__ Tout,
                 float *__restrict__ Tstate, int *__restrict__ last_out,
                 const int *__restrict__ bslot, float *__restrict__ bound,
                 const int2 *__restrict__ witem, const int64_t *__restrict__ cnt,
                 float *__restrict__ fseg) {
#pragma clang fp contract(off)
  constexpr int NT = TW * TH / PPT;
  constexpr int BS = NT;
  constexpr int PX = TW * TH;
  constexpr int kSegLen = seg_len(TW, TH);
  static_assert(kSegLen % BS == 0, "segment ends fall on batch starts");
  __shared__ float4 sA[BS], sB[BS], sC[BS];
  __shared__ uint32_t sM[BS];
  // a one-cell tile needs no cell masks: every record of its list meets it
  // or is rejected pixel by pixel
  constexpr bool kOneCell = CellLayout<TW, TH, PPT>::kCells == 1;
  int gt, seg = 0;
  if constexpr (PASS == 0) {
    gt = (int)order[blockIdx.x];
    if (gt >= n_tiles) return;
  } else {  // one segment of a forward-split tile
    if (blockIdx.x >= cnt[7]) return;
    const int2 wi = witem[blockIdx.x];
    gt = wi.x;
    seg = wi.y;
  }
  const int2 rg = ranges[gt];
  const int nseg = seg_count(rg.y - rg.x, kSegLen);
  if ((PASS == 0) == (nseg >= kFwdSplit)) return;  // the other passes' tile
  const int r_lo = PASS == 0 ? rg.x : rg.x + seg * kSegLen;
  const int r_hi = PASS == 0 ? rg.y : min(r_lo + kSegLen, rg.y);
  const int view = gt / tiles_per_view, tile = gt - view * tiles_per_view;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  {  // this view's images
    const int64_t HWv = (int64_t)W * H;
    rgb += view * 3 * HWv;
    if (depth) depth += view * HWv;
    if (Tout) Tout += view * HWv;
    Tstate += view * HWv;
    last_out += view * HWv;
  }
  const CellLayout<TW, TH, PPT> cell(tx, ty);
  const int lx = threadIdx.x & 7, ly = (threadIdx.x >> 3) & 7;
  const float lxh = (float)lx + 0.5f, lyh = (float)ly + 0.5f;
  float T[PPT], c0[PPT], c1[PPT], c2[PPT], D[PPT];
  int last[PPT];
  bool done[PPT];
  int n_live = 0;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    T[j] = 1.0f;
    c0[j] = c1[j] = c2[j] = D[j] = 0.0f;
    last[j] = -1;
    done[j] = !(cell.X0[j] + lx < W && cell.Y0[j] + ly < H);
    n_live += !done[j];
  }
  // a split tile stores each pixel's state at every segment end: slot
  // bs + i holds it after the records before segment i + 1 (the last slot:
  // after the whole list)
  const int bs = bslot[gt];
  auto lpix = [&](const int j) {
    return (cell.Y0[j] - ty * TH + ly) * TW + (cell.X0[j] - tx * TW + lx);
  };
  if constexpr (PASS == 2) {
    // the transmittance entering this segment: the earlier segments'
    // products in order; a pixel whose chain falls below 1e-4 stopped in
    // an earlier segment and takes nothing here
    n_live = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      float Tr = 1.0f;
      bool dead = done[j];
      for (int q = 0; q < seg && !dead; ++q) {
        const float Tn = Tr * fseg[(int64_t)(bs + q) * kFsegVals * PX + lpix(j)];
        dead = Tn < kTMin;
        Tr = dead ? Tr : Tn;
      }
      T[j] = Tr;
      done[j] = dead;
      n_live += !dead;
    }
  }
  bool dead_in[PPT];
#pragma unroll
  for (int j = 0; j < PPT; ++j) dead_in[j] = done[j];
  auto store_state = [&](const int slot) {
    float *o = bound + (int64_t)slot * kStateVals * (TW * TH);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      const int lp = lpix(j);
      o[lp] = T[j];
      o[TW * TH + lp] = c0[j];
      o[2 * TW * TH + lp] = c1[j];
      o[3 * TW * TH + lp] = c2[j];
      o[4 * TW * TH + lp] = D[j];
    }
  };
  for (int base = r_lo; base < r_hi; base += BS) {
    // once every pixel is saturated no later segment end is needed: a
    // segment's backward reads its end state only for pixels that
    // composited a record behind that end
    if (__syncthreads_count(n_live) == 0) break;
    if (PASS == 0 && bs >= 0 && base > rg.x && (base - rg.x) % kSegLen == 0)
      store_state(bs + (base - rg.x) / kSegLen - 1);
    const int p = base + threadIdx.x;
    if (p < r_hi) {
      const uint32_t g = (uint32_t)pairs[p];
      const float4 *q = rec + 4 * (int64_t)g;  // a 64-byte record: its first 48 bytes
      const float4 A = q[0], B = q[1], C = q[2];
      sA[threadIdx.x] = A;
      sB[threadIdx.x] = B;
      sC[threadIdx.x] = C;
      if constexpr (!kOneCell)
        sM[threadIdx.x] = CellLayout<TW, TH, PPT>::cell_mask(A, B, C, tx, ty);
    }
    __syncthreads();
    const int nb = min(BS, r_hi - base);
    // one compositing step of cell j with the record's sample s: predicated
    // rather than branched inside a cell (a lane that does not composite
    // adds exact zeros, and the wavefront issues no mask bookkeeping);
    // contraction is off in this kernel, so every raster shape composites
    // with the same roundings
    auto composite = [&](const int j, const Sample &s, const bool valid, const float4 &B,
                         const float4 &C, const int pos) {
      if constexpr (PASS == 1) {  // the segment's product of (1 - alpha), no stopping
        const bool act = valid & s.ok & !done[j];
        T[j] = T[j] * (1.0f - (act ? s.alpha : 0.0f));
        return;
      }
      const bool act = valid & s.ok & !done[j];
      const float a = act ? s.alpha : 0.0f;
      const float Tn = T[j] * (1.0f - a);
      const bool stop = act & (Tn < kTMin);
      const bool comp = act & !stop;
      const float w = comp ? a * T[j] : 0.0f;
      c0[j] = __builtin_fmaf(B.z, w, c0[j]);
      c1[j] = __builtin_fmaf(B.w, w, c1[j]);
      c2[j] = __builtin_fmaf(C.x, w, c2[j]);
      D[j] = __builtin_fmaf(C.y, w, D[j]);
      T[j] = comp ? Tn : T[j];
      last[j] = comp ? pos : last[j];
      done[j] = done[j] | stop;
    };
    uint32_t m_next = kOneCell ? 1u : sM[0];  // the next record's cell mask, read a step ahead
    for (int k0 = 0; k0 < nb; k0 += 8) {
      // every 8 records: cells whose pixels are all saturated leave the
      // batch; a wavefront with none left leaves it altogether
      uint32_t live = 0;
#pragma unroll
      for (int j = 0; j < PPT; ++j) live |= (uint32_t)(__ballot(!done[j]) != 0) << j;
      if (live == 0) break;
      const int k1 = min(k0 + 8, nb);
      if constexpr (kOneCell) {
        // one cell per tile: no masks, every record of the list is taken.
        // Records go in straight-line groups: the group's samples do not
        // depend on the compositing state, so their loads and arithmetic
        // overlap, and the compositing steps follow in list order.  A slot
        // past the batch repeats its last record with valid false (it
        // changes nothing).
        for (int kg = k0; kg < k1; kg += kFwdGroup) {
          Sample sg[kFwdGroup];
          float4 Bg[kFwdGroup], Cg[kFwdGroup];
#pragma unroll
          for (int g = 0; g < kFwdGroup; ++g) {
            const int k = min(kg + g, k1 - 1);
            const float4 A = sA[k];
            Bg[g] = sB[k];
            Cg[g] = sC[k];
            sg[g] = sample(lx, ly, lxh, lyh, cell.X0[0], cell.Y0[0], uniform_box(Cg[g]), A, Bg[g]);
          }
#pragma unroll
          for (int g = 0; g < kFwdGroup; ++g)
            composite(0, sg[g], kg + g < k1, Bg[g], Cg[g], base + kg + g);
        }
        continue;
      }
      for (int k = k0; k < k1; ++k) {
        const uint32_t mk = __builtin_amdgcn_readfirstlane(m_next);
        m_next = sM[min(k + 1, BS - 1)];
        const uint32_t hit = cell.mine(mk) & live;
        if (hit == 0) continue;  // no live cell of this wavefront meets the box
        const float4 A = sA[k], B = sB[k], C = sC[k];
        const Box bx = uniform_box(C);
        // one cell at a time (straight-line code over all cells holds more
        // registers and runs slower here)
#pragma unroll
        for (int j = 0; j < PPT; ++j)
          if (hit & (1u << j))
            composite(j, sample(lx, ly, lxh, lyh, cell.X0[j], cell.Y0[j], bx, A, B), true, B, C,
                      base + k);
      }
    }
    n_live = 0;
#pragma unroll
    for (int j = 0; j < PPT; ++j) n_live += !done[j];
  }
  if constexpr (PASS == 1) {
#pragma unroll
    for (int j = 0; j < PPT; ++j) fseg[(int64_t)(bs + seg) * kFsegVals * PX + lpix(j)] = T[j];
    return;
  }
  if constexpr (PASS == 2) {
    // the segment's own colour and depth, its end transmittance, last
    // position and how it ended (the combine kernel makes totals of them)
    store_state(bs + seg);
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
      float *f = fseg + (int64_t)(bs + seg) * kFsegVals * PX + lpix(j);
      f[PX] = __int_as_float(last[j]);
      f[2 * PX] = __int_as_float(dead_in[j] ? kSegDead : done[j] ? kSegStopped : kSegAlive);
    }
    return;
  }
  if (bs >= 0) store_state(bs + nseg - 1);
  const int64_t HW = (int64_t)W * H;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    const int px = cell.X0[j] + lx, py = cell.Y0[j] + ly;
    if (!(px < W && py < H)) continue;
    const int64_t pix = (int64_t)py * W + px;
    rgb[pix] = __builtin_fmaf(T[j], bg0, c0[j]);
    rgb[HW + pix] = __builtin_fmaf(T[j], bg1, c1[j]);
    rgb[2 * HW + pix] = __builtin_fmaf(T[j], bg2, c2[j]);
    if (depth) depth[pix] = D[j];
    if (Tout) Tout[pix] = T[j];
    Tstate[pix] = T[j];
    last_out[pix] = last[j];
  }
}

// The forward of a tile split into kFwdSplit or more segments, finished:
// one thread per pixel of the tile walks its segments in order, adding
// their colour and depth (fixed order) up to the segment where it stopped,
// writes the pixel's outputs, and turns each segment-end state into
// running totals (what the backward reads there).
template <int TW, int TH>
__global__ void __launch_bounds__(TW * TH)
    k_fwd_combine(const int2 *__restrict__ ranges, const int2 *__restrict__ witem,
                  const int64_t *__restrict__ cnt, const int *__restrict__ bslot, int W, int H,
                  int tiles_x, int tiles_per_view, float bg0, float bg1, float bg2,
                  float *__restrict__ rgb, float *__restrict__ depth, float *__restrict__ Tout,
                  float *__restrict__ Tstate, int *__restrict__ last_out,
                  float *__restrict__ bound, const float *__restrict__ fseg) {
#pragma clang fp contract(off)
  constexpr int PX = TW * TH;
  constexpr int kSegLen = seg_len(TW, TH);
  if (blockIdx.x >= cnt[7]) return;
  const int2 wi = witem[blockIdx.x];
  if (wi.y != 0) return;  // one workgroup per tile
  const int gt = wi.x;
  const int2 rg = ranges[gt];
  const int nseg = seg_count(rg.y - rg.x, kSegLen);
  if (nseg < kFwdSplit) return;
  const int bs = bslot[gt];
  const int lp = threadIdx.x;
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, Dd = 0.0f, Tf = 1.0f;
  int lastp = -1;
  bool ended = false;
  for (int i = 0; i < nseg; ++i) {
    float *o = bound + (int64_t)(bs + i) * kStateVals * PX + lp;
    const float *f = fseg + (int64_t)(bs + i) * kFsegVals * PX + lp;
    if (!ended) {
      const int how = __float_as_int(f[2 * PX]);
      if (how == kSegDead) {
        ended = true;
      } else {
        C0 += o[PX];
        C1 += o[2 * PX];
        C2 += o[3 * PX];
        Dd += o[4 * PX];
        Tf = o[0];
        const int l = __float_as_int(f[PX]);
        lastp = l >= 0 ? l : lastp;
        ended = how == kSegStopped;
      }
    }
    o[0] = Tf;
    o[PX] = C0;
    o[2 * PX] = C1;
    o[3 * PX] = C2;
    o[4 * PX] = Dd;
  }
  const int view = gt / tiles_per_view, tile = gt - view * tiles_per_view;
  const int px = (tile % tiles_x) * TW + lp % TW, py = (tile / tiles_x) * TH + lp / TW;
  if (!(px < W && py < H)) return;
  const int64_t HW = (int64_t)W * H, o = (int64_t)py * W + px;
  rgb[(3 * view) * HW + o] = __builtin_fmaf(Tf, bg0, C0);
  rgb[(3 * view + 1) * HW + o] = __builtin_fmaf(Tf, bg1, C1);
  rgb[(3 * view + 2) * HW + o] = __builtin_fmaf(Tf, bg2, C2);
  if (depth) depth[view * HW + o] = Dd;
  if (Tout) Tout[view * HW + o] = Tf;
  Tstate[view * HW + o] = Tf;
  last_out[view * HW + o] = lastp;
}

// Cross-lane moves inside 16-lane rows through DPP (VALU, no LDS path).
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kDppXor1 = 0xB1;    // quad_perm [1,0,3,2]
constexpr int kDppXor2 = 0x4E;    // quad_perm [2,3,0,1]
constexpr int kDppShl4 = 0x104;   // row_shl:4 (lane i reads lane i + 4)
constexpr int kDppShr4 = 0x114;   // row_shr:4 (lane i reads lane i - 4)
constexpr int kDppRor8 = 0x128;   // row_ror:8 (lane i reads lane i ^ 8 in a row)

// Sum of 10 values over a wavefront by a halving butterfly: at each level a
// lane keeps half of its value slots and adds its partner's copy of that
// half, so a slot always stands for one value index.  Levels 1, 2, 4, 8
// stay inside 16-lane rows (DPP); the two cross-row levels move one value
// each (row swaps).  Afterwards the lane whose low 4 bits are l
// holds the wave total of value bitrev4(l) (for bitrev4(l) < 10).  Value
// indices 10..15 do not exist: at the first level the slots that would
// carry them are left to hold anything, which saves their selects.
__device__ __forceinline__ float wave_reduce10(float (&v)[16]) {
  const int lane = threadIdx.x & (kWave - 1);
  {
    const bool hi = lane & 1;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = hi ? v[i] : v[i + 8];
      const float keep = hi ? v[i + 8] : v[i];
      v[i] = keep + dpp<kDppXor1>(send);
    }
    // slots 2..7: values 2..7 on even lanes, nothing (10..15) on odd ones
#pragma unroll
    for (int i = 2; i < 8; ++i) v[i] = v[i] + dpp<kDppXor1>(v[i]);
  }
  {
    const bool hi = lane & 2;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float send = hi ? v[i] : v[i + 4];
      const float keep = hi ? v[i + 4] : v[i];
      v[i] = keep + dpp<kDppXor2>(send);
    }
  }
  {
    const bool hi = lane & 4;
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float send = hi ? v[i] : v[i + 2];
      const float keep = hi ? v[i + 2] : v[i];
      const float up = dpp<kDppShl4>(send), down = dpp<kDppShr4>(send);
      v[i] = keep + (hi ? down : up);
    }
  }
  {
    const bool hi = lane & 8;
    const float send = hi ? v[0] : v[1];
    const float keep = hi ? v[1] : v[0];
    v[0] = keep + dpp<kDppRor8>(send);
  }
  // the two cross-row levels with gfx950's row swaps (VALU, no LDS
  // crossbar): each yields a lane's value and its partner's, lower row
  // first in both lanes
  float r = v[0];
  {
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(r), __float_as_uint(r),
                                                    false, false);
    r = __uint_as_float(q[0]) + __uint_as_float(q[1]);  // lanes l and l ^ 16
  }
  {
    const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(r), __float_as_uint(r),
                                                    false, false);
    r = __uint_as_float(q[0]) + __uint_as_float(q[1]);  // lanes l and l ^ 32
  }
  return r;
}

__device__ __forceinline__ int bitrev4(int l) {
  return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

template <int TW, int TH, int PPT>
__global__ void __launch_bounds__(TW * TH / PPT)
    k_raster_bwd(const uint64_t *__restrict__ pairs, const int2 *__restrict__ ranges,
                 const int2 *__restrict__ witem, const int64_t *__restrict__ cnt,
                 const float4 *__restrict__ rec, int64_t RS, int W, int H, int tiles_x,
                 int n_tiles, int tiles_per_view, float bg0, float bg1, float bg2,
                 const float *__restrict__ Tstate, const int *__restrict__ last_in,
                 const float *__restrict__ dl_drgb, const float *__restrict__ dl_ddepth,
                 float2 *__restrict__ partial, uint64_t *__restrict__ frontier,
                 const int *__restrict__ bslot,
                 const float *__restrict__ bound, const uint32_t *__restrict__ seg_off) {
  constexpr int NT = TW * TH / PPT;
  constexpr int NW = NT / kWave;
  // records per batch: at most 64, so a tile of several wavefronts keeps
  // its LDS (records, masks, per-wavefront reductions) small enough for
  // eight workgroups per CU
  constexpr int BS = NT < 64 ? NT : 64;
  constexpr int NC = 10;
  __shared__ float4 sA[BS], sB[BS], sC[BS];
  __shared__ uint32_t sP[BS], sM[BS];  // gradient slot base of the record, cell mask
  __shared__ uint64_t sT[BS];          // kept-tile mask of the record
  __shared__ float red[NW][BS][NC];
  constexpr bool kOneCell = CellLayout<TW, TH, PPT>::kCells == 1;  // no cell masks needed
  __shared__ int max_last;
  // work item: segment seg of tile gt (the whole list when it is not split)
  if (blockIdx.x >= cnt[6]) return;
  const int2 wi = witem[blockIdx.x];
  const int gt = wi.x, seg = wi.y;
  const int view = gt / tiles_per_view, tile = gt - view * tiles_per_view;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  {  // this view's images and upstream gradients
    const int64_t HWv = (int64_t)W * H;
    Tstate += view * HWv;
    last_in += view * HWv;
    dl_drgb += view * 3 * HWv;
    if (dl_ddepth) dl_ddepth += view * HWv;
  }
  const CellLayout<TW, TH, PPT> cell(tx, ty);
  const int lx = threadIdx.x & 7, ly = (threadIdx.x >> 3) & 7;
  const float lxh = (float)lx + 0.5f, lyh = (float)ly + 0.5f;
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const int2 rg = ranges[gt];
  constexpr int kSegLen = seg_len(TW, TH);
  static_assert(kSegLen % BS == 0, "segment ends fall on batch starts");
  const int nseg = seg_count(rg.y - rg.x, kSegLen);
  const int s_lo = rg.x + seg * kSegLen, s_hi = nseg > 1 ? min(s_lo + kSegLen, rg.y) : rg.y;
  const int bs = nseg > 1 ? bslot[gt] : -1;
  const int64_t HW = (int64_t)W * H;
  // GS = dL/dC . (colour and depth composited behind the current Gaussian,
  // background included): dalpha needs only this dot product
  float T[PPT], g0[PPT], g1[PPT], g2[PPT], gd[PPT], GS[PPT];
  int last[PPT], cell_last[PPT];
  int my_last = -1;
#pragma unroll
  for (int j = 0; j < PPT; ++j) {
    T[j] = 1.0f;
    g0[j] = g1[j] = g2[j] = gd[j] = 0.0f;
    last[j] = -1;
    const int px = cell.X0[j] + lx, py = cell.Y0[j] + ly;
    if (px < W && py < H) {
      const int64_t pix = (int64_t)py * W + px;
      T[j] = Tstate[pix];
      last[j] = last_in[pix];
      g0[j] = dl_drgb[pix];
      g1[j] = dl_drgb[HW + pix];
      g2[j] = dl_drgb[2 * HW + pix];
      if (dl_ddepth) gd[j] = dl_ddepth[pix];
    }
    GS[j] = T[j] * (g0[j] * bg0 + g1[j] * bg1 + g2[j] * bg2);
    if (bs >= 0 && last[j] >= s_hi) {
      // the pixel composited records behind this segment: its sweep enters
      // the segment at the segment's end, with T stored there by the
      // forward and, behind it, the final colour (background included) and
      // depth minus those accumulated up to that end
      const int lp = (cell.Y0[j] - ty * TH + ly) * TW + (cell.X0[j] - tx * TW + lx);
      const float *e = bound + (int64_t)(bs + seg) * kStateVals * (TW * TH) + lp;
      const float *f = bound + (int64_t)(bs + nseg - 1) * kStateVals * (TW * TH) + lp;
      const float Tf = f[0];
      T[j] = e[0];
      GS[j] = g0[j] * ((f[TW * TH] + Tf * bg0) - e[TW * TH]) +
              g1[j] * ((f[2 * TW * TH] + Tf * bg1) - e[2 * TW * TH]) +
              g2[j] * ((f[3 * TW * TH] + Tf * bg2) - e[3 * TW * TH]) +
              gd[j] * (f[4 * TW * TH] - e[4 * TW * TH]);
    }
    // the last list position any pixel of cell j composited (uniform)
    int m = last[j];
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) m = max(m, __shfl_xor(m, off));
    cell_last[j] = __builtin_amdgcn_readfirstlane(m);
    my_last = max(my_last, cell_last[j]);
  }
  if (threadIdx.x == 0) max_last = -1;
  __syncthreads();
  if (lane == 0 && my_last >= 0) atomicMax(&max_last, my_last);
  __syncthreads();
  // top: the deepest position any pixel of the tile composited; the
  // segment holding it (segment 0 when there is none) records the frontier
  const int top = max_last;
  if (threadIdx.x == 0 && ((top >= s_lo && top < s_hi) || (top < rg.x && seg == 0)))
    frontier[gt] = top < rg.x ? 0 : depth_order_key(rec, (uint32_t)pairs[top]);
  const int seg_top = min(top, s_hi - 1);
  for (int end = seg_top + 1; end > s_lo; end -= BS) {
    const int beg = max(s_lo, end - BS);
    const int nb = end - beg;
    if (threadIdx.x < nb) {  // slot k holds position end - 1 - k
      const uint32_t g = (uint32_t)pairs[end - 1 - threadIdx.x];
      const float4 *q = rec + 4 * (int64_t)g;  // one 64-byte record
      const float4 A = q[0], B = q[1], C = q[2], Dq = q[3];
      sP[threadIdx.x] = slot_base(seg_off, Dq);
      sT[threadIdx.x] = (uint64_t)__float_as_uint(Dq.y) | ((uint64_t)__float_as_uint(Dq.z) << 32);
      sA[threadIdx.x] = A;
      sB[threadIdx.x] = B;
      sC[threadIdx.x] = C;
      if constexpr (!kOneCell)
        sM[threadIdx.x] = CellLayout<TW, TH, PPT>::cell_mask(A, B, C, tx, ty);
    }
    __syncthreads();
    // one adjoint step of cell j for the record (s, B, C) at list position
    // pos, into the record's accumulators v (lanes that composited it are
    // added to contrib).  Predicated rather than branched inside a cell: a
    // lane whose pixel does not use this Gaussian runs with alpha = 0 (1 / (1
    // - 0) is exact), which leaves T and S unchanged and adds exact zeros to
    // every term.
    auto adjoint = [&](const int j, const Sample &s, const bool valid, const float4 &B,
                       const float4 &C, const int pos, float (&v)[16], uint64_t &contrib) {
      const bool act = valid & s.ok & (pos <= last[j]);
      contrib |= __ballot(act);
      const float a = act ? s.alpha : 0.0f;
      const float iom = __builtin_amdgcn_rcpf(1.0f - a);
      const float Tk = T[j] * iom;  // transmittance in front of this Gaussian
      const float w = a * Tk;
      v[6] += g0[j] * w;
      v[7] += g1[j] * w;
      v[8] += g2[j] * w;
      v[9] += gd[j] * w;
      // dL/dalpha = dL/dC . (c Tk - S / (1 - alpha)), S what lies behind
      const float gc = g0[j] * B.z + g1[j] * B.w + g2[j] * C.x + gd[j] * C.y;
      const float da = gc * Tk - GS[j] * iom;
      GS[j] += gc * w;
      T[j] = Tk;
      // alpha not clamped: the opacity and the exponent receive gradient
      const bool free_alpha = act & (B.y * s.G <= kAlphaMax);
      const float gG = free_alpha ? s.G : 0.0f;
      const float dp = free_alpha ? a * da : 0.0f;
      v[5] += gG * da;
      // the mean's gradient is linear in (sum dp dx, sum dp dy): the conic
      // (scaled: Q00 dx + Q01 dy = kQ/2 (2 A.z dx + A.w dy)) is applied once
      // per record after the reduction
      v[0] += dp * s.dx;
      v[1] += dp * s.dy;
      // d power / d(Q00, Q01, Q11) = -(dx^2 / 2, dx dy, dy^2 / 2): the
      // constant factors are applied after the reduction
      v[2] += s.dx * s.dx * dp;
      v[3] += s.dx * s.dy * dp;
      v[4] += s.dy * s.dy * dp;
    };
    const int c_red = bitrev4(lane & 15);  // the value a reduction leaves in this lane
    uint32_t m_next = kOneCell ? 1u : sM[0];  // the next record's cell mask, read a step ahead
    for (int k0 = 0; k0 < nb; k0 += 8) {
      // cell j takes part in a group of 8 positions if one of its pixels
      // composited the group's deepest position or one behind it (a cell
      // run for a position none of its pixels reached adds exact zeros)
      const int deepest = end - 1 - min(k0 + 7, nb - 1);
      uint32_t alive = 0;
#pragma unroll
      for (int j = 0; j < PPT; ++j) alive |= (uint32_t)(deepest <= cell_last[j]) << j;
      const int k1 = min(k0 + 8, nb);
      for (int k = k0; k < k1; ++k) {
        uint32_t mk = 1u;
        if constexpr (!kOneCell) {
          mk = __builtin_amdgcn_readfirstlane(m_next);
          m_next = sM[min(k + 1, BS - 1)];
        }
        const int pos = end - 1 - k;
        // ... and the record's cell mask keeps it
        const uint32_t hit = cell.mine(mk) & alive;
        if (hit == 0) {
          if (lane < NC) red[wv][k][lane] = 0.0f;
          continue;
        }
        const float4 A = sA[k], B = sB[k], C = sC[k];
        const Box bx = uniform_box(C);
        float v[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = 0.0f;
        uint64_t contrib = 0;  // lanes that composited this record in some cell
        // every cell hit: one straight-line block the compiler can interleave
        if (hit == (1u << PPT) - 1u) {
#pragma unroll
          for (int j = 0; j < PPT; ++j)
            adjoint(j, sample(lx, ly, lxh, lyh, cell.X0[j], cell.Y0[j], bx, A, B), true, B, C, pos,
                    v, contrib);
        } else {
#pragma unroll
          for (int j = 0; j < PPT; ++j)
            if (hit & (1u << j))
              adjoint(j, sample(lx, ly, lxh, lyh, cell.X0[j], cell.Y0[j], bx, A, B), true, B, C,
                      pos, v, contrib);
        }
        if (contrib != 0) {
          const float r = wave_reduce10(v);
          if (lane < 16 && c_red < NC) red[wv][k][c_red] = r;
        } else if (lane < NC) {
          red[wv][k][lane] = 0.0f;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < nb) {
      const int k = threadIdx.x;
      float s[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        float a = 0.0f;
#pragma unroll
        for (int w = 0; w < NW; ++w) a += red[w][k][c];
        s[c] = a;
      }
      {
        const float4 A = sA[k], B = sB[k];
        const float sx = s[0], sy = s[1];
        s[0] = 0.5f * kQ * (2.0f * A.z * sx + A.w * sy);
        s[1] = 0.5f * kQ * (A.w * sx + 2.0f * B.x * sy);
      }
      s[2] *= -0.5f;
      s[3] = -s[3];
      s[4] *= -0.5f;
      const float4 C = sC[k];
      const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
      const int tx0 = (bx & 0xFFFF) / TW, tx1 = (bx >> 16) / TW;
      const int ty0 = (by & 0xFFFF) / TH, ty1 = (by >> 16) / TH;
      const int wc = tx1 - tx0 + 1;
      const uint32_t slot = sP[k] + kept_rank(sT[k], wc * (ty1 - ty0 + 1),
                                                    (ty - ty0) * wc + (tx - tx0));
      float2 *pp = partial + 5 * (int64_t)slot;  // ten floats, 40 B per slot
      pp[0] = make_float2(s[0], s[1]);
      pp[1] = make_float2(s[2], s[3]);
      pp[2] = make_float2(s[4], s[5]);
      pp[3] = make_float2(s[6], s[7]);
      pp[4] = make_float2(s[8], s[9]);
    }
    __syncthreads();
  }
}

// Chain the ten screen-space gradient terms s[] of one (view, Gaussian)
// record to the raw parameters: out[0..10] for mean, log-scale, quaternion
// and opacity logit; Yb[k] * graw[c] for SH coefficient k of channel c.
template <typename T>
__device__ inline void param_grads(const float *__restrict__ P, int64_t stride, int64_t i,
                                   int deg, const GeoT<T> &g, const CamD &cam, const float s[10],
                                   T out[11], T Yb[16], T graw[3]) {
  const T gu = s[0], gv = s[1], gQ00 = s[2], gQ01 = s[3], gQ11 = s[4];
  const T go = s[5], gz_depth = s[9];
  // conic Q = Sigma2^-1 -> Sigma2 entries a, b, c
  const T det = g.det, a = g.a, b = g.b, c = g.c;
  const T idet = qdiv(T(1), det);
  const T gdet = -(gQ00 * c - gQ01 * b + gQ11 * a) * (idet * idet);
  const T ga = gQ11 * idet + gdet * c;
  const T gb = -gQ01 * idet - T(2) * b * gdet;
  const T gc = gQ00 * idet + gdet * a;
  // Sigma2 = A Sigma A^T: G_Sigma = A^T G2 A, G_A = 2 G2 A Sigma
  const T G2[2][2] = {{ga, T(0.5) * gb}, {T(0.5) * gb, gc}};
  const T A[2][3] = {{g.A0[0], g.A0[1], g.A0[2]}, {g.A1[0], g.A1[1], g.A1[2]}};
  const T *Sg = g.Sig;
  const T Sig[3][3] = {{Sg[0], Sg[1], Sg[2]}, {Sg[1], Sg[3], Sg[4]}, {Sg[2], Sg[4], Sg[5]}};
  T GA[2][3], GS[3][3];
  {
    T G2A[2][3];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k) G2A[r][k] = G2[r][0] * A[0][k] + G2[r][1] * A[1][k];
    for (int r = 0; r < 2; ++r)
      for (int k = 0; k < 3; ++k)
        GA[r][k] = T(2) * (G2A[r][0] * Sig[0][k] + G2A[r][1] * Sig[1][k] + G2A[r][2] * Sig[2][k]);
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < 3; ++k) GS[r][k] = A[0][r] * G2A[0][k] + A[1][r] * G2A[1][k];
  }
  // A = J Rc -> G_J = G_A Rc^T
  T Rc[9];
  for (int k = 0; k < 9; ++k) Rc[k] = (T)cam.R[k];
  T GJ[2][3];
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k)
      GJ[r][k] = GA[r][0] * Rc[3 * k] + GA[r][1] * Rc[3 * k + 1] + GA[r][2] * Rc[3 * k + 2];
  const T iz = qdiv(T(1), g.Z), iz2 = iz * iz, iz3 = iz2 * iz;
  const T fx = (T)cam.fx, fy = (T)cam.fy, X = g.X, Y = g.Y;
  T gX = GJ[0][2] * (-fx * iz2) + gu * fx * iz;
  T gY = GJ[1][2] * (-fy * iz2) + gv * fy * iz;
  T gZ = GJ[0][0] * (-fx * iz2) + GJ[0][2] * (T(2) * fx * X * iz3) +
              GJ[1][1] * (-fy * iz2) + GJ[1][2] * (T(2) * fy * Y * iz3) +
              gu * (-fx * X * iz2) + gv * (-fy * Y * iz2) + gz_depth;
  T gmu[3];
  for (int k = 0; k < 3; ++k) gmu[k] = Rc[k] * gX + Rc[3 + k] * gY + Rc[6 + k] * gZ;
  // Sigma = M M^T, M = Rg diag(s)
  T GM[3][3];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k)
      GM[r][k] = T(2) * (GS[r][0] * g.M[k] + GS[r][1] * g.M[3 + k] + GS[r][2] * g.M[6 + k]);
  T GR[3][3], gls[3];
  for (int k = 0; k < 3; ++k) {
    T gsk = T(0);
    for (int r = 0; r < 3; ++r) {
      GR[r][k] = GM[r][k] * g.s[k];
      gsk += GM[r][k] * g.Rg[3 * r + k];
    }
    gls[k] = gsk * g.s[k];
  }
  const T w = g.qn[0], x = g.qn[1], y = g.qn[2], z = g.qn[3];
  T gqn[4];
  gqn[0] = T(2) * (-z * GR[0][1] + y * GR[0][2] + z * GR[1][0] - x * GR[1][2] - y * GR[2][0] + x * GR[2][1]);
  gqn[1] = T(2) * (y * GR[0][1] + z * GR[0][2] + y * GR[1][0] - T(2) * x * GR[1][1] - w * GR[1][2] +
                  z * GR[2][0] + w * GR[2][1] - T(2) * x * GR[2][2]);
  gqn[2] = T(2) * (-T(2) * y * GR[0][0] + x * GR[0][1] + w * GR[0][2] + x * GR[1][0] + z * GR[1][2] -
                  w * GR[2][0] + z * GR[2][1] - T(2) * y * GR[2][2]);
  gqn[3] = T(2) * (-T(2) * z * GR[0][0] - w * GR[0][1] + x * GR[0][2] + w * GR[1][0] - T(2) * z * GR[1][1] +
                  y * GR[1][2] + x * GR[2][0] + y * GR[2][1]);
  const T dq = g.qn[0] * gqn[0] + g.qn[1] * gqn[1] + g.qn[2] * gqn[2] + g.qn[3] * gqn[3];
  T gq[4];
  const T iqn = qdiv(T(1), g.qnorm);
  for (int k = 0; k < 4; ++k) gq[k] = (gqn[k] - g.qn[k] * dq) * iqn;
  const T glogit = go * g.o * (T(1) - g.o);
  // colour
  T dir[3], dn, raw[3];
  color_raw(P + 11 * stride + i, stride, deg, g, cam, dir, dn, Yb, raw);
  for (int ch = 0; ch < 3; ++ch) graw[ch] = raw[ch] > T(0) ? (T)s[6 + ch] : T(0);
  const int K = (deg + 1) * (deg + 1);
  if (deg > 0) {
    T f[16];
    f[0] = T(0);
#pragma unroll 4
    for (int k = 1; k < K; ++k) {
      T a = T(0);
      for (int ch = 0; ch < 3; ++ch) a += (T)P[(11 + 3 * k + ch) * stride + i] * graw[ch];
      f[k] = a;
    }
    T gd[3];
    sh_grad_dot(deg, dir[0], dir[1], dir[2], f, gd);
    const T dd = dir[0] * gd[0] + dir[1] * gd[1] + dir[2] * gd[2];
    const T idn = qdiv(T(1), dn);
    for (int k = 0; k < 3; ++k) gmu[k] += (gd[k] - dir[k] * dd) * idn;
  }
  out[0] = gmu[0]; out[1] = gmu[1]; out[2] = gmu[2];
  out[3] = gls[0]; out[4] = gls[1]; out[5] = gls[2];
  out[6] = gq[0]; out[7] = gq[1]; out[8] = gq[2]; out[9] = gq[3];
  out[10] = glogit;
}

// Per record (view v, Gaussian g) with a non-empty tile rect: the sum of its
// per-tile partials (only tiles whose backward reached it), written as ten
// planes s2d[c][r].  Integer box, slot base and kept-tile mask from the
// record.  A record of at most kSumBig kept tiles is summed by its own
// thread in slot order; a wavefront's larger records are then summed one at
// a time by the whole wavefront (slot s on lane s mod 64, each lane in slot
// order, then the butterfly), so one record with hundreds of tiles no longer
// holds 63 idle lanes for hundreds of steps.  Which way a record goes, and
// so its additions, depends on the record alone.
constexpr uint32_t kSumBig = 16;

__device__ __forceinline__ uint32_t lane_u32(uint32_t x, int src) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, src);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int src) {
  return (uint64_t)lane_u32((uint32_t)x, src) | ((uint64_t)lane_u32((uint32_t)(x >> 32), src) << 32);
}

__global__ void __launch_bounds__(256)
    k_sum_partials(const int64_t *__restrict__ cnt, int64_t RS, int TW, int TH, int tiles_x,
                   int tiles_per_view, const float4 *__restrict__ rec,
                   const uint32_t *__restrict__ count, const uint32_t *__restrict__ seg_off,
                   const uint64_t *__restrict__ frontier, const float2 *__restrict__ partial,
                   float *__restrict__ s2d, int zero_undrawn) {
  if (cnt[3] != 0) return;  // uniform: the window overflowed
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n = cnt[0], nr = cnt[1];
  const int lane = threadIdx.x & (kWave - 1);
  // no early exit below: every lane of a wavefront takes part in summing
  // its large records
  const bool valid = r < nr;
  const uint32_t c = valid ? count[r] : 0u;  // kept tiles: popcount(m), or n_rect beyond 64
  int tx0 = 0, ty0 = 0, wc = 1, n_rect = 0, tile_base = 0;
  uint64_t m = 0, key = 0;
  uint32_t slot = 0;
  if (c > 0) {
    const float4 C = rec[4 * r + 2], D = rec[4 * r + 3];
    const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
    tx0 = (int)(bx & 0xFFFF) / TW;
    ty0 = (int)(by & 0xFFFF) / TH;
    wc = (int)(bx >> 16) / TW - tx0 + 1;
    n_rect = wc * ((int)(by >> 16) / TH - ty0 + 1);
    m = (uint64_t)__float_as_uint(D.y) | ((uint64_t)__float_as_uint(D.z) << 32);
    tile_base = (int)(r / n) * tiles_per_view;
    slot = slot_base(seg_off, D);
    // the record's place in the depth order (depth_order_key, from C)
    key = ((uint64_t)__float_as_uint(C.y) << 32) | (uint32_t)r;
  }
  if (c <= kSumBig) {
    float s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t mm = m;
    // the kept tiles in slot order (lowest mask bit first), four at a time:
    // their frontier reads, then the partial reads of the reached ones, are
    // issued together, and the sums are taken in slot order afterwards
    for (uint32_t b = 0; b < c; b += 4) {
      int t[4];
      bool ok[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        ok[i] = b + i < c;
        int k = 0;
        if (ok[i]) {
          if (n_rect > 64) {
            k = (int)(b + i);
          } else {
            k = __builtin_ctzll(mm);
            mm &= mm - 1;
          }
        }
        t[i] = tile_base + (ty0 + k / wc) * tiles_x + tx0 + k % wc;
      }
      uint64_t f[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) f[i] = ok[i] ? frontier[t[i]] : 0;
      float2 q[4][5];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float2 *pp = partial + 5 * (int64_t)(slot + b + i);
#pragma unroll
        for (int j = 0; j < 5; ++j) q[i][j] = make_float2(0.0f, 0.0f);
        if (ok[i] && f[i] >= key) {  // that tile's backward reached the record
#pragma unroll
          for (int j = 0; j < 5; ++j) q[i][j] = pp[j];
        }
      }
      // an unreached tile adds exact zeros (s never holds -0)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          s[2 * j] += q[i][j].x;
          s[2 * j + 1] += q[i][j].y;
        }
    }
    // the projection backward reads only drawn records: an undrawn one's
    // planes are written (as zeros) only for a caller's own output buffer
    if (valid && (c > 0 || zero_undrawn)) {
#pragma unroll
      for (int j = 0; j < 10; ++j) s2d[j * RS + r] = s[j];
    }
  }
  const int c_red = bitrev4(lane & 15);  // the value a reduction leaves in this lane
  for (uint64_t big = __ballot(c > kSumBig); big != 0; big &= big - 1) {
    const int src = __builtin_ctzll(big);
    const uint32_t bc = lane_u32(c, src), bslot = lane_u32(slot, src);
    const int btx0 = (int)lane_u32((uint32_t)tx0, src), bty0 = (int)lane_u32((uint32_t)ty0, src);
    const int bwc = (int)lane_u32((uint32_t)wc, src), bn_rect = (int)lane_u32((uint32_t)n_rect, src);
    const int btile_base = (int)lane_u32((uint32_t)tile_base, src);
    const uint64_t bm = lane_u64(m, src), bkey = lane_u64(key, src);
    const int64_t br = (int64_t)lane_u64((uint64_t)r, src);
    float v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = 0.0f;
    for (uint32_t sl = (uint32_t)lane; sl < bc; sl += kWave) {
      const int k = bn_rect > 64 ? (int)sl : nth_set_bit(bm, (int)sl);
      const int t = btile_base + (bty0 + k / bwc) * tiles_x + btx0 + k % bwc;
      if (frontier[t] >= bkey) {
        const float2 *pp = partial + 5 * (int64_t)(bslot + sl);
#pragma unroll
        for (int j = 0; j < 5; ++j) {
          const float2 q = pp[j];
          v[2 * j] += q.x;
          v[2 * j + 1] += q.y;
        }
      }
    }
    const float sum = wave_reduce10(v);
    if (lane < 16 && c_red < 10) s2d[c_red * RS + br] = sum;
  }
}

// Projection backward over all views: one thread per Gaussian; record
// r = v n + g of every view that drew it contributes, in view order, with
// float32 accumulation (the same additions as one single-view backward per
// view accumulating into the gradient buffer).  The eleven geometry rows
// accumulate in registers, the 3 (DEG+1)^2 SH rows in this thread's LDS
// column (one global write per row instead of a read-modify-write per
// view).
template <int DEG>
__global__ void __launch_bounds__(256)
    k_preprocess_bwd(const float *__restrict__ P, const int64_t *__restrict__ cnt,
                     int64_t stride, const CamD *__restrict__ cams, int V,
                     const uint32_t *__restrict__ count, const float *__restrict__ s2d,
                     int64_t RS, float *__restrict__ grad, int64_t gstride, int accumulate) {
  constexpr int K = (DEG + 1) * (DEG + 1), R = 11 + 3 * K;
  __shared__ float sh[3 * K][256];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + t;
  const int64_t n = cnt[0];
  if (i >= n || cnt[3] != 0) return;
  float acc[11];
#pragma unroll
  for (int r = 0; r < 11; ++r) acc[r] = accumulate ? grad[r * gstride + i] : 0.0f;
  bool sh_written = accumulate != 0;
  if (accumulate)
    for (int r = 0; r < 3 * K; ++r) sh[r][t] = grad[(int64_t)(11 + r) * gstride + i];
  GeoT<float> g;
  load_gauss(P, stride, i, g);  // camera-independent: once for all views
  unsigned drawn = 0;  // views that drew the Gaussian (independent loads, issued together)
  for (int v = 0; v < V; ++v) drawn |= (count[v * n + i] != 0 ? 1u : 0u) << v;
  for (int v = 0; v < V; ++v) {
    const int64_t rr = v * n + i;
    if (!((drawn >> v) & 1u)) continue;
    const CamD &cam = cams[v];
    project(cam, g, false);  // drawn by the forward: no culling decisions
    float s[10];
#pragma unroll
    for (int c = 0; c < 10; ++c) s[c] = s2d[c * RS + rr];
    float out[11], Yb[16], graw[3];
    param_grads(P, stride, i, DEG, g, cam, s, out, Yb, graw);
#pragma unroll
    for (int r = 0; r < 11; ++r) acc[r] += out[r];
#pragma unroll 1
    for (int k = 0; k < K; ++k)
      for (int ch = 0; ch < 3; ++ch) {
        const float val = Yb[k] * graw[ch];
        float &a = sh[3 * k + ch][t];
        a = sh_written ? a + val : 0.0f + val;
      }
    sh_written = true;
  }
#pragma unroll
  for (int r = 0; r < 11; ++r) grad[r * gstride + i] = acc[r];
  for (int r = 11; r < R; ++r) grad[r * gstride + i] = sh_written ? sh[r - 11][t] : 0.0f;
}

// ---- work measurement (outside the hot path) ----
// Per tile: the list positions each pixel's compositing walks (start to its
// last contributor) and how many of them have the pixel inside the record's
// box.  out[2 * tile] / out[2 * tile + 1].
__global__ void __launch_bounds__(256)
    k_work(const uint64_t *__restrict__ pairs, const int2 *__restrict__ ranges,
           const float4 *__restrict__ rec, int W, int H, int TW, int TH, int tiles_x,
           int tiles_per_view, const int *__restrict__ last, long long *__restrict__ out) {
  __shared__ unsigned long long s_walk, s_in;
  const int gt = blockIdx.x;
  const int view = gt / tiles_per_view, tile = gt - view * tiles_per_view;
  const int tx = tile % tiles_x, ty = tile / tiles_x;
  const int2 rg = ranges[gt];
  if (threadIdx.x == 0) s_walk = s_in = 0;
  __syncthreads();
  unsigned long long walk = 0, inbox = 0;
  for (int t = threadIdx.x; t < TW * TH; t += blockDim.x) {
    const int px = tx * TW + t % TW, py = ty * TH + t / TW;
    if (px >= W || py >= H) continue;
    const int l = last[(int64_t)view * W * H + (int64_t)py * W + px];
    if (l < rg.x) continue;
    walk += (unsigned long long)(l - rg.x + 1);
    for (int p = rg.x; p <= l; ++p) {
      const float4 C = rec[4 * (int64_t)(uint32_t)pairs[p] + 2];
      const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
      inbox += (px >= (int)(bx & 0xFFFF) && px <= (int)(bx >> 16) && py >= (int)(by & 0xFFFF) &&
                py <= (int)(by >> 16));
    }
  }
  atomicAdd(&s_walk, walk);
  atomicAdd(&s_in, inbox);
  __syncthreads();
  if (threadIdx.x == 0) {
    out[2 * gt] = (long long)s_walk;
    out[2 * gt + 1] = (long long)s_in;
  }
}

// ---- export helpers (tests) ----
__global__ void k_export_keys(const uint64_t *__restrict__ pairs, int64_t P,
                              const uint32_t *__restrict__ zkey, uint64_t *__restrict__ keys,
                              int32_t *__restrict__ values) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= P) return;
  const uint64_t p = pairs[k];
  const uint32_t g = (uint32_t)p;
  if (keys) keys[k] = (p & 0xFFFFFFFF00000000ull) | zkey[g];
  if (values) values[k] = (int32_t)g;
}

__global__ void k_export_rec(const float4 *__restrict__ rec, int64_t RS,
                             const uint32_t *__restrict__ count, int64_t n,
                             float *__restrict__ out, int32_t *__restrict__ box) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const bool cul = count[i] == 0;  // a culled record is never written
  const float4 z = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  const float4 A = cul ? z : rec[4 * i], B = cul ? z : rec[4 * i + 1],
               C = cul ? z : rec[4 * i + 2];
  const uint32_t bx = __float_as_uint(C.z), by = __float_as_uint(C.w);
  const int i0 = bx & 0xFFFF, j0 = by & 0xFFFF;
  if (out) {
    out[0 * n + i] = cul ? 0.0f : A.x + (float)i0;
    out[1 * n + i] = cul ? 0.0f : A.y + (float)j0;
    out[2 * n + i] = A.z * kQ;         // the conic Q00, Q01, Q11
    out[3 * n + i] = A.w * (0.5f * kQ);
    out[4 * n + i] = B.x * kQ;
    out[5 * n + i] = B.y;
    out[6 * n + i] = B.z;
    out[7 * n + i] = B.w;
    out[8 * n + i] = C.x;
    out[9 * n + i] = C.y;
  }
  if (box) {
    box[0 * n + i] = i0;
    box[1 * n + i] = (int)(bx >> 16);
    box[2 * n + i] = j0;
    box[3 * n + i] = (int)(by >> 16);
  }
}

__global__ void k_copy_u32_as_i32(const uint32_t *__restrict__ a, int64_t n, int32_t *__restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int32_t)a[i];
}

inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// Workgroups of a raster launch over nt tiles (a multiple of the 8 XCDs).
inline int raster_grid(int nt) { return 8 * ((nt + 7) / 8); }

int64_t *counters(dcgs_state *s, hipStream_t st);

__global__ void k_fill_i64(int64_t *__restrict__ a, int64_t n, int64_t v) {
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) a[i] = v;
}

template <int TW, int TH, int PPT>
void launch_fwd_t(dcgs_state *s, hipStream_t st, float *rgb, float *depth, float *T) {
  const int nt = s->tiles_x * s->tiles_y * s->V;
  const unsigned grid = (unsigned)raster_grid(nt), wgrid = (unsigned)s->fcap;
  const int64_t *cnt = counters(s, st);
  // segments of the longest lists first (products, then compositing), the
  // whole-list tiles, then the split tiles' totals
#define DCGS_FWD_PASS(P, G)                                                                        \
  hipLaunchKernelGGL((k_raster_fwd<TW, TH, PPT, P>), dim3(G), dim3(TW * TH / PPT), 0, st,          \
                     s->pairs.p, s->ranges.p, s->torder.p, s->rec.p, s->rs, s->W, s->H, s->tiles_x, \
                     nt, s->tiles_x * s->tiles_y, s->bg[0], s->bg[1], s->bg[2], rgb, depth, T,      \
                     s->T_final.p, s->last.p, s->bslot.p, s->bound.p, s->witem.p, cnt, s->fseg.p); \
  DCGS_LAUNCH_CHECK()
  DCGS_FWD_PASS(1, wgrid);
  DCGS_FWD_PASS(2, wgrid);
  DCGS_FWD_PASS(0, grid);
#undef DCGS_FWD_PASS
  hipLaunchKernelGGL((k_fwd_combine<TW, TH>), dim3(wgrid), dim3(TW * TH), 0, st, s->ranges.p,
                     s->witem.p, cnt, s->bslot.p, s->W, s->H, s->tiles_x, s->tiles_x * s->tiles_y,
                     s->bg[0], s->bg[1], s->bg[2], rgb, depth, T, s->T_final.p, s->last.p,
                     s->bound.p, s->fseg.p);
  DCGS_LAUNCH_CHECK();
}

template <int TW, int TH, int PPT>
void launch_bwd_t(dcgs_state *s, hipStream_t st, const float *dl_drgb, const float *dl_ddepth) {
  const int nt = s->tiles_x * s->tiles_y * s->V;
  // one workgroup per work item (tile segment); the grid is sized for the
  // most the pair capacity allows, the count is read on the device
  const unsigned grid = (unsigned)raster_grid((int)s->wcap);
  hipLaunchKernelGGL((k_raster_bwd<TW, TH, PPT>), dim3(grid), dim3(TW * TH / PPT), 0, st,
                     s->pairs.p, s->ranges.p, s->witem.p, counters(s, st), s->rec.p, s->rs, s->W,
                     s->H, s->tiles_x, nt, s->tiles_x * s->tiles_y, s->bg[0], s->bg[1], s->bg[2],
                     s->T_final.p, s->last.p, dl_drgb, dl_ddepth, s->partial.p, s->frontier.p,
                     s->bslot.p, s->bound.p, s->seg_off.p);
  DCGS_LAUNCH_CHECK();
}

// Raster shapes: tile width x height and pixels per lane.
#define DCGS_RASTER_SHAPES(X) \
  X(16, 16, 1) X(16, 16, 2) X(16, 16, 4) X(8, 8, 1) X(32, 16, 2) X(32, 16, 4) X(32, 16, 8)

void launch_fwd(dcgs_state *s, hipStream_t st, float *rgb, float *depth, float *T) {
#define X(a, b, c)                                                   \
  if (s->TW == a && s->TH == b && s->ppt == c) {                     \
    launch_fwd_t<a, b, c>(s, st, rgb, depth, T);                     \
    return;                                                          \
  }
  DCGS_RASTER_SHAPES(X)
#undef X
  throw Error{DCGS_E_INVALID, "unsupported raster shape"};
}

void launch_bwd(dcgs_state *s, hipStream_t st, const float *dl_drgb, const float *dl_ddepth) {
#define X(a, b, c)                                                   \
  if (s->TW == a && s->TH == b && s->ppt_bwd == c) {                     \
    launch_bwd_t<a, b, c>(s, st, dl_drgb, dl_ddepth);                \
    return;                                                          \
  }
  DCGS_RASTER_SHAPES(X)
#undef X
  throw Error{DCGS_E_INVALID, "unsupported raster shape"};
}

// Camera constants and the two host-known counts (n, nr) travel to the
// device in one copy from pinned staging: [CamD x kMaxViews][int64 x 2].
// On the device the block continues with the counters the kernels write:
// [n, nr, pairs, overflow, sticky overflow, unused x 3].
constexpr size_t kCamBytes = kMaxViews * sizeof(CamD);
constexpr size_t kStageBytes = kCamBytes + 2 * sizeof(int64_t);
constexpr size_t kDevBytes = kCamBytes + 8 * sizeof(int64_t);

void stage_cams(const dcgs_state *s, void *pinned, int64_t n) {
  CamD *hc = (CamD *)pinned;
  for (int v = 0; v < s->V; ++v) hc[v] = make_cam(s->cams[v]);
  int64_t *c = (int64_t *)((char *)pinned + kCamBytes);
  c[0] = n;
  c[1] = n * s->V;
}

// Device block of a state (cameras, then counters); allocated once, the
// counters zeroed then.
int64_t *counters(dcgs_state *s, hipStream_t st) {
  if (!s->cam_dev.p) {
    s->cam_dev.need(kDevBytes);
    hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st,
                       (int64_t *)(s->cam_dev.p + kCamBytes), (int64_t)8, (int64_t)0);
    DCGS_LAUNCH_CHECK();
  }
  return (int64_t *)(s->cam_dev.p + kCamBytes);
}

// Buffers for records of n_grid Gaussians (record planes RS = n_grid * V
// apart) and tile/pixel state.  No allocation happens when they are large
// enough already.
void size_buffers(dcgs_state *s, int64_t n_grid) {
  const int V = s->V;
  const int nt = s->tiles_x * s->tiles_y * V;
  const int64_t nr = n_grid * V;
  const int64_t HW = (int64_t)s->W * s->H;
  s->rs = nr;
  s->rec.need(4 * (size_t)nr + 1);
  s->zkey.need(nr + 1);
  s->count.need(nr + 1);
  s->order.need(nr + 1);
  s->key_tmp.need(2 * (size_t)nr + 2);
  s->val_tmp.need(nr + 1);
  s->seg_tot.need((size_t)V * blocks_for(n_grid, kPrepThreads) + 1);
  s->seg_off.need((size_t)V * blocks_for(n_grid, kPrepThreads) + 2);
  s->tmask.need(nr + 1);
  s->scan.need(nr + 2);
  s->ranges.need(nt + 1);
  s->frontier.need(nt + 1);
  s->torder.need(4 * (size_t)raster_grid(nt) + 4);  // keys, order, and their sort buffers
  const size_t gs = (size_t)raster_grid(nt) + 2;
  s->segc.need(2 * gs);
  s->segs.need(2 * gs);
  s->segpart.need(2 * (scan_part_size(raster_grid(nt)) + 2));
  s->bslot.need(nt + 1);
  s->T_final.need(V * HW + 1);
  s->last.need(V * HW + 1);
  s->scan_part.need(scan_part_size(nr) + 2);
  s->count_part.need(nr / 256 + 2);
}

// Projection, depth order and pair count for a grid of n_grid Gaussians
// (the device counter holds the real n <= n_grid).
void enqueue_front(dcgs_state *s, const float *params, int64_t n_grid, int64_t stride,
                   const uint16_t *gmask, int mask_shift, int64_t pcap, hipStream_t st) {
  dcgs_ctx *ctx = s->ctx;
  const int V = s->V;
  const int64_t RS = s->rs, nr = n_grid * V;
  int64_t *cnt = counters(s, st);
  const CamD *dc = (const CamD *)s->cam_dev.p;
  uint32_t *sortkey = s->key_tmp.p, *order = s->order.p;
  if (n_grid > 0) {
    StageTimer tp(ctx, DCGS_STAGE_PREPROCESS, st);
    hipLaunchKernelGGL(k_preprocess, dim3(blocks_for(n_grid, kPrepThreads)), dim3(kPrepThreads),
                       0, st, params,
                       cnt, stride, s->sh_degree, dc, V, gmask, mask_shift, s->TW, s->TH,
                       s->rec.p, RS, s->zkey.p, sortkey, order, s->count.p, s->tmask.p,
                       s->seg_tot.p);
    DCGS_LAUNCH_CHECK();
  }
  if (nr > 0) {
    StageTimer ts(ctx, DCGS_STAGE_DEPTH_SORT, st);
    // depth order of all records: stable sort of the float32 depth bits
    sort_u32_pairs(sortkey, order, sortkey + RS + 1, s->val_tmp.p, nr, 32, s->hist, st,
                   cnt + 1);
    hipLaunchKernelGGL(k_depth_counts, dim3(blocks_for(nr, kCountThreads)), dim3(kCountThreads),
                       0, st, order, s->count.p, cnt, sortkey + RS + 1, s->count_part.p);
    DCGS_LAUNCH_CHECK();
  }
  StageTimer te(ctx, DCGS_STAGE_SCAN_EMIT, st);
  // the depth sort's second key buffer holds the counts in depth order now
  scan_u32(sortkey + RS + 1, nullptr, s->scan.p, nr, s->scan_part.p, st, cnt + 1);
  hipLaunchKernelGGL(k_pairs_total, dim3(1), dim3(kTotalThreads), 0, st, s->count_part.p, cnt,
                     pcap);
  DCGS_LAUNCH_CHECK();
  // gradient slot bases of the projection's segments
  if (n_grid > 0)
    scan_u32(s->seg_tot.p, nullptr, s->seg_off.p, (int64_t)V * blocks_for(n_grid, kPrepThreads),
             s->scan_part.p, st);
}

// Pair emission, tile sort, ranges and the forward raster for pcap pair
// slots (the device counter holds the real count).
void enqueue_back(dcgs_state *s, int64_t n_grid, int64_t pcap, hipStream_t st, float *rgb,
                  float *depth, float *T) {
  dcgs_ctx *ctx = s->ctx;
  const int V = s->V;
  const int tpv = s->tiles_x * s->tiles_y;
  const int nt = tpv * V;
  const int64_t nr = n_grid * V;
  int64_t *cnt = counters(s, st);
  if (nr > 0) {
    StageTimer te(ctx, DCGS_STAGE_SCAN_EMIT, st);
    hipLaunchKernelGGL(k_emit, dim3(blocks_for(nr, kEmitThreads)), dim3(kEmitThreads), 0, st,
                       s->order.p, s->key_tmp.p + s->rs + 1, s->scan.p, s->rec.p, s->tmask.p,
                       cnt, s->TW, s->TH, s->tiles_x, tpv, s->pairs.p);
    DCGS_LAUNCH_CHECK();
  }
  int tile_bits = 0;
  while ((1 << tile_bits) < nt) ++tile_bits;
  if (pcap > 0) {
    StageTimer tt(ctx, DCGS_STAGE_TILE_SORT, st);
    sort_u64_bits(s->pairs.p, s->pairs_tmp.p, pcap, 32, tile_bits, s->hist, st, cnt + 2);
  }
  {
    StageTimer tr(ctx, DCGS_STAGE_RANGES, st);
    hipLaunchKernelGGL(k_ranges, dim3(blocks_for(nt, 256)), dim3(256), 0, st, s->pairs.p, cnt,
                       nt, s->ranges.p);
    DCGS_LAUNCH_CHECK();
    // the raster launch order, longest lists first
    const int grid = raster_grid(nt);
    uint32_t *key = s->torder.p + grid, *ktmp = key + grid, *vtmp = ktmp + grid;
    hipLaunchKernelGGL(k_order_keys, dim3(blocks_for(grid, 256)), dim3(256), 0, st, s->ranges.p,
                       cnt, nt, grid, seg_len(s->TW, s->TH), key, s->torder.p);
    DCGS_LAUNCH_CHECK();
    sort_u32_pairs(key, s->torder.p, ktmp, vtmp, grid, kOrderBits, s->hist, st);
    // the backward's work list: long lists split into segments, in launch order
    uint32_t *cw = s->segc.p, *cb = cw + grid + 2, *sw = s->segs.p, *sb = sw + grid + 2;
    hipLaunchKernelGGL(k_seg_count, dim3(blocks_for(grid, 256)), dim3(256), 0, st, s->torder.p,
                       s->ranges.p, nt, grid, seg_len(s->TW, s->TH), cw, cb);
    DCGS_LAUNCH_CHECK();
    scan_u32(cw, nullptr, sw, grid, s->segpart.p, st);
    scan_u32(cb, nullptr, sb, grid, s->segpart.p + scan_part_size(grid) + 2, st);
    hipLaunchKernelGGL(k_seg_fill, dim3(blocks_for(grid, 256)), dim3(256), 0, st, s->torder.p,
                       s->ranges.p, nt, grid, seg_len(s->TW, s->TH), cw, sw, cb, sb, s->witem.p,
                       s->bslot.p, cnt);
    DCGS_LAUNCH_CHECK();
  }
  StageTimer tf(ctx, DCGS_STAGE_RASTER_FWD, st);
  launch_fwd(s, st, rgb, depth, T);
}

void size_pairs(dcgs_state *s, int64_t pcap) {
  s->pairs.need((size_t)pcap + 1);
  s->pairs_tmp.need((size_t)pcap + 1);
  s->partial.need(5 * (size_t)pcap + 5);
  // a split tile has more than S pairs: at most pcap / S extra work
  // items, and at most 2 pcap / S boundary states
  const int64_t nt = (int64_t)s->tiles_x * s->tiles_y * s->V;
  const int64_t S = seg_len(s->TW, s->TH);
  s->wcap = nt + pcap / S + 1;
  s->fcap = std::min(s->wcap, kFwdSplit * pcap / ((kFwdSplit - 1) * S) + 1);
  s->witem.need((size_t)s->wcap + 8);
  s->bound.need((size_t)(2 * (pcap / S) + 1) * kStateVals * s->TW * s->TH);
  s->fseg.need((size_t)(2 * (pcap / S) + 1) * kFsegVals * s->TW * s->TH);
}

}  // namespace

void render_forward(dcgs_state *s, const float *params, int64_t n, int64_t stride,
                    const uint16_t *gmask, int mask_shift, hipStream_t st, float *rgb,
                    float *depth, float *T) {
  s->fwd_ok = false;
  s->n = n;
  s->n_grid = n;
  size_buffers(s, n);
  int64_t *cnt = counters(s, st);
  // cameras and counts -> device (the pinned staging copy is complete:
  // every forward synchronises its stream before returning)
  if (!s->cam_pinned) DCGS_HIP(hipHostMalloc(&s->cam_pinned, kStageBytes, hipHostMallocDefault));
  stage_cams(s, s->cam_pinned, n);
  DCGS_HIP(hipMemcpyAsync(s->cam_dev.p, s->cam_pinned, kStageBytes, hipMemcpyHostToDevice, st));
  // an eager forward starts clean: no overflow carried over from the last one
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(64), 0, st, cnt + 3, (int64_t)2, (int64_t)0);
  DCGS_LAUNCH_CHECK();
  // no pair capacity here (the pair buffers are sized after the count),
  // only the 2^31 - 1 limit of 32-bit pair indexing
  enqueue_front(s, params, n, stride, gmask, mask_shift, INT64_MAX, st);
  int64_t c23[2] = {0, 0};
  DCGS_HIP(hipMemcpyAsync(c23, cnt + 2, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  if (c23[1] != 0) {
    s->n_pairs = 0;
    throw Error{DCGS_E_CAPACITY, "render_fwd: " + std::to_string(c23[1]) +
                                     " (tile, Gaussian) pairs exceed the limit of 2^31 - 1"};
  }
  const int64_t total = c23[0];
  s->n_pairs = total;
  size_pairs(s, total);
  enqueue_back(s, n, total, st, rgb, depth, T);
  s->fwd_ok = true;
}

void render_plan(dcgs_state *s, int64_t n_cap, int64_t pcap) {
  s->n_grid = n_cap;
  s->pcap = pcap;
  size_buffers(s, n_cap);
  size_pairs(s, pcap);
  const int nt = s->tiles_x * s->tiles_y * s->V;
  s->hist.need(radix_scratch(std::max({s->rs, pcap, (int64_t)raster_grid(nt)})));
}

bool raster_shape_supported(int tw, int th, int ppt) {
#define X(a, b, c) \
  if (tw == a && th == b && ppt == c) return true;
  DCGS_RASTER_SHAPES(X)
#undef X
  return false;
}

size_t render_stage_bytes() { return kStageBytes; }

void render_stage(const dcgs_state *s, void *pinned, int64_t n) { stage_cams(s, pinned, n); }

void render_forward_planned(dcgs_state *s, const float *params, int64_t stride,
                            const uint16_t *gmask, hipStream_t st, float *rgb, float *depth,
                            float *T) {
  enqueue_front(s, params, s->n_grid, stride, gmask, 0, s->pcap, st);
  enqueue_back(s, s->n_grid, s->pcap, st, rgb, depth, T);
  s->fwd_ok = true;
}

int64_t *render_counters(dcgs_state *s, hipStream_t st) { return counters(s, st); }

void render_backward(dcgs_state *s, const float *params, int64_t n, int64_t stride,
                     const float *dl_drgb, const float *dl_ddepth, float *grad,
                     int64_t grad_stride, int accumulate, float *grad2d, hipStream_t st) {
  (void)n;
  {
    StageTimer tb(s->ctx, DCGS_STAGE_RASTER_BWD, st);
    launch_bwd(s, st, dl_drgb, dl_ddepth);
  }
  const int64_t n_grid = s->n_grid;
  if (n_grid > 0) {
    StageTimer tp(s->ctx, DCGS_STAGE_PREPROCESS_BWD, st);
    const CamD *dc = (const CamD *)s->cam_dev.p;
    const int tpv = s->tiles_x * s->tiles_y;
    const int64_t nr = n_grid * s->V;
    float *s2d = grad2d ? grad2d : s->grad2d.need(10 * (size_t)s->rs + 1);
    int64_t *cnt = counters(s, st);
    hipLaunchKernelGGL(k_sum_partials, dim3(blocks_for(nr, 256)), dim3(256), 0, st, cnt,
                       s->rs, s->TW, s->TH, s->tiles_x, tpv, s->rec.p, s->count.p,
                       s->seg_off.p, s->frontier.p, s->partial.p, s2d,
                       grad2d ? 1 : 0);
    DCGS_LAUNCH_CHECK();
#define DCGS_PBWD(D)                                                                        \
  hipLaunchKernelGGL(k_preprocess_bwd<D>, dim3(blocks_for(n_grid, 256)), dim3(256), 0, st,   \
                     params, cnt, stride, dc, s->V, s->count.p, s2d, s->rs, grad,            \
                     grad_stride, accumulate)
    switch (s->sh_degree) {
      case 0: DCGS_PBWD(0); break;
      case 1: DCGS_PBWD(1); break;
      case 2: DCGS_PBWD(2); break;
      default: DCGS_PBWD(3); break;
    }
#undef DCGS_PBWD
    DCGS_LAUNCH_CHECK();
  }
}

void state_work(const dcgs_state *s, int64_t *walk, int64_t *inbox, hipStream_t st) {
  const int tpv = s->tiles_x * s->tiles_y, nt = tpv * s->V;
  DCGS_CHECK(nt > 0 && s->ranges.p && s->last.p, DCGS_E_INVALID, "state_work: no forward");
  long long *d = nullptr;
  DCGS_HIP(hipMalloc(&d, 2 * (size_t)nt * sizeof(long long)));
  struct Free {
    void *p;
    ~Free() { (void)hipFree(p); }
  } fr{d};
  hipLaunchKernelGGL(k_work, dim3(nt), dim3(256), 0, st, s->pairs.p, s->ranges.p,
                     s->rec.p, s->W, s->H, s->TW, s->TH, s->tiles_x, tpv, s->last.p,
                     d);
  DCGS_LAUNCH_CHECK();
  std::vector<long long> h(2 * (size_t)nt);
  DCGS_HIP(hipMemcpyAsync(h.data(), d, h.size() * sizeof(long long), hipMemcpyDeviceToHost, st));
  DCGS_HIP(hipStreamSynchronize(st));
  int64_t a = 0, b = 0;
  for (int t = 0; t < nt; ++t) {
    a += h[2 * t];
    b += h[2 * t + 1];
  }
  *walk = a;
  *inbox = b;
}

void export_state(const dcgs_state *s, uint64_t *keys, int32_t *values, int32_t *ranges,
                  int32_t *counts, float *records, int32_t *box, int32_t *last,
                  hipStream_t st) {
  const int64_t P = s->n_pairs, nr = s->n * s->V;
  const int nt = s->tiles_x * s->tiles_y * s->V;
  if ((keys || values) && P > 0) {
    hipLaunchKernelGGL(k_export_keys, dim3(blocks_for(P, 256)), dim3(256), 0, st, s->pairs.p,
                       P, s->zkey.p, keys, values);
    DCGS_LAUNCH_CHECK();
  }
  if (ranges && nt > 0)
    DCGS_HIP(hipMemcpyAsync(ranges, s->ranges.p, nt * sizeof(int2), hipMemcpyDeviceToDevice, st));
  if (counts && nr > 0) {
    hipLaunchKernelGGL(k_copy_u32_as_i32, dim3(blocks_for(nr, 256)), dim3(256), 0, st,
                       s->count.p, nr, counts);
    DCGS_LAUNCH_CHECK();
  }
  if ((records || box) && nr > 0) {
    hipLaunchKernelGGL(k_export_rec, dim3(blocks_for(nr, 256)), dim3(256), 0, st, s->rec.p,
                       s->rs, s->count.p, nr, records, box);
    DCGS_LAUNCH_CHECK();
  }
  if (last)
    DCGS_HIP(hipMemcpyAsync(last, s->last.p, (size_t)s->V * s->W * s->H * sizeof(int),
                            hipMemcpyDeviceToDevice, st));
}

}  // namespace dcgs
