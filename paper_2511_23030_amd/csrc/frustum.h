// Exact box-frustum intersection test (Sec. III-D "Frustum Culling"),
// shared by chunk selection and the prefetch labels.  A chunk's closed cell
// box and the camera's near/far-clipped view frustum (image sides at pixel
// 0 and W/H) are both convex; they are disjoint exactly when one of 26
// candidate axes separates their projections (separating axis theorem).
// All geometry in float64.
#pragma once

#include "internal.h"

namespace dcgs {
namespace frustum {

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
__device__ inline void make_axis(const Cam &c, int ax, double out[3]) {
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

// Interval of the frustum's eight corners on every candidate axis.
__device__ inline void build_axes(const Cam &c, int ax, ViewAxes &va) {
  double a[3];
  make_axis(c, ax, a);
  double lo = 1e300, hi = -1e300;
  for (int k = 0; k < 8; ++k) {
    double P[3];
    corner(c, k, P);
    double d = a[0] * P[0] + a[1] * P[1] + a[2] * P[2];
    lo = fmin(lo, d);
    hi = fmax(hi, d);
  }
  va.a[ax][0] = a[0];
  va.a[ax][1] = a[1];
  va.a[ax][2] = a[2];
  va.lo[ax] = lo;
  va.hi[ax] = hi;
}

// True when the cube with centre cc and half side h meets the frustum.
__device__ inline bool box_meets(const ViewAxes &va, const double cc[3], double h) {
  for (int ax = 0; ax < kAxes; ++ax) {
    const double *a = va.a[ax];
    double c = a[0] * cc[0] + a[1] * cc[1] + a[2] * cc[2];
    double r = h * (fabs(a[0]) + fabs(a[1]) + fabs(a[2]));
    if ((c + r < va.lo[ax]) || (c - r > va.hi[ax])) return false;
  }
  return true;
}

inline Cam to_cam(const dcgs_camera &in) {
  Cam c{};
  for (int j = 0; j < 9; ++j) c.R[j] = in.R[j];
  for (int j = 0; j < 3; ++j) c.t[j] = in.t[j];
  c.fx = in.fx;
  c.fy = in.fy;
  c.cx = in.cx;
  c.cy = in.cy;
  c.W = in.width;
  c.H = in.height;
  c.zn = in.z_near;
  c.zf = in.z_far;
  return c;
}

}  // namespace frustum
}  // namespace dcgs
