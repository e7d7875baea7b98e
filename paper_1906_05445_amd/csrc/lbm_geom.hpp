// lbm_geom.hpp -- solid geometry on the device: position at time t, node
// classification, link fraction q (Sec. 2.2, Fig. 1), wall velocity.
//
// Classification and q must agree bit for bit with an FP64 evaluation of the
// same definitions on any IEEE machine, so every function here is compiled
// without floating-point contraction and sums components in x, y, z order.
#pragma once

#include "lbm_internal.hpp"

namespace lbm {

enum { K_SPHERE = 0, K_CYLINDER = 1, K_PLANE = 2 };

struct Box3 {
  int nx, ny, nz, D;
};

__device__ inline int box_dim(const Box3 &b, int a) { return a == 0 ? b.nx : (a == 1 ? b.ny : b.nz); }

// Centre at time t: c0 + (t - tref) U, wrapped into [0, L).  Prescribed
// motion has tref = 0 (the centre is never accumulated); a free solid's c0 is
// its centre at tref.
__device__ inline double centre_at(const DevSolid &s, int a, int64_t t, const Box3 &b) {
#pragma clang fp contract(off)
  if (!s.moving) return s.c0[a];
  const double L = (double)box_dim(b, a);
  double y = s.c0[a] + (double)(t - s.tref) * s.U[a];
  if (y >= 0.0 && y < L) return y;  // fmod(y, L) is exactly y here; skip the costly call
  y = fmod(y, L);
  if (y < 0.0) y = y + L;
  return y;
}

// Shortest periodic image of a separation along an axis of length L.
__device__ inline double min_image(double d, int L) {
#pragma clang fp contract(off)
  const double h = 0.5 * (double)L;
  if (d > h) return d - (double)L;
  if (d < -h) return d + (double)L;
  return d;
}

// Separation of point p from the solid's centre (cylinder: axial part dropped).
__device__ inline void separation(const DevSolid &s, const double c[3], double px, double py, double pz,
                                  const Box3 &b, double d[3]) {
#pragma clang fp contract(off)
  d[0] = min_image(px - c[0], b.nx);
  d[1] = min_image(py - c[1], b.ny);
  d[2] = b.D == 2 ? 0.0 : min_image(pz - c[2], b.nz);
  if (s.kind == K_CYLINDER) d[s.ax] = 0.0;
}

// Node inside solid s (inverted solids: outside the surface).
__device__ inline bool inside_solid(const DevSolid &s, const double c[3], int x, int y, int z, const Box3 &b) {
#pragma clang fp contract(off)
  bool in;
  if (s.kind == K_PLANE) {
    const double p = s.ax == 0 ? (double)x : (s.ax == 1 ? (double)y : (double)z);
    in = (double)s.sgn * (p - c[s.ax]) <= 0.0;
  } else {
    double d[3];
    separation(s, c, (double)x, (double)y, (double)z, b, d);
    double r2 = d[0] * d[0];
    r2 = r2 + d[1] * d[1];
    r2 = r2 + d[2] * d[2];
    in = r2 <= s.R * s.R;
  }
  return s.inverted ? !in : in;
}

// Node within distance w of the surface of a sphere or cylinder (planes:
// always).  Used to skip nodes that can neither change classification nor
// carry a boundary link; w carries a generous margin, so rounding here never
// drops a node that the exact tests above would keep.
__device__ inline bool near_surface(const DevSolid &s, const double c[3], int x, int y, int z, const Box3 &b,
                                    double w) {
  if (s.kind == K_PLANE) return true;
  double d[3];
  separation(s, c, (double)x, (double)y, (double)z, b, d);
  const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  const double hi = s.R + w, lo = s.R - w;
  return r2 <= hi * hi && (lo <= 0.0 || r2 >= lo * lo);
}

// Fraction q in (0, 1] of the segment from fluid node (x,y,z) along e_ibar
// (towards the solid node) where it crosses the surface of s.
__device__ inline double link_fraction(const DevSolid &s, const double c[3], int x, int y, int z, int eix,
                                       int eiy, int eiz, const Box3 &b) {
#pragma clang fp contract(off)
  double e[3] = {(double)-eix, (double)-eiy, (double)-eiz};
  double t;
  if (s.kind == K_PLANE) {
    const double p = s.ax == 0 ? (double)x : (s.ax == 1 ? (double)y : (double)z);
    const double dist = (double)s.sgn * (p - c[s.ax]);
    t = dist / (-(double)s.sgn * e[s.ax]);
  } else {
    double d[3];
    separation(s, c, (double)x, (double)y, (double)z, b, d);
    if (s.kind == K_CYLINDER) e[s.ax] = 0.0;
    if (b.D == 2) e[2] = 0.0;
    double a2 = e[0] * e[0];
    a2 = a2 + e[1] * e[1];
    a2 = a2 + e[2] * e[2];
    double bb = d[0] * e[0];
    bb = bb + d[1] * e[1];
    bb = bb + d[2] * e[2];
    double dd = d[0] * d[0];
    dd = dd + d[1] * d[1];
    dd = dd + d[2] * d[2];
    const double cc = dd - s.R * s.R;
    double disc = bb * bb - a2 * cc;
    if (disc < 0.0) disc = 0.0;
    const double sq = sqrt(disc);
    // a t^2 + 2 b t + cc = 0, the root in (0, 1] without cancellation
    if (!s.inverted)
      t = cc / (-bb + sq);
    else if (bb > 0.0)
      t = -cc / (bb + sq);
    else
      t = (-bb + sq) / a2;
  }
  if (!(t >= 0x1p-52)) t = 0x1p-52;
  if (t > 1.0) t = 1.0;
  return t;
}

// Lever from the centre (shortest image; planes: plain difference).
__device__ inline void lever_arm(const DevSolid &s, const double c[3], double px, double py, double pz,
                                 const Box3 &b, double r[3]) {
#pragma clang fp contract(off)
  if (s.kind == K_PLANE) {
    r[0] = px - c[0];
    r[1] = py - c[1];
    r[2] = b.D == 2 ? 0.0 : pz - c[2];
    return;
  }
  r[0] = min_image(px - c[0], b.nx);
  r[1] = min_image(py - c[1], b.ny);
  r[2] = b.D == 2 ? 0.0 : min_image(pz - c[2], b.nz);
}

// Rigid-body wall velocity U + Omega x r.
__device__ inline void wall_vel(const DevSolid &s, const double r[3], double uw[3]) {
#pragma clang fp contract(off)
  uw[0] = s.U[0] + (s.W[1] * r[2] - s.W[2] * r[1]);
  uw[1] = s.U[1] + (s.W[2] * r[0] - s.W[0] * r[2]);
  uw[2] = s.U[2] + (s.W[0] * r[1] - s.W[1] * r[0]);
}

// Displacement of solid s at time t since its Lagrangian points were placed
// (prescribed motion at any t, free motion at t = tref).
__device__ inline void solid_disp(const DevSolid &s, int64_t t, double d[3]) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; a++) d[a] = s.moving ? s.dsp[a] + (double)(t - s.tref) * s.U[a] : s.dsp[a];
}

__device__ inline void solid_centre(const DevSolid &s, int64_t t, const Box3 &b, double c[3]) {
  c[0] = centre_at(s, 0, t, b);
  c[1] = centre_at(s, 1, t, b);
  c[2] = b.D == 2 ? s.c0[2] : centre_at(s, 2, t, b);
}

}  // namespace lbm
