// lbm_ibb.hpp -- interpolated bounce-back of one boundary link and its
// momentum-exchange force/torque terms (Sec. 2.2: Eq. 10, Eq. 11, Eq. 12-14,
// Eq. 16; Eq. 17).
//
// A link is evaluated in three parts: its geometry (wall point, lever arm,
// wall velocity, neighbours), the formula and coefficients that the method,
// q and the fluid neighbours select, and the arithmetic on the populations.
// The bounce-back kernel runs all three every step; for fixed solids the
// first two are tabulated once per lbm_step call and the sweep runs only the
// third (except for Zhao-Yong, whose pre-collision input lives in the array
// the next sweep overwrites: its links stay with the kernel).  Both routes call these same functions, compiled without
// floating-point contraction, so they produce the same bits.
#pragma once

#include <cstddef>

#include "lbm_geom.hpp"

namespace lbm {

// Formula of a link: Eq. 11a / 11b (quadratic, x_ff and x_fff fluid), Yu's
// unified scheme (Eq. 12-14, x_ff and x_fff fluid), the linear interpolations
// for q < 1/2 (x_ff fluid) and q >= 1/2, plain bounce-back (Eq. 10; also the
// linear scheme for q < 1/2 without x_ff), and Zhao & Yong's single-node
// scheme (Eq. 16).
enum { LK_PLAIN = 0, LK_Q2_NEAR = 1, LK_Q2_FAR = 2, LK_Q1_NEAR = 3, LK_Q1_FAR = 4, LK_YU = 5, LK_ZY = 6 };

// k1..k4 weigh the populations of the formula; kB scales the wall term B of
// Eq. 10 (1 except for Yu and Zhao-Yong).
template <typename C>
struct LinkCoef {
  int kind;
  C k1, k2, k3, k4;
  double kB;
};

template <typename C>
__device__ inline LinkCoef<C> link_coef(int method, double q, bool ffok, bool fffok) {
#pragma clang fp contract(off)
  LinkCoef<C> k{LK_PLAIN, C(0), C(0), C(0), C(0), 1.0};
  if (method == LBM_IBB_ZHAO_YONG) {
    // Eq. 16: only x_f is read, whatever its neighbours are
    k.kind = LK_ZY;
    k.k1 = (C)(2.0 * q / (1.0 + 2.0 * q));
    k.k2 = (C)(1.0 / (1.0 + 2.0 * q));
    k.kB = 1.0 / (1.0 + 2.0 * q);
  } else if (method == LBM_IBB_YU && ffok && fffok) {
    // Eq. 12-14 in one formula: interpolate f*_ibar at the point 1 - q from
    // x_f (weights q(1+q)/2, (1+q)(1-q), -q(1-q)/2), bounce at the wall (+B),
    // interpolate f_i at x_f from the wall point (-q), x_ff and x_fff (weights
    // 2/((1+q)(2+q)), 2q/(1+q), -q/(2+q)).  The products give q/(2+q),
    // 2(1-q)/(2+q), -q(1-q)/((1+q)(2+q)) on f*_ibar; the weight of f_i(x_fff)
    // is -q/(2+q) as well, so k1 serves both.
    k.kind = LK_YU;
    k.k1 = (C)(q / (2.0 + q));
    k.k2 = (C)(2.0 * (1.0 - q) / (2.0 + q));
    k.k3 = (C)(q * (1.0 - q) / ((1.0 + q) * (2.0 + q)));
    k.k4 = (C)(2.0 * q / (1.0 + q));
    k.kB = 2.0 / ((1.0 + q) * (2.0 + q));
  } else if (method == LBM_IBB_QUADRATIC && ffok && fffok) {
    if (q < 0.5) {
      k.kind = LK_Q2_NEAR;
      k.k1 = (C)(q * (2.0 * q + 1.0));
      k.k2 = (C)((1.0 + 2.0 * q) * (1.0 - 2.0 * q));
      k.k3 = (C)(q * (1.0 - 2.0 * q));
    } else {
      k.kind = LK_Q2_FAR;
      k.k1 = (C)(1.0 / (q * (2.0 * q + 1.0)));
      k.k2 = (C)((2.0 * q - 1.0) / q);
      k.k3 = (C)((2.0 * q - 1.0) / (1.0 + 2.0 * q));
    }
  } else if (method == LBM_IBB_QUADRATIC || method == LBM_IBB_YU || method == LBM_IBB_LINEAR) {
    if (q < 0.5) {
      if (ffok) {
        k.kind = LK_Q1_NEAR;
        k.k1 = (C)(2.0 * q);
        k.k2 = (C)(1.0 - 2.0 * q);
      }
    } else {
      k.kind = LK_Q1_FAR;
      k.k1 = (C)(2.0 * q);
      k.k2 = (C)((2.0 * q - 1.0) / (2.0 * q));
    }
  }
  return k;
}

// The wall term as the formula uses it, kB * B, rounded once to the compute
// type (for kB = 1 this is B itself).
template <typename C>
__device__ inline C link_wall(const LinkCoef<C> &k, double B) {
#pragma clang fp contract(off)
  return (C)(k.kB * B);
}

// Unknown deviation h_i(x_f, t+1).  hb_*: post-collision h_ibar at x_f, x_ff,
// x_fff; hs_*: post-collision h_i at x_f, x_ff (= h_i at x_ff, x_fff after
// streaming); hpre: h_ibar(x_f, t) before the collision (Zhao-Yong only).
// Bw: the wall term from link_wall.  The coefficients of every scheme sum to
// one, so the formulas hold for the deviations as written for f.  Values a
// formula does not use may be anything.
template <typename C>
__device__ inline C link_value(const LinkCoef<C> &k, C Bw, C hb_f, C hb_ff, C hb_fff, C hs_f, C hs_ff, C hpre) {
#pragma clang fp contract(off)
  switch (k.kind) {
    case LK_Q2_NEAR: return k.k1 * hb_f + k.k2 * hb_ff - k.k3 * hb_fff + Bw;  // Eq. 11a
    case LK_Q2_FAR: return k.k1 * (hb_f + Bw) + k.k2 * hs_f - k.k3 * hs_ff;   // Eq. 11b
    case LK_Q1_NEAR: return k.k1 * hb_f + k.k2 * hb_ff + Bw;
    case LK_Q1_FAR: return (hb_f + Bw) / k.k1 + k.k2 * hs_f;
    case LK_YU: return k.k1 * hb_f + k.k2 * hb_ff - k.k3 * hb_fff + k.k4 * hs_f - k.k1 * hs_ff + Bw;  // Eq. 12-14
    case LK_ZY: return k.k1 * hs_f + k.k2 * hpre + Bw;  // Eq. 16
    default: return hb_f + Bw;  // Eq. 10
  }
}

// Geometry of link (x_f, i) of solid sd with centre c: x_f = cell (x, y, z),
// direction i, fraction q.  Returns the wall term B (FP64) and the constants
// of Eq. 17, dF = hout a - hin b - d with a = -e_i - u_w, b = e_i - u_w,
// d = 2 w_i e_i (the rest-state part w (e_ibar - u_w) - w (e_i - u_w) of
// f = w + h), and the lever arm r from the centre to the wall point; also the
// cells x_b = x_f - e_i, x_ff, x_fff.
struct LinkGeo {
  double B;
  double a[3], b[3], d[3], r[3];
  uint32_t nb, nff, nfff;
};

template <int Q>
__device__ inline LinkGeo link_geo(int i, double q, const DevSolid &sd, const double c[3], int x, int y, int z,
                                   const Box3 &box) {
#pragma clang fp contract(off)
  using L = Lat<Q>;
  int ex = 0, ey = 0, ez = 0;
  double w = 0.0;
#pragma unroll
  for (int k = 1; k < Q; k++)
    if (k == i) {
      ex = L::ex(k);
      ey = L::ey(k);
      ez = L::ez(k);
      w = wgt<Q>(k);
    }
  LinkGeo g;
  double uw[3];
  lever_arm(sd, c, (double)x - q * ex, (double)y - q * ey, (double)z - q * ez, box, g.r);
  wall_vel(sd, g.r, uw);
  g.B = 6.0 * w * (ex * uw[0] + ey * uw[1] + ez * uw[2]);
  const double e[3] = {(double)ex, (double)ey, (double)ez};
  for (int k = 0; k < 3; k++) {
    g.a[k] = -e[k] - uw[k];
    g.b[k] = e[k] - uw[k];
    g.d[k] = 2.0 * w * e[k];
  }
  auto id = [&](int dx, int dy, int dz) {
    return (uint32_t)wrapi(x + dx, box.nx) +
           (uint32_t)box.nx * ((uint32_t)wrapi(y + dy, box.ny) + (uint32_t)box.ny * (uint32_t)wrapi(z + dz, box.nz));
  };
  g.nb = id(-ex, -ey, -ez);
  g.nff = id(ex, ey, ez);
  g.nfff = id(2 * ex, 2 * ey, 2 * ez);
  return g;
}

// Eq. 17 force (acc 0..2) and torque about the centre (acc 3..5) of one link
// from the stored outgoing h_ibar(x_f) and incoming h_i(x_f, t+1), in FP64.
__device__ inline void link_ft(double hin, double hout, const double a[3], const double b[3], const double d[3],
                               const double r[3], double acc[6]) {
#pragma clang fp contract(off)
  double dF[3];
  for (int k = 0; k < 3; k++) dF[k] = hout * a[k] - hin * b[k] - d[k];
  acc[0] = dF[0];
  acc[1] = dF[1];
  acc[2] = dF[2];
  acc[3] = r[1] * dF[2] - r[2] * dF[1];
  acc[4] = r[2] * dF[0] - r[0] * dF[2];
  acc[5] = r[0] * dF[1] - r[1] * dF[0];
}

// Tabulated part of a link of a fixed solid, as the sweep reads it (48 bytes
// for FP32 and FP16 storage, 64 for FP64), stored in sweep-segment order.
// B holds the scaled wall term (link_wall).
// The four words that address the link's loads (n, nff, nfff, kind_dir) come
// first after the coefficients, 16-byte aligned, so that the sweep can fetch
// them in one load before its own pulls (LinkRec::head).
template <typename C>
struct alignas(16) LinkRec {
  C k1, k2, k3, B;
  uint32_t n, nff, nfff;  // x_f, x_ff, x_fff
  uint32_t kind_dir;      // kind | i << 8
  uint32_t nb;            // x_b
  uint32_t l;             // link index (order of the force sums)
  C k4;
  __device__ static uint4 head(const LinkRec *r) { return *reinterpret_cast<const uint4 *>(&r->n); }
};
static_assert(sizeof(LinkRec<float>) == 48 && sizeof(LinkRec<double>) == 64, "link record size");
static_assert(offsetof(LinkRec<float>, n) % 16 == 0 && offsetof(LinkRec<double>, n) % 16 == 0 &&
                  offsetof(LinkRec<float>, kind_dir) == offsetof(LinkRec<float>, n) + 12,
              "link record head");

// Chunk partials of links evaluated in the sweep: the same per-link terms,
// summed over the same 64 lanes in the same order, as the bounce-back kernel
// forms from its registers (the link's geometry formed again from its cell,
// direction and q, exactly as when its record was tabulated).  Block `blk`
// (256 threads): chunk units 4*blk .. 4*blk+3, one per wavefront.
template <int Q>
__device__ inline void chunk_sum_waves(const ChunkSumArgs &a, uint32_t blk) {
  const int lane = threadIdx.x & 63;
  const uint32_t u = blk * 4 + (threadIdx.x >> 6);
  const uint32_t s = u / a.per, bx = u - s * a.per;
  if ((int)s >= a.nsolid) return;
  const SolidLinks sl = a.sl[s];
  if (!(bx < sl.nchunks && (uint64_t)sl.chunk_base + bx < a.max_partials)) return;
  const uint32_t li = bx * kLinkChunk + lane;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  // (links are numbered below stride; the test only guards the table bounds)
  if (li < sl.count && (uint64_t)sl.start + li < a.max_links && (uint64_t)sl.start + li < a.stride) {
    const uint64_t l = (uint64_t)sl.start + li;
    double hin, hout;
    if (a.cbytes == 8) {
      hin = static_cast<const double *>(a.io)[l];
      hout = static_cast<const double *>(a.io)[a.stride + l];
    } else {
      hin = (double)static_cast<const float *>(a.io)[l];
      hout = (double)static_cast<const float *>(a.io)[a.stride + l];
    }
    const uint32_t n = a.lcell[l], meta = a.lmeta[l];
    const double q = a.lq[l];
    const uint32_t yz = fdiv(n, a.fx);
    const int x = (int)(n - yz * (uint32_t)a.nx), z = (int)fdiv(yz, a.fy);
    const int y = (int)(yz - (uint32_t)z * (uint32_t)a.ny);
    const Box3 box{a.nx, a.ny, a.nz, a.D};
    const DevSolid sd = a.solids[s];
    double c[3];
    solid_centre(sd, 0, box, c);  // a fixed solid: its centre at any time
    const LinkGeo g = link_geo<Q>((int)(meta & 31u), q, sd, c, x, y, z, box);
    link_ft(hin, hout, g.a, g.b, g.d, g.r, acc);
  }
  for (int k = 0; k < 6; k++) {
    const double tot = wave_sum(acc[k]);
    if (lane == 0) a.partials[(uint64_t)(sl.chunk_base + bx) * 6 + k] = tot;
  }
}

}  // namespace lbm
