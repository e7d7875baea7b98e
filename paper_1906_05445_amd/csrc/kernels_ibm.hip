// kernels_ibm.hip -- direct-forcing immersed boundary method (Sec. 2.1,
// Eq. 5-9) with Peskin's 4-point delta (Eq. 6) or the 3- and 2-point deltas
// compared in Sec. 3.1, iterated n_iter times (Sec. 3.1), and the
// force/torque on each solid from its Lagrangian forces.
//
// Data: the Lagrangian points (FP64 positions, per-axis delta weights, the
// shell index of each of their 4^D stencil cells), the shell (the sorted
// union of all stencil cells) with, per shell cell, the list of (point,
// stencil slot) that cover it sorted by point.  Interpolation is a gather
// per point; spreading is a gather per shell cell over that list, so no
// atomics are used and every sum has a fixed order.
//
// A step's forcing is a chain of launches, one per phase (u0, then
// interpolation and spreading per iteration): the phases depend on each other
// across the whole shell, and a kernel boundary is the cheapest device-wide
// synchronisation available.  Single contexts and batches run different
// kernels around the same contraction-free arithmetic, in the same order, so
// they produce the same bits.
#include <algorithm>

#include "lbm_args.hpp"

namespace lbm {

// Eq. 6, one factor.
__device__ inline double phi4(double r) {
  r = fabs(r);
  if (r >= 2.0) return 0.0;
  if (r >= 1.0) return 0.125 * (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r));
  return 0.125 * (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r));
}
// The other deltas of Sec. 3.1 (not printed there): Roma et al.'s 3-point
// function, support |r| < 3/2, (1 + sqrt(1 - 3r^2))/3 on |r| <= 1/2 and
// (5 - 3|r| - sqrt(1 - 3(1 - |r|)^2))/6 beyond; the 2-point hat 1 - |r|.
// Both vanish outside floor(X) - 1 .. floor(X) + 2, so the 4-node stencil of
// Eq. 6 holds them with exact zeros at the extra nodes.
__device__ inline double phi3(double r) {
  r = fabs(r);
  if (r >= 1.5) return 0.0;
  if (r >= 0.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
  return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
}
__device__ inline double phi2(double r) {
  r = fabs(r);
  return r >= 1.0 ? 0.0 : 1.0 - r;
}
__device__ inline double phi_of(int points, double r) {
  return points == 3 ? phi3(r) : (points == 2 ? phi2(r) : phi4(r));
}


// setup: delta weights and desired velocity U^d = U + Omega x (X - Y)
__global__ void k_ibm_weights(IbmArgs a) {
  const int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (l >= a.nlag) return;
  for (int ax = 0; ax < 3; ax++)
    for (int k = 0; k < 4; k++)
      a.wts[l * 12 + ax * 4 + k] =
          (ax == 2 && a.b.D == 2) ? (k == 0 ? 1.0 : 0.0)
                                  : phi_of(a.delta, (double)(a.base[l * 3 + ax] + k) - a.X[l * 3 + ax]);
  const DevSolid &s = a.solids[a.sid[l]];
  double c[3], r[3], ud[3];
  solid_centre(s, a.t, a.b, c);
  lever_arm(s, c, a.X[l * 3], a.X[l * 3 + 1], a.X[l * 3 + 2], a.b, r);
  wall_vel(s, r, ud);
  if (a.b.D == 2) ud[2] = 0.0;
  for (int k = 0; k < 3; k++) a.Ud[l * 3 + k] = ud[k];
}
__global__ void k_ibm_mark(IbmArgs a) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.nshell) return;
  const uint32_t n = a.shell_cell[s];
  a.flags[n] = (uint8_t)(a.flags[n] | F_IBM);
}

// u0 = (j + g/2)/rho at cell n from the populations f(t), gathered from the
// shifted state (A_i(x - e_i)); the body force only where it acts.
template <int Q, typename S>
__device__ inline void ibm_u0_cell(const S *__restrict__ A, const IbmArgs &a, uint32_t n,
                                   typename Store<S>::C (&u)[3]) {
#pragma clang fp contract(off)
  using C = typename Store<S>::C;
  using L = Lat<Q>;
  const uint32_t yz = fdiv(n, a.fx);
  const int x = (int)(n - yz * (uint32_t)a.b.nx);
  const int z = (int)fdiv(yz, a.fy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)a.b.ny);
  C drho = 0, j[3] = {0, 0, 0};
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const uint32_t src = (uint32_t)wrapi(x - L::ex(i), a.b.nx) +
                         (uint32_t)a.b.nx * ((uint32_t)wrapi(y - L::ey(i), a.b.ny) +
                                             (uint32_t)a.b.ny * (uint32_t)wrapi(z - L::ez(i), a.b.nz));
    const C h = Store<S>::ld(A + pidx<Q>(i, src));
    drho += h;
    j[0] += C(L::ex(i)) * h;
    j[1] += C(L::ey(i)) * h;
    j[2] += C(L::ez(i)) * h;
  }
  const C rho = C(1) + drho;
  const bool body = !(a.flags[n] & F_NOBODY);
  for (int k = 0; k < 3; k++) u[k] = (j[k] + C(0.5) * (body ? (C)a.g[k] : C(0))) / rho;
}

// u0 at shell cell s (cell n) into the shell's velocity; clears its spread force.
template <int Q, typename S>
__device__ inline void ibm_u0_at(const S *__restrict__ A, const IbmArgs &a, int64_t s, uint32_t n) {
  using C = typename Store<S>::C;
  C v[3];
  ibm_u0_cell<Q, S>(A, a, n, v);
  C *u = static_cast<C *>(a.ushell);
  C *f = static_cast<C *>(a.fshell);
  for (int k = 0; k < 3; k++) {
    u[k * a.nshell + s] = v[k];
    f[k * a.nshell + s] = C(0);
  }
}

// Eq. 5 and Eq. 7: interpolate u to the point, F = rho0 (U^d - U~)/dt.
// One wavefront per point, one stencil cell per lane (4^D cells), summed by
// a fixed-order wave reduction.
constexpr int kIbmPointsPerBlock = 4;  // 256-thread blocks

template <typename C>
__device__ inline C wave_sum_c(C v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Delta weight of stencil slot (kx + 4 ky + 16 kz) from the per-axis weights.
template <typename C>
__device__ inline C ibm_weight(const double *w, uint32_t slot) {
#pragma clang fp contract(off)
  return (C)((w[slot & 3u] * w[4 + ((slot >> 2) & 3u)]) * w[8 + (slot >> 4)]);
}

// Stencil slot's share of the interpolated velocity (before the wave sum).
template <typename C>
__device__ inline void ibm_interp_terms(const C *u, int64_t nshell, uint32_t si, C wt, C v[3]) {
#pragma clang fp contract(off)
  v[0] = u[si] * wt;
  v[1] = u[nshell + si] * wt;
  v[2] = u[2 * nshell + si] * wt;
}

// The same share from the velocity values themselves.
template <typename C>
__device__ inline void ibm_interp_values(const C (&u)[3], C wt, C v[3]) {
#pragma clang fp contract(off)
  v[0] = u[0] * wt;
  v[1] = u[1] * wt;
  v[2] = u[2] * wt;
}

// One entry of a row of the point coupling: acc += A_lm F_m.
template <typename C>
__device__ inline void ibm_couple_term(C A, const C (&Fm)[3], C acc[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; k++) acc[k] = acc[k] + A * Fm[k];
}

// Point force of one iteration, F = U^d - U~ (Eq. 7 with rho0 = dt = 1), and
// its running sum over the iterations.
template <typename C>
__device__ inline C ibm_point_force(C ud, C us, double *sum) {
#pragma clang fp contract(off)
  const C F = ud - us;
  *sum = *sum + (double)F;
  return F;
}

// Eq. 8 and Eq. 9: f(x) = sum_l F_l delta dV_l, u += f dt / rho0.
// kSpreadLanes lanes per shell cell share its (point, slot) list, lane k
// taking entries k, k + kSpreadLanes, ...; the lane partials are then summed
// in a fixed tree order.

// One (point, slot) entry of a shell cell's list: f += F_l delta dV_l.
template <typename C>
__device__ inline void ibm_spread_term(const C *Fk, uint32_t l, C wt, C dv, C f[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; k++) f[k] = f[k] + Fk[(uint64_t)l * 3 + k] * wt * dv;
}

// The same with the summed point force (FP64) of all iterations.
template <typename C>
__device__ inline void ibm_spread_sum_term(const double *Fs, C wt, C dv, C f[3]) {
#pragma clang fp contract(off)
  for (int k = 0; k < 3; k++) f[k] = f[k] + (C)Fs[k] * wt * dv;
}

// Fixed-order sum over the lanes of a shell cell; lane 0 holds it.
template <typename C>
__device__ inline void ibm_spread_reduce(C f[3]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int off = kSpreadLanes / 2; off > 0; off >>= 1)
    for (int k = 0; k < 3; k++) f[k] = f[k] + __shfl_down(f[k], off, kSpreadLanes);
}

template <typename C>
__device__ inline C ibm_add(C x, C y) {
#pragma clang fp contract(off)
  return x + y;
}

// ---- fixed solids: the forcing iterations in point space -------------------
// With fixed points, interpolating u^k = u^(k-1) + f^k (Eq. 9) after spreading
// f^k = sum_m F^k_m delta(x - X_m) dV_m (Eq. 8) gives, by linearity,
//   U~^(k+1)_l = U~^k_l + sum_m A_lm F^k_m,
//   A_lm = dV_m sum_x delta(x - X_l) delta(x - X_m),
// so after one interpolation of u0 (Eq. 5) the n_iter iterations of Eq. 7
// run on the points, and the summed force is spread once.  The delta
// function is a product over the axes, and so is the sum over the shared
// stencil cells: A_lm = dV_m prod_a S_a with S_a = sum over the node pairs
// (k, k') of the two stencils that fall on the same node (periodically) of
// w_l[a][k] w_m[a][k'].

// Eq. 5 at the first iteration: u0 at the point's 4^D stencil cells (one
// lane each, pulled from the state as ibm_u0_cell does) times the delta
// weight, wave-summed; then Eq. 7, F = U^d - U~, the first term of the sum.
template <int Q, typename S>
__device__ inline void ibm_interp0_body(const S *__restrict__ A, const IbmArgs &a, int64_t l) {
  using C = typename Store<S>::C;
  const int slot = (int)(threadIdx.x & 63);
  const int kz = slot >> 4;
  const bool pt = l < a.nlag;
  // the point's operands, fetched before the sums that come later need them
  double ud[3] = {0.0, 0.0, 0.0};
  if (pt && slot == 0)
    for (int k = 0; k < 3; k++) ud[k] = a.Ud[l * 3 + k];
  C v[3] = {0, 0, 0};
  if (pt && kz < (a.b.D == 2 ? 1 : 4)) {
    C u[3];
    ibm_u0_cell<Q, S>(A, a, a.idx[l * 64 + slot], u);  // the slot's cell
    ibm_interp_values<C>(u, ibm_weight<C>(a.wts + l * 12, (uint32_t)slot), v);
  }
  for (int k = 0; k < 3; k++) v[k] = wave_sum_c(v[k]);
  if (slot != 0 || !pt) return;
  IbmF4<C> F;
  C *Ut = static_cast<C *>(a.Ut);
  C f[3];
  for (int k = 0; k < 3; k++) {
    double sum = 0.0;
    Ut[l * 3 + k] = v[k];
    f[k] = ibm_point_force<C>((C)ud[k], v[k], &sum);
    a.Fsum[l * 3 + k] = sum;
  }
  F.x = f[0], F.y = f[1], F.z = f[2], F.w = C(0);
  static_cast<IbmF4<C> *>(a.Fk)[l] = F;
}

// Iteration it >= 1: U~ += A F (the forces of iteration it - 1, buffer
// (it - 1) & 1), then F = U^d - U~ into buffer it & 1 and the running sum.
// One wavefront per point, one row entry per lane (rows padded to a fixed
// width with zeros), a fixed-order wave sum.
template <typename C>
__device__ inline void ibm_iter_body(const IbmArgs &a, int it, int64_t l) {
  const int lane = (int)(threadIdx.x & 63);
  const IbmF4<C> *Fp = static_cast<const IbmF4<C> *>(((it - 1) & 1) ? a.Fk2 : a.Fk);
  IbmF4<C> *Fc = static_cast<IbmF4<C> *>((it & 1) ? a.Fk2 : a.Fk);
  const IbmEntry<C> *row = static_cast<const IbmEntry<C> *>(a.nrow);
  const bool pt = l < a.nlag;
  C ut[3] = {0, 0, 0};
  double ud[3] = {0.0, 0.0, 0.0}, fs[3] = {0.0, 0.0, 0.0};
  if (pt && lane == 0) {
    const C *Ut = static_cast<const C *>(a.Ut);
    for (int k = 0; k < 3; k++) {
      ut[k] = Ut[l * 3 + k];
      ud[k] = a.Ud[l * 3 + k];
      fs[k] = a.Fsum[l * 3 + k];
    }
  }
  C acc[3] = {0, 0, 0};
  if (pt)
    for (int j = lane; j < a.nw; j += 64) {
      const IbmEntry<C> e = row[l * a.nw + j];
      const IbmF4<C> F = Fp[e.col];
      const C Fm[3] = {F.x, F.y, F.z};
      ibm_couple_term<C>(e.val, Fm, acc);
    }
  for (int k = 0; k < 3; k++) acc[k] = wave_sum_c(acc[k]);
  if (lane != 0 || !pt) return;
  C *Ut = static_cast<C *>(a.Ut);
  C f[3];
  for (int k = 0; k < 3; k++) {
    const C us = ibm_add<C>(ut[k], acc[k]);
    Ut[l * 3 + k] = us;
    f[k] = ibm_point_force<C>((C)ud[k], us, &fs[k]);
    a.Fsum[l * 3 + k] = fs[k];
  }
  IbmF4<C> F;
  F.x = f[0], F.y = f[1], F.z = f[2], F.w = C(0);
  Fc[l] = F;
}

// The iterations in one pass: with F^(k+1) = F^k - A F^k (Eq. 7 after the
// point-space update), the summed force is sum_{k < n_iter} (I - A)^k F^0 =
// P F^0, and P, a polynomial in A, is formed once per set of fixed points
// (host, FP64).  Row l of P (nptr[l] entries, fixed row stride nw) times the
// first iteration's forces, one wavefront per point, the lane products summed
// in FP64 in a fixed order.
template <typename C>
__device__ inline void ibm_psum_body(const IbmArgs &a, int64_t l) {
#pragma clang fp contract(off)
  const int lane = (int)(threadIdx.x & 63);
  if (l >= a.nlag) return;
  const IbmF4<C> *F0 = static_cast<const IbmF4<C> *>(a.Fk);
  const IbmEntry<C> *row = static_cast<const IbmEntry<C> *>(a.nrow) + l * a.nw;
  double acc[3] = {0.0, 0.0, 0.0};
  const int len = (int)a.nptr[l];
  auto add = [&](const IbmEntry<C> &e, const IbmF4<C> &F) {
    acc[0] = acc[0] + (double)(e.val * F.x);
    acc[1] = acc[1] + (double)(e.val * F.y);
    acc[2] = acc[2] + (double)(e.val * F.z);
  };
  // twelve entries per lane at a time (a row of up to 768 entries in one
  // pass): their loads, then their gathers, are in flight together, and the
  // sums take them in the order of the row
  constexpr int U = 12;
  for (int j = lane; j < len; j += 64 * U) {
    IbmEntry<C> e[U];
    IbmF4<C> F[U];
#pragma unroll
    for (int k = 0; k < U; k++)
      if (j + 64 * k < len) e[k] = row[j + 64 * k];
#pragma unroll
    for (int k = 0; k < U; k++)
      if (j + 64 * k < len) F[k] = F0[e[k].col];
#pragma unroll
    for (int k = 0; k < U; k++)
      if (j + 64 * k < len) add(e[k], F[k]);
  }
  for (int k = 0; k < 3; k++) acc[k] = wave_sum(acc[k]);
  if (lane == 0)
    for (int k = 0; k < 3; k++) a.Fsum[l * 3 + k] = acc[k];
}

// Setup: the values of row l of A (one wavefront per point, one entry per
// lane; the padding keeps value 0).
template <typename C>
__device__ inline void ibm_amat_body(const IbmArgs &a, int64_t l) {
#pragma clang fp contract(off)
  const int lane = (int)(threadIdx.x & 63);
  if (l >= a.nlag) return;
  const int Ls[3] = {a.b.nx, a.b.ny, a.b.nz};
  IbmEntry<C> *row = static_cast<IbmEntry<C> *>(a.nrow) + l * a.nw;
  for (int j = lane; j < (int)a.nptr[l]; j += 64) {
    const uint32_t m = row[j].col;
    double A = a.dV[m];
    for (int ax = 0; ax < 3; ax++) {
      double S = 0.0;
      const int bl = a.base[l * 3 + ax], bm = a.base[(int64_t)m * 3 + ax];
      for (int k = 0; k < 4; k++)
        for (int k2 = 0; k2 < 4; k2++)
          if (wrapi(bl + k - bm - k2, Ls[ax]) == 0) S = S + a.wts[l * 12 + ax * 4 + k] * a.wts[(int64_t)m * 12 + ax * 4 + k2];
      A = A * S;
    }
    row[j].val = (C)A;
  }
}

// Eq. 8 once, with the summed force: f(x) = sum_l (sum_k F^k_l) delta dV_l
// over the shell cell's (point, slot) list, into the force field the sweep
// reads (kSpreadLanes lanes per cell, fixed-order lane sum).
template <typename C>
__device__ inline void ibm_spread_sum_body(const IbmArgs &a, int64_t s) {
  const int lane = (int)(threadIdx.x & (kSpreadLanes - 1));
  C f[3] = {0, 0, 0};
  if (s < a.nshell) {
    const uint32_t e1 = a.rowptr[s + 1];
    for (uint32_t e = a.rowptr[s] + lane; e < e1; e += kSpreadLanes) {
      const uint32_t v = a.ent[e];
      const uint32_t l = v >> 6;
      ibm_spread_sum_term<C>(a.Fsum + (uint64_t)l * 3, ibm_weight<C>(a.wts + (uint64_t)l * 12, v & 63u), (C)a.dV[l],
                             f);
    }
  }
  ibm_spread_reduce<C>(f);
  if (lane != 0 || s >= a.nshell) return;
  C *fb = static_cast<C *>(a.fibm);
  const uint32_t n = a.shell_cell[s];
  for (int k = 0; k < 3; k++) fb[k * a.stride + n] = f[k];
}

// ---- one moving solid ------------------------------------------------------
// The points move rigidly with the solid: X_l(t) = X_l(placed) + d(t).  With
// d = n + delta (n whole cells, delta in [0, 1) per axis), the 4-node stencil
// of a point, floor(X - 1) .. floor(X) + 2, lies inside the 5-node box
// floor(X_placed) - 1 + n .. + 4 whatever delta is.  The shell is the union of
// these boxes where the points were placed, built once with its transpose;
// at step t it is moved by n, and the box nodes outside a point's stencil
// take exact zeros from the delta function.
constexpr int kMvBox = 5;

// Cell of shell cell s under the whole-cell shift sh[0..2].
__device__ inline uint32_t mv_cell(const IbmArgs &a, int64_t s, const int32_t *sh) {
  const uint32_t n = a.shell_cell[s];
  const uint32_t yz = fdiv(n, a.fx);
  const int x = (int)(n - yz * (uint32_t)a.b.nx);
  const int z = (int)fdiv(yz, a.fy);
  const int y = (int)(yz - (uint32_t)z * (uint32_t)a.b.ny);
  return (uint32_t)wrapi(x + sh[0], a.b.nx) +
         (uint32_t)a.b.nx * ((uint32_t)wrapi(y + sh[1], a.b.ny) + (uint32_t)a.b.ny * (uint32_t)wrapi(z + sh[2], a.b.nz));
}

// Per point, 16 threads: the 15 box weights for the displacement d(t), one
// each; the last thread the position, lever arm and U^d, and (point 0) the
// shift of step t.
constexpr int kMoveLanes = 16;
__global__ __launch_bounds__(256) void k_ibm_move(IbmArgs a) {
#pragma clang fp contract(off)
  const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t l = g / kMoveLanes;
  const int j = (int)(g % kMoveLanes);
  if (l >= a.nlag) return;
  const DevSolid &s = a.solids[a.sid[l]];
  double d[3];
  solid_disp(s, a.t, d);
  if (j < 3 * kMvBox) {
    const int ax = j / kMvBox, k = j % kMvBox;
    double w = k == 0 ? 1.0 : 0.0;  // the z axis of D2Q9
    if (ax < a.b.D) {
      const double del = d[ax] - floor(d[ax]);
      w = phi_of(a.delta, (double)(a.base[l * 3 + ax] + k) - (a.X[l * 3 + ax] + del));
    }
    a.wts[l * 24 + j] = w;
    return;
  }
  double X[3], c[3], r[3], ud[3];
  int n[3];
  for (int ax = 0; ax < 3; ax++) {
    const bool on = ax < a.b.D;
    n[ax] = on ? (int)floor(d[ax]) : 0;
    X[ax] = on ? a.X[l * 3 + ax] + d[ax] : a.X[l * 3 + ax];
  }
  double *w = a.wts + l * 24;
  solid_centre(s, a.t, a.b, c);
  lever_arm(s, c, X[0], X[1], X[2], a.b, r);
  wall_vel(s, r, ud);
  if (a.b.D == 2) ud[2] = 0.0;
  for (int k = 0; k < 3; k++) {
    a.Ud[l * 3 + k] = ud[k];
    w[16 + k] = r[k];
  }
  if (l == 0)
    for (int k = 0; k < 3; k++) a.shift[4 * (int)(a.t & 1) + k] = n[k];
}

// u0 on the shell moved to step t; the boundary force and the F_IBM flag of
// the shell of step t - 1 are cleared (the spreading of this step sets them
// on the new cells).
template <int Q, typename S>
__global__ void k_ibm_u0_mv(const S *__restrict__ A, IbmArgs a) {
  using C = typename Store<S>::C;
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= a.nshell) return;
  const int cur = (int)(a.t & 1);
  const uint32_t old = mv_cell(a, s, a.shift + 4 * (cur ^ 1));
  a.flags[old] = (uint8_t)(a.flags[old] & ~F_IBM);
  C *fb = static_cast<C *>(a.fibm);
  for (int k = 0; k < 3; k++) fb[k * a.stride + old] = C(0);
  ibm_u0_at<Q, S>(A, a, s, mv_cell(a, s, a.shift + 4 * cur));
}

template <typename C>
__device__ inline C mv_weight(const double *w, uint32_t slot) {
#pragma clang fp contract(off)
  return (C)((w[slot % 5u] * w[5 + (slot / 5u) % 5u]) * w[10 + slot / 25u]);
}

template <typename C>
__global__ __launch_bounds__(256) void k_ibm_interp_mv(IbmArgs a, int first) {
  const int64_t l = (int64_t)blockIdx.x * kIbmPointsPerBlock + (threadIdx.x >> 6);
  const int lane = (int)(threadIdx.x & 63);
  const int nsl = a.b.D == 2 ? kMvBox * kMvBox : kMvBox * kMvBox * kMvBox;
  const C *u = static_cast<const C *>(a.ushell);
  C v[3] = {0, 0, 0};
  for (int p = 0; p < 2; p++) {
    const int slot = lane + 64 * p;
    if (l < a.nlag && slot < nsl) {
      C t[3];
      ibm_interp_terms<C>(u, a.nshell, a.idx[l * 128 + slot], mv_weight<C>(a.wts + l * 24, (uint32_t)slot), t);
      for (int k = 0; k < 3; k++) v[k] = ibm_add<C>(v[k], t[k]);
    }
  }
  for (int k = 0; k < 3; k++) v[k] = wave_sum_c(v[k]);
  if (lane != 0 || l >= a.nlag) return;
  C *Fk = static_cast<C *>(a.Fk);
  for (int k = 0; k < 3; k++) {
    double sum = first ? 0.0 : a.Fsum[l * 3 + k];
    Fk[l * 3 + k] = ibm_point_force<C>((C)a.Ud[l * 3 + k], v[k], &sum);
    a.Fsum[l * 3 + k] = sum;
  }
}

template <typename C>
__global__ __launch_bounds__(256) void k_ibm_spread_mv(IbmArgs a, int last) {
  const int64_t s = (int64_t)blockIdx.x * kSpreadCellsPerBlock + (threadIdx.x / kSpreadLanes);
  const int lane = (int)(threadIdx.x & (kSpreadLanes - 1));
  const C *Fk = static_cast<const C *>(a.Fk);
  C f[3] = {0, 0, 0};
  if (s < a.nshell) {
    const uint32_t e1 = a.rowptr[s + 1];
    for (uint32_t e = a.rowptr[s] + lane; e < e1; e += kSpreadLanes) {
      const uint32_t v = a.ent[e];
      const uint32_t l = v >> 7;
      ibm_spread_term<C>(Fk, l, mv_weight<C>(a.wts + (uint64_t)l * 24, v & 127u), (C)a.dV[l], f);
    }
  }
  ibm_spread_reduce<C>(f);
  if (lane != 0 || s >= a.nshell) return;
  C *u = static_cast<C *>(a.ushell);
  C *fs = static_cast<C *>(a.fshell);
  for (int k = 0; k < 3; k++) {
    u[k * a.nshell + s] = ibm_add<C>(u[k * a.nshell + s], f[k]);
    fs[k * a.nshell + s] = ibm_add<C>(fs[k * a.nshell + s], f[k]);
  }
  if (last) {
    C *fb = static_cast<C *>(a.fibm);
    const uint32_t n = mv_cell(a, s, a.shift + 4 * (int)(a.t & 1));
    for (int k = 0; k < 3; k++) fb[k * a.stride + n] = fs[k * a.nshell + s];
    a.flags[n] = (uint8_t)(a.flags[n] | F_IBM);
  }
}

// (consecutive points, which lie close together on the mesh, go to one XCD:
// their stencils' populations then come once into that XCD's L2)
template <int Q, typename S>
__global__ __launch_bounds__(256) void k_ibm_interp0(const S *__restrict__ A, IbmArgs a) {
  ibm_interp0_body<Q, S>(A, a,
                         (int64_t)xcd_remap(blockIdx.x, gridDim.x) * kIbmPointsPerBlock + (threadIdx.x >> 6));
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_iter(IbmArgs a, int it) {
  ibm_iter_body<C>(a, it, (int64_t)blockIdx.x * kIbmPointsPerBlock + (threadIdx.x >> 6));
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_spread_sum(IbmArgs a) {
  ibm_spread_sum_body<C>(a, (int64_t)blockIdx.x * kSpreadCellsPerBlock + (threadIdx.x / kSpreadLanes));
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_psum(IbmArgs a) {
  ibm_psum_body<C>(a, (int64_t)blockIdx.x * kIbmPointsPerBlock + (threadIdx.x >> 6));
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_amat(IbmArgs a) {
  ibm_amat_body<C>(a, (int64_t)blockIdx.x * kIbmPointsPerBlock + (threadIdx.x >> 6));
}
__global__ __launch_bounds__(kBlock) void k_ibm_ft(IbmFtArgs f) { ibm_ft_body(f, blockIdx.x); }

// Batched forms over the IBM members of a batch (state P[cur0 ^ (k & 1)] at
// t = t0 + k); a member takes part in forcing iteration `it` while
// it < n_iter.  Units: 128 shell cells or points; one solid for the force.
template <int Q, typename S>
__global__ __launch_bounds__(256) void k_ibm_interp0_batch(const BatchSlot *__restrict__ slots,
                                                           const WorkList *__restrict__ wl,
                                                           const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    IbmArgs a = SLOT(m, im);
    a.t = SLOT(m, t0) + k;
    ibm_interp0_body<Q, S>(static_cast<const S *>(SLOT(m, P[SLOT(m, cur0) ^ (int)(k & 1)])), a,
                           (int64_t)u * kIbmPointsPerBlock + (threadIdx.x >> 6));
  });
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_iter_batch(const BatchSlot *__restrict__ slots,
                                                        const WorkList *__restrict__ wl, int it) {
  batch_units(wl, 0, [&](int m, uint32_t u) {
    if (it < SLOT(m, n_iter)) {
      const IbmArgs a = SLOT(m, im);
      const int64_t l = (int64_t)u * kIbmPointsPerBlock + (threadIdx.x >> 6);
      if (!a.poly) ibm_iter_body<C>(a, it, l);
      else if (it == 1) ibm_psum_body<C>(a, l);  // all iterations in one product
    }
  });
}
template <typename C>
__global__ __launch_bounds__(256) void k_ibm_spread_sum_batch(const BatchSlot *__restrict__ slots,
                                                              const WorkList *__restrict__ wl) {
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const IbmArgs a = SLOT(m, im);
    ibm_spread_sum_body<C>(a, (int64_t)u * kSpreadCellsPerBlock + (threadIdx.x / kSpreadLanes));
  });
}
__global__ __launch_bounds__(kBlock) void k_ibm_ft_batch(const BatchSlot *__restrict__ slots,
                                                      const WorkList *__restrict__ wl,
                                                      const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const int64_t t = SLOT(m, t0) + k;
    const IbmFtArgs f = ibm_ft_args(SLOT(m, im), t, SLOT(m, lag_start), SLOT(m, lag_count),
                                    SLOT(m, hist) + (uint64_t)(t % kHistCap) * (uint64_t)SLOT(m, max_solids) * 6);
    ibm_ft_body(f, (int)u);
  });
}

static IbmArgs ibm_args(lbm_ctx *c, int64_t t) {
  IbmArgs a{};
  a.b = Box3{c->p.nx, c->p.ny, c->p.nz, c->D};
  a.N = (uint32_t)c->N;
  a.fx = c->fx;
  a.fy = c->fy;
  a.stride = c->L.stride;
  a.nlag = c->nlag;
  a.nshell = c->nshell;
  a.delta = c->delta;
  a.X = c->at<double>(c->L.lag_X);
  a.dV = c->at<double>(c->L.lag_dV);
  a.sid = c->at<int32_t>(c->L.lag_sid);
  a.Ud = c->at<double>(c->L.lag_Ud);
  a.base = c->at<int32_t>(c->L.lag_base);
  a.wts = c->at<double>(c->L.lag_w);
  a.idx = c->at<uint32_t>(c->L.lag_idx);
  a.Fsum = c->at<double>(c->L.lag_Fsum);
  a.Fk = c->ws + c->L.lag_Fk;
  a.shell_cell = c->at<uint32_t>(c->L.shell_cell);
  a.rowptr = c->at<uint32_t>(c->L.shell_rowptr);
  a.ent = c->at<uint32_t>(c->L.shell_ent);
  a.ushell = c->ws + c->L.shell_u;
  a.fshell = c->ws + c->L.shell_f;
  a.fibm = c->ws + c->L.fibm;
  a.flags = c->at<uint8_t>(c->L.flags);
  a.solids = c->at<DevSolid>(c->L.solids);
  for (int k = 0; k < 3; k++) a.g[k] = c->p.body_force[k];
  a.t = t;
  a.mv = c->ibm_moving ? 1 : 0;
  a.shift = c->at<int32_t>(c->L.misc + 64 + 16 * (size_t)c->L.max_solids);
  a.nptr = c->at<uint32_t>(c->L.lag_nptr);
  a.nrow = c->ws + c->L.lag_nrow;
  a.nw = c->ibm_nw;
  a.poly = c->ibm_poly ? 1 : 0;
  a.Ut = c->ws + c->L.lag_Ut;
  a.Fk2 = c->ws + c->L.lag_Fk2;
  return a;
}

void launch_ibm_setup(lbm_ctx *c) {
  if (c->nlag <= 0) return;
  IbmArgs a = ibm_args(c, c->t);
  if (c->ibm_moving)
    hipLaunchKernelGGL(k_ibm_move, dim3((uint32_t)((c->nlag * kMoveLanes + 255) / 256)), dim3(256), 0, c->stream, a);
  else {
    hipLaunchKernelGGL(k_ibm_weights, dim3((uint32_t)((c->nlag + 127) / 128)), dim3(128), 0, c->stream, a);
    const dim3 g((uint32_t)((c->nlag + kIbmPointsPerBlock - 1) / kIbmPointsPerBlock));
    if (c->p.storage == LBM_F64) hipLaunchKernelGGL(k_ibm_amat<double>, g, dim3(256), 0, c->stream, a);
    else hipLaunchKernelGGL(k_ibm_amat<float>, g, dim3(256), 0, c->stream, a);
  }
  hipLaunchKernelGGL(k_ibm_mark, dim3((uint32_t)((c->nshell + 255) / 256)), dim3(256), 0, c->stream, a);
}

template <typename S>
static void ibm_step_t(lbm_ctx *c, const void *A, int64_t t, bool with_ft) {
  using C = typename Store<S>::C;
  IbmArgs a = ibm_args(c, t);
  const dim3 gs((uint32_t)((c->nshell + 127) / 128)),
      gl((uint32_t)((c->nlag + kIbmPointsPerBlock - 1) / kIbmPointsPerBlock)),
      gsp((uint32_t)((c->nshell + kSpreadCellsPerBlock - 1) / kSpreadCellsPerBlock));
  if (c->ibm_moving) {
    hipLaunchKernelGGL(k_ibm_move, dim3((uint32_t)((c->nlag * kMoveLanes + 255) / 256)), dim3(256), 0, c->stream, a);
    if (c->Q == 9)
      hipLaunchKernelGGL((k_ibm_u0_mv<9, S>), gs, dim3(128), 0, c->stream, static_cast<const S *>(A), a);
    else
      hipLaunchKernelGGL((k_ibm_u0_mv<19, S>), gs, dim3(128), 0, c->stream, static_cast<const S *>(A), a);
    for (int it = 0; it < c->n_iter; it++) {
      hipLaunchKernelGGL(k_ibm_interp_mv<C>, gl, dim3(256), 0, c->stream, a, it == 0 ? 1 : 0);
      hipLaunchKernelGGL(k_ibm_spread_mv<C>, gsp, dim3(256), 0, c->stream, a, it == c->n_iter - 1 ? 1 : 0);
    }
    if (c->ibm_free) launch_ibm_ft_free(c, t);  // force of step t, then the motion to t + 1 (Eq. 23)
    else if (with_ft)
      hipLaunchKernelGGL(k_ibm_ft, dim3((uint32_t)c->nsolid), dim3(kBlock), 0, c->stream, ibm_ft_args_of(c, t));
    return;
  }
  // fixed solids: u0 and the first interpolation, n_iter - 1 point-space
  // iterations, one spreading of the summed force
  if (c->Q == 9)
    hipLaunchKernelGGL((k_ibm_interp0<9, S>), gl, dim3(256), 0, c->stream, static_cast<const S *>(A), a);
  else
    hipLaunchKernelGGL((k_ibm_interp0<19, S>), gl, dim3(256), 0, c->stream, static_cast<const S *>(A), a);
  if (c->ibm_poly) {
    if (c->n_iter > 1) hipLaunchKernelGGL(k_ibm_psum<C>, gl, dim3(256), 0, c->stream, a);
  } else
    for (int it = 1; it < c->n_iter; it++) hipLaunchKernelGGL(k_ibm_iter<C>, gl, dim3(256), 0, c->stream, a, it);
  hipLaunchKernelGGL(k_ibm_spread_sum<C>, gsp, dim3(256), 0, c->stream, a);
  if (with_ft)
    hipLaunchKernelGGL(k_ibm_ft, dim3((uint32_t)c->nsolid), dim3(kBlock), 0, c->stream, ibm_ft_args_of(c, t));
}

void fill_ibm_args(lbm_ctx *c, IbmArgs *a) { *a = ibm_args(c, c->t); }

template <typename S>
static void ibm_batch_t(const BatchLaunch &b, const WorkList *spread, const WorkList *lag, const WorkList *ft,
                        int max_iter, uint32_t grid) {
  using C = typename Store<S>::C;
  if (b.Q == 9)
    hipLaunchKernelGGL((k_ibm_interp0_batch<9, S>), dim3(grid), dim3(256), 0, b.stream, b.slots, lag, b.step);
  else
    hipLaunchKernelGGL((k_ibm_interp0_batch<19, S>), dim3(grid), dim3(256), 0, b.stream, b.slots, lag, b.step);
  for (int it = 1; it < max_iter; it++)
    hipLaunchKernelGGL(k_ibm_iter_batch<C>, dim3(grid), dim3(256), 0, b.stream, b.slots, lag, it);
  hipLaunchKernelGGL(k_ibm_spread_sum_batch<C>, dim3(grid), dim3(256), 0, b.stream, b.slots, spread);
  hipLaunchKernelGGL(k_ibm_ft_batch, dim3(std::min<uint32_t>(grid, 1024)), dim3(kBlock), 0, b.stream, b.slots, ft,
                     b.step);
}

void launch_ibm_batch(const BatchLaunch &b, const WorkList *spread, const WorkList *lag, const WorkList *ft,
                      int max_iter, uint32_t grid) {
  if (b.storage == LBM_F64) ibm_batch_t<double>(b, spread, lag, ft, max_iter, grid);
  else if (b.storage == LBM_F32_DEV) ibm_batch_t<float>(b, spread, lag, ft, max_iter, grid);
  else ibm_batch_t<_Float16>(b, spread, lag, ft, max_iter, grid);
}

IbmFtArgs ibm_ft_args_of(lbm_ctx *c, int64_t t) {
  return ibm_ft_args(ibm_args(c, t), t, c->at<int64_t>(c->L.misc + 64),
                     c->at<int64_t>(c->L.misc + 64 + 8 * c->L.max_solids),
                     c->at<double>(c->L.hist) + (uint64_t)(t % kHistCap) * c->L.max_solids * 6);
}

void launch_ibm_step(lbm_ctx *c, const void *A, int64_t t, bool with_ft) {
  if (c->nlag <= 0 || c->n_iter <= 0) return;
  if (c->p.storage == LBM_F64) ibm_step_t<double>(c, A, t, with_ft);
  else if (c->p.storage == LBM_F32_DEV) ibm_step_t<float>(c, A, t, with_ft);
  else ibm_step_t<_Float16>(c, A, t, with_ft);
}

}  // namespace lbm
