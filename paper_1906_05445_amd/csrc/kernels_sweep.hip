// kernels_sweep.hip -- launches of the fused pull stream-collide sweep
// (sweep_core.hpp) on periodic domains and in batches, and the per-cell
// helper kernels (state encode/decode, macroscopic fields, watchdog, copy).
#include <hip/hip_ext.h>

#include "sweep_core.hpp"

namespace lbm {

// Batched sweep: the tiles of every lattice of a work list in one persistent
// launch; each lattice keeps its own arguments, size and state parity.
template <int Q, int COLL, typename S, int NT>
__global__ __launch_bounds__(kBlock) void k_sweep_batch(const BatchSlot *__restrict__ slots,
                                                         const WorkList *__restrict__ wl,
                                                         const int64_t *__restrict__ step, int order) {
  const int par = (int)(*step & 1);
  batch_units(wl, order, [&](int m, uint32_t blk) {
    const int cur = SLOT(m, cur0) ^ par;
    SweepArgs a = SLOT(m, sw);
    a.seed = sr_seed(SLOT(m, t0) + *step);
    // (a member holds fewer than 2^31 values per array: 32-bit offsets)
    sweep_body<Q, COLL, S, 1, NT, 0, 1>(static_cast<const S *>(SLOT(m, P[cur])), static_cast<S *>(SLOT(m, P[cur ^ 1])),
                                     a, nullptr, blk);
  });
}

template <int Q, typename S>
static void sweep_batch_t(const BatchLaunch &b, const WorkList *wl, int coll, int nt, int order, uint32_t grid,
                          hipEvent_t e0, hipEvent_t e1) {
  // events (tuning, timing) are attached to the dispatch; graph capture takes plain launches
#define LBM_SB(CC, NN)                                                                                          \
  do {                                                                                                          \
    if (e0 || e1)                                                                                               \
      hipExtLaunchKernelGGL((k_sweep_batch<Q, CC, S, NN>), dim3(grid), dim3(kBlock), 0, b.stream, e0, e1, 0,    \
                            b.slots, wl, b.step, order);                                                        \
    else                                                                                                        \
      hipLaunchKernelGGL((k_sweep_batch<Q, CC, S, NN>), dim3(grid), dim3(kBlock), 0, b.stream, b.slots, wl,     \
                         b.step, order);                                                                        \
  } while (0)
  if (coll == COLL_BGK) {
    if (nt) LBM_SB(COLL_BGK, 1);
    else LBM_SB(COLL_BGK, 0);
  } else if (coll == COLL_TRT) {
    if (nt) LBM_SB(COLL_TRT, 1);
    else LBM_SB(COLL_TRT, 0);
  } else {
    if (nt) LBM_SB(COLL_MRT, 1);
    else LBM_SB(COLL_MRT, 0);
  }
#undef LBM_SB
}

void launch_sweep_batch(const BatchLaunch &b, const WorkList *wl, int coll, int nt, int order, uint32_t grid,
                        hipEvent_t e0, hipEvent_t e1) {
  if (b.Q == 9) {
    if (b.storage == LBM_F64) sweep_batch_t<9, double>(b, wl, coll, nt, order, grid, e0, e1);
    else if (b.storage == LBM_F32_DEV) sweep_batch_t<9, float>(b, wl, coll, nt, order, grid, e0, e1);
    else sweep_batch_t<9, _Float16>(b, wl, coll, nt, order, grid, e0, e1);
  } else {
    if (b.storage == LBM_F64) sweep_batch_t<19, double>(b, wl, coll, nt, order, grid, e0, e1);
    else if (b.storage == LBM_F32_DEV) sweep_batch_t<19, float>(b, wl, coll, nt, order, grid, e0, e1);
    else sweep_batch_t<19, _Float16>(b, wl, coll, nt, order, grid, e0, e1);
  }
}

// Batch step counter: advanced once at the end of every batched step.
__global__ void k_tick(int64_t *step) {
  if (threadIdx.x == 0) step[0] = step[0] + 1;
}
void launch_tick(hipStream_t s, int64_t *step) { hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, step); }

template <typename S>
static void sweep_dispatch(lbm_ctx *c, const void *A, void *B, const SweepArgs &a, const SweepLinkArgs &la, int coll,
                           bool flags, bool nt, int inl, hipEvent_t e0, hipEvent_t e1) {
  const uint32_t tiles = (uint32_t)((c->N + kBlock - 1) / kBlock);
  const uint32_t grid =
      (tiles + sweep_cpt_of<S>() - 1) / sweep_cpt_of<S>() + a.rblocks + a.iblocks + (inl ? la.cblocks : 0u);
  const S *As = static_cast<const S *>(A);
  S *Bs = static_cast<S *>(B);
  // the events (when given) are attached to the dispatch itself and time the kernel alone
  // 32-bit offsets when Q * stride < 2^32
  const bool idx32 = (uint64_t)c->Q * c->L.stride < (1ull << 32);
#define LBM_SWEEP1(QQ, CC, FF, NN, II, XX)                                                                   \
  hipExtLaunchKernelGGL((k_sweep<QQ, CC, S, FF, NN, II, XX>), dim3(grid), dim3(kBlock), 0, c->stream, e0, e1, 0, \
                        As, Bs, a, la)
#define LBM_SWEEP(QQ, CC, FF, NN, II)               \
  do {                                              \
    if (idx32) LBM_SWEEP1(QQ, CC, FF, NN, II, 1);   \
    else LBM_SWEEP1(QQ, CC, FF, NN, II, 0);         \
  } while (0)
#define LBM_SWEEP2(QQ, CC)                     \
  do {                                         \
    if (inl == 2) {                            \
      if (nt) LBM_SWEEP(QQ, CC, 1, 1, 2);      \
      else LBM_SWEEP(QQ, CC, 1, 0, 2);         \
    } else if (inl) {                          \
      if (nt) LBM_SWEEP(QQ, CC, 1, 1, 1);      \
      else LBM_SWEEP(QQ, CC, 1, 0, 1);         \
    } else if (flags) {                        \
      if (nt) LBM_SWEEP(QQ, CC, 1, 1, 0);      \
      else LBM_SWEEP(QQ, CC, 1, 0, 0);         \
    } else {                                   \
      if (nt) LBM_SWEEP(QQ, CC, 0, 1, 0);      \
      else LBM_SWEEP(QQ, CC, 0, 0, 0);         \
    }                                          \
  } while (0)
  if (c->Q == 9) {
    if (coll == COLL_BGK) LBM_SWEEP2(9, COLL_BGK);
    else if (coll == COLL_TRT) LBM_SWEEP2(9, COLL_TRT);
    else LBM_SWEEP2(9, COLL_MRT);
  } else {
    if (coll == COLL_BGK) LBM_SWEEP2(19, COLL_BGK);
    else if (coll == COLL_TRT) LBM_SWEEP2(19, COLL_TRT);
    else LBM_SWEEP2(19, COLL_MRT);
  }
#undef LBM_SWEEP2
#undef LBM_SWEEP
#undef LBM_SWEEP1
}

// Two-rate test: every even non-conserved row shares one rate, every odd
// non-conserved row another.
static bool two_rate(const lbm_ctx *c, double *sp, double *sm) {
  int se = -1, so = -1;
  for (int k = 0; k < c->Q; k++) {
    const bool cons = c->Q == 9 ? conserved<9>(k) : conserved<19>(k);
    if (cons) continue;
    const bool odd = c->Q == 9 ? odd_row<9>(k) : odd_row<19>(k);
    int &ref = odd ? so : se;
    if (ref < 0) ref = k;
    else if (c->rates[ref] != c->rates[k]) return false;
  }
  *sp = c->rates[se];
  *sm = c->rates[so];
  return true;
}

template <int Q>
static void mrt_coeffs(const lbm_ctx *c, SweepArgs &a) {
  for (int k = 0; k < Q; k++) {
    const double n = (double)mnorm<Q>(k);
    a.sA[k] = -c->rates[k] / n;
    a.sB[k] = (1.0 - 0.5 * c->rates[k]) / n;
  }
}

// Sweep arguments of a context; returns the collision kind.
static int make_sweep_args(lbm_ctx *c, SweepArgs &a) {
  a = SweepArgs{};
  a.N = (uint32_t)c->N;
  a.nx = (uint32_t)c->p.nx;
  a.ny = (uint32_t)c->p.ny;
  a.nz = (uint32_t)c->p.nz;
  a.fx = c->fx;
  a.fy = c->fy;
  a.stride = c->L.stride;
  a.flags = c->at<uint8_t>(c->L.flags);
  a.fibm = c->ws + c->L.fibm;
  for (int k = 0; k < 3; k++) a.g[k] = c->p.body_force[k];
  for (int k = 0; k < 3; k++) a.bc[k] = c->p.boundary[k];
  a.uin = c->p.inflow;
  a.uo = c->p.boundary[0] == BND_OPEN ? c->ws + c->L.uo : nullptr;
  a.sr = c->p.storage == LBM_F16_SR ? 1u : 0u;
  a.seed = sr_seed(c->t);
  int coll;
  if (c->p.collision == LBM_BGK) {
    coll = COLL_BGK;
    a.omega = 1.0 / c->p.tau;
  } else if (two_rate(c, &a.sp, &a.sm)) {
    coll = COLL_TRT;
  } else {
    coll = COLL_MRT;
    if (c->Q == 9) mrt_coeffs<9>(c, a);
    else mrt_coeffs<19>(c, a);
  }
  return coll;
}

int collision_kind(const lbm_ctx *c, double *sp, double *sm) {
  double a, b;
  if (c->p.collision == LBM_BGK) return COLL_BGK;
  if (two_rate(c, sp ? sp : &a, sm ? sm : &b)) return COLL_TRT;
  return COLL_MRT;
}

void fill_sweep_args(lbm_ctx *c, SweepArgs *a) { make_sweep_args(c, *a); }

void launch_sweep(lbm_ctx *c, const void *A, void *B, int policy, hipEvent_t e0, hipEvent_t e1, int64_t reduce_t,
                  int64_t ibm_t, int64_t link_t, int64_t sum_t, bool ghost) {
  SweepArgs a;
  const int coll = make_sweep_args(c, a);
  const int nt = policy & 1;
  a.xcd = (uint32_t)((policy >> 1) & 1);
  if (reduce_t >= 0 && c->k5_chunks > 0) {
    a.ft = ft_reduce_args(c, reduce_t);
    a.ft.partials = partials_of(c, reduce_t);
    a.rblocks = (uint32_t)((c->nsolid + 3) / 4);
  }
  if (ibm_t >= 0) {
    a.ift = ibm_ft_args_of(c, ibm_t);
    a.iblocks = (uint32_t)c->nsolid;
  }
  SweepLinkArgs la{};
  // Zhao-Yong links are evaluated after the relaxation of step link_t itself,
  // the other schemes' links of step link_t when step link_t + 1 pulls them
  const int inl = (link_t >= 0 && c->link_lists) ? (c->method == LBM_IBB_ZHAO_YONG ? 2 : 1) : 0;
  if (inl) {
    la.seg_link = c->at<SegLink>(c->L.seg_link);
    la.cell_list = c->at<uint32_t>(c->L.cell_list);
    la.nseg = (uint32_t)((c->N + 63) / 64);
    la.rec = link_rec_of(c);
    la.io = link_io_of(c, link_t);
    la.stride = c->link_stride;
    la.sr = a.sr;
    la.lseed = sr_seed(link_t);
    la.ghost = ghost ? 1u : 0u;
    if (sum_t >= 0) {
      la.cs = chunk_sum_args(c, sum_t);
      la.cblocks = chunk_sum_blocks(c);
    }
  }
  if (bounded(c)) {
    launch_sweep_bnd(c, A, B, a, la, coll, inl, e0, e1);
    return;
  }
  const bool flags = c->nsolid > 0;
  const bool ntb = nt != 0;
  if (c->p.storage == LBM_F64) sweep_dispatch<double>(c, A, B, a, la, coll, flags, ntb, inl, e0, e1);
  else if (c->p.storage == LBM_F32_DEV) sweep_dispatch<float>(c, A, B, a, la, coll, flags, ntb, inl, e0, e1);
  else sweep_dispatch<_Float16>(c, A, B, a, la, coll, flags, ntb, inl, e0, e1);
}

// ----------------------------------------------------------------------------
// state encode / decode (host-visible populations are f_i(x) before the next
// collision; the device keeps them shifted by e_i, A_i(y) = h_i(y + e_i))
// ----------------------------------------------------------------------------
__device__ inline void cell_xyz(uint32_t n, const CellArgs &a, int &x, int &y, int &z) {
  const uint32_t yz = fdiv(n, a.fx);
  x = (int)(n - yz * a.nx);
  z = (int)fdiv(yz, a.fy);
  y = (int)(yz - (uint32_t)z * a.ny);
}
__device__ inline uint32_t cell_id(int x, int y, int z, const CellArgs &a) {
  return (uint32_t)wrapi(x, a.nx) + a.nx * ((uint32_t)wrapi(y, a.ny) + a.ny * (uint32_t)wrapi(z, a.nz));
}

template <typename S>
__global__ void k_encode(const double *__restrict__ f, S *__restrict__ A, int Q, int dir, int ex, int ey, int ez,
                         double w, CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz(n, a, x, y, z);
  Store<S>::st(A + pidx_rt(Q, dir, n), (typename Store<S>::C)(f[cell_id(x + ex, y + ey, z + ez, a)] - w));
}
template <typename S>
__global__ void k_shift_raw(const S *__restrict__ src, S *__restrict__ A, int Q, int dir, int ex, int ey, int ez,
                            CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz(n, a, x, y, z);
  A[pidx_rt(Q, dir, n)] = src[cell_id(x + ex, y + ey, z + ez, a)];
}
template <typename S>
__global__ void k_decode(const S *__restrict__ A, double *__restrict__ f, int Q, int dir, int ex, int ey, int ez,
                         double w, const uint8_t *flags, CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz(n, a, x, y, z);
  const bool solid = flags && (flags[n] & F_SOLID);
  f[n] = solid ? 0.0 : w + (double)Store<S>::ld(A + pidx_rt(Q, dir, cell_id(x - ex, y - ey, z - ez, a)));
}
template <typename S>
__global__ void k_gather_raw(const S *__restrict__ A, S *__restrict__ dst, int Q, int dir, int ex, int ey, int ez,
                             CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz(n, a, x, y, z);
  dst[n] = A[pidx_rt(Q, dir, cell_id(x - ex, y - ey, z - ez, a))];
}

static CellArgs cell_args(const lbm_ctx *c) {
  CellArgs a{};
  a.N = (uint32_t)c->N;
  a.nx = (uint32_t)c->p.nx;
  a.ny = (uint32_t)c->p.ny;
  a.nz = (uint32_t)c->p.nz;
  a.fx = c->fx;
  a.fy = c->fy;
  a.stride = c->L.stride;
  a.bnd = bounded(c) ? 1 : 0;
  for (int k = 0; k < 3; k++) a.bc[k] = c->p.boundary[k];
  a.uin = c->p.inflow;
  return a;
}

static void dir_vec(int Q, int i, int &ex, int &ey, int &ez, double &w) {
  if (Q == 9) {
    ex = Lat<9>::ex(i);
    ey = Lat<9>::ey(i);
    ez = 0;
    w = wgt<9>(i);
  } else {
    ex = Lat<19>::ex(i);
    ey = Lat<19>::ey(i);
    ez = Lat<19>::ez(i);
    w = wgt<19>(i);
  }
}

template <typename S>
static void encode_t(lbm_ctx *c, int dir, const double *src, void *A, bool raw) {
  CellArgs a = cell_args(c);
  int ex, ey, ez;
  double w;
  dir_vec(c->Q, dir, ex, ey, ez, w);
  S *As = static_cast<S *>(A);
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
  if (raw)
    hipLaunchKernelGGL(k_shift_raw<S>, dim3(grid), dim3(256), 0, c->stream, reinterpret_cast<const S *>(src), As,
                       c->Q, dir, ex, ey, ez, a);
  else
    hipLaunchKernelGGL(k_encode<S>, dim3(grid), dim3(256), 0, c->stream, src, As, c->Q, dir, ex, ey, ez, w, a);
}
template <typename S>
static void decode_t(lbm_ctx *c, int dir, const void *A, double *dst, bool raw) {
  CellArgs a = cell_args(c);
  int ex, ey, ez;
  double w;
  dir_vec(c->Q, dir, ex, ey, ez, w);
  const S *As = static_cast<const S *>(A);
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
  const uint8_t *fl = c->nsolid > 0 ? c->at<uint8_t>(c->L.flags) : nullptr;
  if (raw)
    hipLaunchKernelGGL(k_gather_raw<S>, dim3(grid), dim3(256), 0, c->stream, As, reinterpret_cast<S *>(dst), c->Q,
                       dir, ex, ey, ez, a);
  else
    hipLaunchKernelGGL(k_decode<S>, dim3(grid), dim3(256), 0, c->stream, As, dst, c->Q, dir, ex, ey, ez, w, fl, a);
}

void launch_encode_shift(lbm_ctx *c, int dir, const double *src, void *A, bool raw) {
  if (bounded(c)) return launch_transfer_bnd(c, dir, src, A, true, raw);
  if (c->p.storage == LBM_F64) encode_t<double>(c, dir, src, A, raw);
  else if (c->p.storage == LBM_F32_DEV) encode_t<float>(c, dir, src, A, raw);
  else encode_t<_Float16>(c, dir, src, A, raw);
}
void launch_decode_gather(lbm_ctx *c, int dir, const void *A, double *dst, bool raw) {
  if (bounded(c)) return launch_transfer_bnd(c, dir, dst, const_cast<void *>(A), false, raw);
  if (c->p.storage == LBM_F64) decode_t<double>(c, dir, A, dst, raw);
  else if (c->p.storage == LBM_F32_DEV) decode_t<float>(c, dir, A, dst, raw);
  else decode_t<_Float16>(c, dir, A, dst, raw);
}

// ----------------------------------------------------------------------------
// macroscopic fields
// ----------------------------------------------------------------------------
// Stored deviation h_i arriving at (x, y, z) before a collision: A_i(x - e_i),
// or on a bounded domain the slot bnd_src names plus the inlet term.
template <int Q, typename S>
__device__ inline double gather_h(const S *__restrict__ src, const CellArgs &a, int i, int x, int y, int z) {
  using L = Lat<Q>;
  if (a.bnd) {
    const BndSrc s = bnd_src(L::ex(i), L::ey(i), L::ez(i), x, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
    const double v = (double)Store<S>::ld(src + pidx<Q>(bnd_dir<Q>(i, s), s.cell));
    return s.inlet ? v + 6.0 * wgt<Q>(i) * ((double)L::ex(i) * a.uin) : v;
  }
  const uint32_t sn = cell_id(x - L::ex(i), y - L::ey(i), z - L::ez(i), a);
  return (double)Store<S>::ld(src + pidx<Q>(i, sn));
}

// src holds populations in the shifted (pull) form, so gathering A_i(x - e_i)
// gives the populations that arrive at x before a collision.
// initial (no step since the state was set): u = j / rho.
// otherwise src is the input array of the last collision, which no later
// kernel writes (the sweep, bounce-back and refill all write the other
// array): the gather returns exactly what that collision used, and
// u = (j + F/2) / rho with the force F of that collision.
template <int Q, typename S>
__device__ inline void macros_body(const S *__restrict__ src, double *__restrict__ out, const MacroArgs &m,
                                   uint32_t n) {
  using L = Lat<Q>;
  const CellArgs &a = m.ca;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz(n, a, x, y, z);
  const uint8_t fl = m.flags ? m.flags[n] : 0;
  const bool solid = fl & m.solid_bit;
  if (solid && m.owner[n] < m.nsolid) {
    DevSolid s = m.solids[m.owner[n]];
    if (m.moved && s.free) {
      // a free solid's table already holds the next step; its state at the collision
      for (int k = 0; k < 3; k++) {
        s.c0[k] = s.cp[k];
        s.U[k] = s.Up[k];
        s.W[k] = s.Wp[k];
      }
      s.tref = m.t_geom;
    }
    Box3 b{(int)a.nx, (int)a.ny, (int)a.nz, m.D};
    double c[3], r[3], uw[3];
    solid_centre(s, m.t_geom, b, c);
    lever_arm(s, c, (double)x, (double)y, (double)z, b, r);
    wall_vel(s, r, uw);
    out[n] = 0.0;
    out[a.N + n] = uw[0];
    out[2ull * a.N + n] = uw[1];
    out[3ull * a.N + n] = uw[2];
    return;
  }
  double drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const double h = gather_h<Q, S>(src, a, i, x, y, z);
    drho += h;
    jx += L::ex(i) * h;
    jy += L::ey(i) * h;
    jz += L::ez(i) * h;
  }
  const double rho = 1.0 + drho;
  double F[3] = {0.0, 0.0, 0.0};
  if (!m.initial) {
    // a node fluid at the collision gets the body force unless it lies inside
    // an IBM solid (translating solids are IBB: their flags already moved on)
    if (m.moved || !(fl & F_NOBODY))
      for (int k = 0; k < 3; k++) F[k] = m.g[k];
    if (fl & F_IBM) {
      using C = typename Store<S>::C;
      const C *fb = reinterpret_cast<const C *>(m.fibm);
      for (int k = 0; k < m.D; k++) F[k] += (double)fb[k * a.stride + n];
    }
  }
  out[n] = rho;
  out[a.N + n] = (jx + 0.5 * F[0]) / rho;
  out[2ull * a.N + n] = (jy + 0.5 * F[1]) / rho;
  out[3ull * a.N + n] = (jz + 0.5 * F[2]) / rho;
}
template <int Q, typename S>
__global__ void k_macros(const S *__restrict__ src, double *__restrict__ out, MacroArgs m) {
  macros_body<Q, S>(src, out, m, blockIdx.x * blockDim.x + threadIdx.x);
}

// Strain rate s_ab and dissipation 2 nu s_ab s_ab of the last collision from
// its non-equilibrium moments (Sec. 3.1, Eq. 19), in FP64: the same gather,
// density, velocity and force as macros_body, then Pi_ab = sum e_a e_b
// (h - h_eq) and Guo's second moment u_a F_b + u_b F_a.  The first-order
// Chapman-Enskog balance of a second-order row k with rate s_k,
// -s_k m_k + (1 - s_k/2) psi_k = 2 rho0 c_s^2 (row k of s) + (row k of uF + Fu),
// with psi_k the row of uF + Fu, gives row k of s = -(3/2) s_k m_k
// - (3/4) s_k (row k of uF + Fu) (rho0 = 1, c_s^2 = 1/3), solved for s over
// the trace and the traceless rows.  IBB solid nodes give 0.
template <int Q, typename S>
__device__ inline void strain_body(const S *__restrict__ src, double *__restrict__ out, const StrainArgs &sa,
                                   uint32_t n) {
  using L = Lat<Q>;
  const MacroArgs &m = sa.m;
  const CellArgs &a = m.ca;
  if (n >= a.N) return;
  double sv[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const uint8_t fl = m.flags ? m.flags[n] : 0;
  if (!(fl & m.solid_bit)) {
    int x, y, z;
    cell_xyz(n, a, x, y, z);
    double h[Q];
    double drho = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < Q; i++) {
      h[i] = gather_h<Q, S>(src, a, i, x, y, z);
      drho += h[i];
      jx += L::ex(i) * h[i];
      jy += L::ey(i) * h[i];
      jz += L::ez(i) * h[i];
    }
    const double rho = 1.0 + drho;
    double F[3] = {0.0, 0.0, 0.0};
    if (m.moved || !(fl & F_NOBODY))
      for (int k = 0; k < 3; k++) F[k] = m.g[k];
    if (fl & F_IBM) {
      using C = typename Store<S>::C;
      const C *fb = reinterpret_cast<const C *>(m.fibm);
      for (int k = 0; k < m.D; k++) F[k] += (double)fb[k * a.stride + n];
    }
    const double u[3] = {(jx + 0.5 * F[0]) / rho, (jy + 0.5 * F[1]) / rho, (jz + 0.5 * F[2]) / rho};
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    // Pi^neq: xx, yy, zz, xy, yz, xz
    double P[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const double ex = L::ex(i), ey = L::ey(i), ez = L::ez(i);
      const double eu = ex * u[0] + ey * u[1] + ez * u[2];
      const double d = h[i] - wgt<Q>(i) * (drho + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
      P[0] += ex * ex * d;
      P[1] += ey * ey * d;
      P[2] += ez * ez * d;
      P[3] += ex * ey * d;
      P[4] += ey * ez * d;
      P[5] += ex * ez * d;
    }
    const double G[6] = {2.0 * u[0] * F[0], 2.0 * u[1] * F[1], 2.0 * u[2] * F[2],
                         u[0] * F[1] + u[1] * F[0], u[1] * F[2] + u[2] * F[1], u[0] * F[2] + u[2] * F[0]};
    auto row = [&](double s, double mk, double gk) { return -1.5 * s * mk - 0.75 * s * gk; };
    if (Q == 9) {
      const double XT = row(sa.s[0], P[0] + P[1], G[0] + G[1]);
      const double XN = row(sa.s[1], P[0] - P[1], G[0] - G[1]);
      sv[0] = 0.5 * (XT + XN);
      sv[1] = 0.5 * (XT - XN);
      sv[3] = row(sa.s[3], P[3], G[3]);
    } else {
      const double XT = row(sa.s[0], P[0] + P[1] + P[2], G[0] + G[1] + G[2]);
      const double XP = row(sa.s[1], 2.0 * P[0] - P[1] - P[2], 2.0 * G[0] - G[1] - G[2]);
      const double XW = row(sa.s[2], P[1] - P[2], G[1] - G[2]);
      const double rest = (2.0 * XT - XP) / 3.0;
      sv[0] = (XT + XP) / 3.0;
      sv[1] = 0.5 * (rest + XW);
      sv[2] = 0.5 * (rest - XW);
      sv[3] = row(sa.s[3], P[3], G[3]);
      sv[4] = row(sa.s[4], P[4], G[4]);
      sv[5] = row(sa.s[5], P[5], G[5]);
    }
  }
  if (sa.part == 0) {
    const double ss = sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2] +
                      2.0 * (sv[3] * sv[3] + sv[4] * sv[4] + sv[5] * sv[5]);
    out[n] = sv[0];
    out[a.N + n] = sv[1];
    out[2ull * a.N + n] = sv[2];
    out[3ull * a.N + n] = 2.0 * sa.nu * ss;
  } else {
    out[n] = sv[3];
    out[a.N + n] = sv[4];
    out[2ull * a.N + n] = sv[5];
  }
}
template <int Q, typename S>
__global__ void k_strain(const S *__restrict__ src, double *__restrict__ out, StrainArgs sa) {
  strain_body<Q, S>(src, out, sa, blockIdx.x * blockDim.x + threadIdx.x);
}

// mode 0: no step since the state was set; mode 1: fields of the last
// collision, in the geometry of that collision.
void fill_macro_args(lbm_ctx *c, MacroArgs *mp, int mode) {
  MacroArgs &m = *mp;
  m = MacroArgs{};
  m.ca = cell_args(c);
  m.flags = c->nsolid > 0 ? c->at<uint8_t>(c->L.flags) : nullptr;
  const bool prev = mode == 1 && c->any_moving;
  m.owner = c->at<uint16_t>(prev ? c->L.owner1 : c->L.owner0);
  m.solid_bit = prev ? F_WAS_SOLID : F_SOLID;
  m.moved = prev ? 1 : 0;
  m.solids = c->at<DevSolid>(c->L.solids);
  m.fibm = c->ws + c->L.fibm;
  for (int k = 0; k < 3; k++) m.g[k] = c->p.body_force[k];
  m.t_geom = mode == 1 ? c->t - 1 : c->t;
  m.D = c->D;
  m.initial = mode == 0 ? 1 : 0;
  m.nsolid = c->nsolid;
}

void launch_strain(lbm_ctx *c, const void *src, double *out, int part) {
  StrainArgs sa{};
  fill_macro_args(c, &sa.m, 1);
  sa.part = part;
  sa.nu = (c->p.tau - 0.5) / 3.0;
  // rows of the rates in the moment order of lbm.h
  static const int r19[6] = {1, 9, 11, 13, 14, 15}, r9[6] = {1, 7, 7, 8, 8, 8};
  for (int k = 0; k < 6; k++)
    sa.s[k] = c->p.collision == LBM_BGK ? 1.0 / c->p.tau : c->rates[c->Q == 9 ? r9[k] : r19[k]];
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
#define LBM_STR(QQ, SS) \
  hipLaunchKernelGGL((k_strain<QQ, SS>), dim3(grid), dim3(256), 0, c->stream, static_cast<const SS *>(src), out, sa)
  if (c->Q == 9) {
    if (c->p.storage == LBM_F64) LBM_STR(9, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_STR(9, float);
    else LBM_STR(9, _Float16);
  } else {
    if (c->p.storage == LBM_F64) LBM_STR(19, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_STR(19, float);
    else LBM_STR(19, _Float16);
  }
#undef LBM_STR
}

void launch_macros(lbm_ctx *c, const void *src, double *out, int mode) {
  MacroArgs m;
  fill_macro_args(c, &m, mode);
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
#define LBM_MAC(QQ, SS) \
  hipLaunchKernelGGL((k_macros<QQ, SS>), dim3(grid), dim3(256), 0, c->stream, static_cast<const SS *>(src), out, m)
  if (c->Q == 9) {
    if (c->p.storage == LBM_F64) LBM_MAC(9, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_MAC(9, float);
    else LBM_MAC(9, _Float16);
  } else {
    if (c->p.storage == LBM_F64) LBM_MAC(19, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_MAC(19, float);
    else LBM_MAC(19, _Float16);
  }
#undef LBM_MAC
}


// ----------------------------------------------------------------------------
// zero fill, finiteness watchdog, copy probe
// ----------------------------------------------------------------------------
__global__ void k_zero(uint4 *p, uint64_t n16) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n16; i += (uint64_t)gridDim.x * blockDim.x)
    p[i] = make_uint4(0, 0, 0, 0);
}
void launch_fill_zero(lbm_ctx *c, void *A) {
  const uint64_t bytes = (uint64_t)c->Q * c->L.stride * c->store_bytes;
  hipLaunchKernelGGL(k_zero, dim3(2048), dim3(256), 0, c->stream, static_cast<uint4 *>(A), bytes / 16);
}

// Every slot of direction i (every cell, solid nodes and tile padding
// included) set to the stored deviation v[i]: a uniform state, whose pull
// gives the same populations at every cell.
template <typename S>
__global__ void k_fill_uniform(S *__restrict__ A, uint64_t count, uint32_t Q, DirVals v) {
  for (uint64_t k = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; k < count; k += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = (uint32_t)((k / kTile) % Q);
    A[k] = (S)v.v[i];
  }
}

void launch_fill_uniform(lbm_ctx *c, void *A, const double *h) {
  const uint64_t count = (uint64_t)c->Q * c->L.stride;
  DirVals v;
  for (int i = 0; i < kMaxQ; i++) v.v[i] = i < c->Q ? h[i] : 0.0;
  if (c->store_bytes == 8)
    hipLaunchKernelGGL(k_fill_uniform<double>, dim3(2048), dim3(256), 0, c->stream, static_cast<double *>(A), count,
                       (uint32_t)c->Q, v);
  else if (c->store_bytes == 4)
    hipLaunchKernelGGL(k_fill_uniform<float>, dim3(2048), dim3(256), 0, c->stream, static_cast<float *>(A), count,
                       (uint32_t)c->Q, v);
  else
    hipLaunchKernelGGL(k_fill_uniform<_Float16>, dim3(2048), dim3(256), 0, c->stream, static_cast<_Float16 *>(A),
                       count, (uint32_t)c->Q, v);
}

template <typename S>
__global__ void k_finite(const S *__restrict__ A, uint64_t count, uint32_t *flag) {
  using C = typename Store<S>::C;
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < count; i += (uint64_t)gridDim.x * blockDim.x) {
    const C v = (C)A[i];
    bad |= !(v - v == C(0));
  }
  if (bad) atomicOr(flag, 1u);
}
int launch_check_finite(lbm_ctx *c, const void *A, uint32_t *flag) {
  (void)hipMemsetAsync(flag, 0, sizeof(uint32_t), c->stream);
  const uint64_t count = (uint64_t)c->Q * c->L.stride;
  if (c->p.storage == LBM_F64)
    hipLaunchKernelGGL(k_finite<double>, dim3(1024), dim3(256), 0, c->stream, static_cast<const double *>(A), count,
                       flag);
  else if (c->p.storage == LBM_F32_DEV)
    hipLaunchKernelGGL(k_finite<float>, dim3(1024), dim3(256), 0, c->stream, static_cast<const float *>(A), count,
                       flag);
  else
    hipLaunchKernelGGL(k_finite<_Float16>, dim3(1024), dim3(256), 0, c->stream, static_cast<const _Float16 *>(A),
                       count, flag);
  return 0;
}

__global__ __launch_bounds__(256) void k_copy(const uint4 *__restrict__ s, uint4 *__restrict__ d, uint64_t n16) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < n16) d[i] = s[i];
}
void launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s) {
  const uint64_t n16 = bytes / 16;
  hipLaunchKernelGGL(k_copy, dim3((uint32_t)((n16 + 255) / 256)), dim3(256), 0, s, static_cast<const uint4 *>(src),
                     static_cast<uint4 *>(dst), n16);
}

}  // namespace lbm
