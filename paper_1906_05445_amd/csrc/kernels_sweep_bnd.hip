// kernels_sweep_bnd.hip -- the sweep on a domain with bounded axes (Sec. 3.4:
// velocity inlet, stress-free planes, convective outflow), the outflow
// condition after it, and the state transfers that follow the same slots.
//
// Pull form: every node stores its post-collision values in its own slots.
// A population that arrives at a node across a bounded face is read from the
// slot bnd_src names (lbm_device.hpp): the mirrored direction in the node's
// own layer at a stress-free plane; the node's own slot of the reverse
// direction at the inlet (plus the inlet term) and at the outlet.  The map
// from (node, direction) to slot stays one to one, so the sweep writes no
// slot that another node of the same sweep reads, and get/set of the state
// are exact inverses.
#include <hip/hip_ext.h>

#include "sweep_core.hpp"

namespace lbm {

// Bounded domains always take the flag variant (solids or not), and always
// store with non-temporal hints: the tuner's choice of store hint does not
// apply.  Offsets are 32-bit when the arrays hold fewer than 2^32 values.
template <typename S>
static void sweep_bnd_dispatch(lbm_ctx *c, const void *A, void *B, const SweepArgs &a, const SweepLinkArgs &la,
                               int coll, int inl, hipEvent_t e0, hipEvent_t e1) {
  const uint32_t tiles = (uint32_t)((c->N + kBlock - 1) / kBlock);
  const uint32_t grid =
      (tiles + sweep_cpt_of<S>() - 1) / sweep_cpt_of<S>() + a.rblocks + a.iblocks + (inl ? la.cblocks : 0u);
  const S *As = static_cast<const S *>(A);
  S *Bs = static_cast<S *>(B);
  const bool idx32 = (uint64_t)c->Q * c->L.stride < (1ull << 32);
#define LBM_SWEEP_BND1(QQ, CC, II, XX)                                                                         \
  hipExtLaunchKernelGGL((k_sweep<QQ, CC, S, 1, 1, II, XX, 1>), dim3(grid), dim3(kBlock), 0, c->stream, e0, e1, \
                        0, As, Bs, a, la)
#define LBM_SWEEP_BND(QQ, CC, II)                \
  do {                                           \
    if (idx32) LBM_SWEEP_BND1(QQ, CC, II, 1);    \
    else LBM_SWEEP_BND1(QQ, CC, II, 0);          \
  } while (0)
#define LBM_SWEEP_BND2(QQ, CC)                 \
  do {                                         \
    if (inl == 2) LBM_SWEEP_BND(QQ, CC, 2);    \
    else if (inl) LBM_SWEEP_BND(QQ, CC, 1);    \
    else LBM_SWEEP_BND(QQ, CC, 0);             \
  } while (0)
  if (c->Q == 9) {
    if (coll == COLL_BGK) LBM_SWEEP_BND2(9, COLL_BGK);
    else if (coll == COLL_TRT) LBM_SWEEP_BND2(9, COLL_TRT);
    else LBM_SWEEP_BND2(9, COLL_MRT);
  } else {
    if (coll == COLL_BGK) LBM_SWEEP_BND2(19, COLL_BGK);
    else if (coll == COLL_TRT) LBM_SWEEP_BND2(19, COLL_TRT);
    else LBM_SWEEP_BND2(19, COLL_MRT);
  }
#undef LBM_SWEEP_BND2
#undef LBM_SWEEP_BND
#undef LBM_SWEEP_BND1
}

void launch_sweep_bnd(lbm_ctx *c, const void *A, void *B, const SweepArgs &a, const SweepLinkArgs &la, int coll,
                      int inl, hipEvent_t e0, hipEvent_t e1) {
  if (c->p.storage == LBM_F64) sweep_bnd_dispatch<double>(c, A, B, a, la, coll, inl, e0, e1);
  else if (c->p.storage == LBM_F32_DEV) sweep_bnd_dispatch<float>(c, A, B, a, la, coll, inl, e0, e1);
  else sweep_bnd_dispatch<_Float16>(c, A, B, a, la, coll, inl, e0, e1);
}

// ----------------------------------------------------------------------------
// convective outflow (Sec. 3.4)
// ----------------------------------------------------------------------------
// After the sweep of step t (A its input, B its output): for every node of
// the last layer x = N and every direction i entering it from outside (e_ix < 0),
//   h_i(N, t+1) = [h_i(N, t) + U_o h_i(N-1, t+1)] / (1 + U_o),
// U_o = max(u_x of the node's collision at step t, 0) (kept by the sweep in uo).
// h_i(N, t) is in the node's own slot of the reverse direction in A (where the
// sweep pulled it), h_i(N-1, t+1) is what node (N-1, y, z) pulls from B, and
// the result goes to the node's reverse slot in B, which the sweep filled with
// a value that leaves the domain.  The weights sum to one, so the condition
// reads the same on f and on the stored deviations h = f - w.
template <int Q, typename S>
__global__ __launch_bounds__(256) void k_outflow(const S *__restrict__ A, S *__restrict__ B,
                                                 const typename Store<S>::C *__restrict__ uo, SweepArgs a) {
  using C = typename Store<S>::C;
  using L = Lat<Q>;
  const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;  // y + ny z
  if (p >= a.ny * a.nz) return;
  const int x = (int)a.nx - 1;
  const int y = (int)(p % a.ny), z = (int)(p / a.ny);
  const uint32_t n = (uint32_t)x + a.nx * p;
  C U = uo[p];
  if (U < C(0)) U = C(0);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    if (L::ex(i) >= 0) continue;
    const C old = Store<S>::ld(A + pidx<Q>(opp(i), n));
    const BndSrc s = bnd_src(L::ex(i), L::ey(i), L::ez(i), x - 1, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
    const C up = Store<S>::ld(B + pidx<Q>(bnd_dir<Q>(i, s), s.cell));
    B[pidx<Q>(opp(i), n)] = store_value<S, C>((old + U * up) / (C(1) + U), a.sr != 0,
                                                a.sr ? hash32((n * 32u + (uint32_t)opp(i)) ^ a.seed) >> 19 : 0u);
  }
}

template <typename S>
static void outflow_t(lbm_ctx *c, const void *A, void *B, const SweepArgs &a) {
  using C = typename Store<S>::C;
  const uint32_t plane = a.ny * a.nz;
  const C *uo = static_cast<const C *>(a.uo);
  if (c->Q == 9)
    hipLaunchKernelGGL((k_outflow<9, S>), dim3((plane + 255) / 256), dim3(256), 0, c->stream,
                       static_cast<const S *>(A), static_cast<S *>(B), uo, a);
  else
    hipLaunchKernelGGL((k_outflow<19, S>), dim3((plane + 255) / 256), dim3(256), 0, c->stream,
                       static_cast<const S *>(A), static_cast<S *>(B), uo, a);
}

void launch_outflow(lbm_ctx *c, const void *A, void *B) {
  SweepArgs a;
  fill_sweep_args(c, &a);
  if (c->p.storage == LBM_F64) outflow_t<double>(c, A, B, a);
  else if (c->p.storage == LBM_F32_DEV) outflow_t<float>(c, A, B, a);
  else outflow_t<_Float16>(c, A, B, a);
}

// ----------------------------------------------------------------------------
// state transfer on bounded domains
// ----------------------------------------------------------------------------
// One direction of the host-visible populations f_i(x) (before the next
// collision) to or from the slots that hold them.  d: the direction's vector,
// its reverse and its mirror images jf[mask] (dir_flip), w_i and the inlet
// term 6 w_i e_ix U_in.  raw: the stored bits as they are (no inlet term).
struct DirBnd {
  int ex, ey, ez, jo;
  int jf[8];
  double w, binl;
};

__device__ inline void cell_xyz_b(uint32_t n, const CellArgs &a, int &x, int &y, int &z) {
  const uint32_t yz = fdiv(n, a.fx);
  x = (int)(n - yz * a.nx);
  z = (int)fdiv(yz, a.fy);
  y = (int)(yz - (uint32_t)z * a.ny);
}

template <typename S>
__global__ void k_encode_bnd(const double *__restrict__ f, const S *__restrict__ raw_src, S *__restrict__ A, int Q,
                             DirBnd d, CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz_b(n, a, x, y, z);
  const BndSrc s = bnd_src(d.ex, d.ey, d.ez, x, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
  const int j = s.open ? d.jo : d.jf[s.flip];
  S *slot = A + pidx_rt(Q, j, s.cell);
  if (raw_src) *slot = raw_src[n];
  else Store<S>::st(slot, (typename Store<S>::C)((f[n] - d.w) - (s.inlet ? d.binl : 0.0)));
}

template <typename S>
__global__ void k_decode_bnd(const S *__restrict__ A, double *__restrict__ f, S *__restrict__ raw_dst, int Q,
                             DirBnd d, const uint8_t *flags, CellArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz_b(n, a, x, y, z);
  const BndSrc s = bnd_src(d.ex, d.ey, d.ez, x, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
  const int j = s.open ? d.jo : d.jf[s.flip];
  const S v = A[pidx_rt(Q, j, s.cell)];
  if (raw_dst) {
    raw_dst[n] = v;
    return;
  }
  const bool solid = flags && (flags[n] & F_SOLID);
  f[n] = solid ? 0.0 : d.w + ((double)(typename Store<S>::C)v + (s.inlet ? d.binl : 0.0));
}

template <int Q>
static DirBnd dir_bnd_q(int i, double uin) {
  DirBnd d{};
  d.ex = Lat<Q>::ex(i);
  d.ey = Lat<Q>::ey(i);
  d.ez = Lat<Q>::ez(i);
  d.jo = opp(i);
  for (int m = 0; m < 8; m++) d.jf[m] = dir_flip<Q>(i, m);
  d.w = wgt<Q>(i);
  d.binl = 6.0 * wgt<Q>(i) * ((double)Lat<Q>::ex(i) * uin);
  return d;
}

static CellArgs cell_args_bnd(const lbm_ctx *c) {
  CellArgs a{};
  a.N = (uint32_t)c->N;
  a.nx = (uint32_t)c->p.nx;
  a.ny = (uint32_t)c->p.ny;
  a.nz = (uint32_t)c->p.nz;
  a.fx = c->fx;
  a.fy = c->fy;
  a.stride = c->L.stride;
  a.bnd = 1;
  for (int k = 0; k < 3; k++) a.bc[k] = c->p.boundary[k];
  a.uin = c->p.inflow;
  return a;
}

template <typename S>
static void transfer_bnd_t(lbm_ctx *c, int dir, const double *f, void *A, bool encode, bool raw) {
  const DirBnd d = c->Q == 9 ? dir_bnd_q<9>(dir, c->p.inflow) : dir_bnd_q<19>(dir, c->p.inflow);
  const CellArgs a = cell_args_bnd(c);
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
  S *As = static_cast<S *>(A);
  if (encode)
    hipLaunchKernelGGL(k_encode_bnd<S>, dim3(grid), dim3(256), 0, c->stream, raw ? nullptr : f,
                       raw ? reinterpret_cast<const S *>(f) : nullptr, As, c->Q, d, a);
  else {
    const uint8_t *fl = c->nsolid > 0 ? c->at<uint8_t>(c->L.flags) : nullptr;
    double *dst = const_cast<double *>(f);
    hipLaunchKernelGGL(k_decode_bnd<S>, dim3(grid), dim3(256), 0, c->stream, As, raw ? nullptr : dst,
                       raw ? reinterpret_cast<S *>(dst) : nullptr, c->Q, d, fl, a);
  }
}

void launch_transfer_bnd(lbm_ctx *c, int dir, const double *f, void *A, bool encode, bool raw) {
  if (c->p.storage == LBM_F64) transfer_bnd_t<double>(c, dir, f, A, encode, raw);
  else if (c->p.storage == LBM_F32_DEV) transfer_bnd_t<float>(c, dir, f, A, encode, raw);
  else transfer_bnd_t<_Float16>(c, dir, f, A, encode, raw);
}

// A uniform state h (every slot of direction i holding h_i) made exact on a
// bounded domain: each slot that bnd_src names across a bounded face gets the
// value of the direction that pulls it, less the inlet term where it applies.
template <int Q, typename S>
__global__ void k_bnd_uniform(S *__restrict__ A, DirVals h, CellArgs a) {
  using L = Lat<Q>;
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  cell_xyz_b(n, a, x, y, z);
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const BndSrc s = bnd_src(L::ex(i), L::ey(i), L::ez(i), x, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
    if (!s.open && s.flip == 0) continue;
    const double b = s.inlet ? 6.0 * wgt<Q>(i) * ((double)L::ex(i) * a.uin) : 0.0;
    Store<S>::st(A + pidx<Q>(bnd_dir<Q>(i, s), s.cell), (typename Store<S>::C)(h.v[i] - b));
  }
}

template <typename S>
static void bnd_uniform_t(lbm_ctx *c, void *A, const double *hv) {
  DirVals h{};
  for (int i = 0; i < c->Q; i++) h.v[i] = hv[i];
  const CellArgs a = cell_args_bnd(c);
  const uint32_t grid = (uint32_t)((c->N + 255) / 256);
  if (c->Q == 9)
    hipLaunchKernelGGL((k_bnd_uniform<9, S>), dim3(grid), dim3(256), 0, c->stream, static_cast<S *>(A), h, a);
  else
    hipLaunchKernelGGL((k_bnd_uniform<19, S>), dim3(grid), dim3(256), 0, c->stream, static_cast<S *>(A), h, a);
}

void launch_bnd_uniform(lbm_ctx *c, void *A, const double *h) {
  if (c->p.storage == LBM_F64) bnd_uniform_t<double>(c, A, h);
  else if (c->p.storage == LBM_F32_DEV) bnd_uniform_t<float>(c, A, h);
  else bnd_uniform_t<_Float16>(c, A, h);
}

}  // namespace lbm
