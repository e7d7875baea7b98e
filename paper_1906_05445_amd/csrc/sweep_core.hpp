// sweep_core.hpp -- the fused pull stream-collide sweep: pull, relaxation,
// in-sweep boundary links and the kernel template, shared by the periodic
// sweeps (kernels_sweep.hip) and the bounded-domain ones (kernels_sweep_bnd.hip).
//
// One thread owns one cell.  It gathers f_i(x, t+1) = f*_i(x - e_i, t) from
// the source array (pull streaming; where x - e_i is a solid node, the
// bounce-back value: written into that slot beforehand by the bounce-back
// kernel, or, for fixed solids, evaluated by the sweep itself from the
// source array), relaxes them (Eq. 1 or Eq. 3 with the second-order
// body-force term of Sec. 2.1) and writes the post-collision values of its
// own cell to the destination array.  Storage is the deviation h_i = f_i - w_i (FP64, FP32 or FP16),
// arithmetic is FP64 for FP64 storage and FP32 otherwise.  Arrays are SoA,
// [Q][stride], x fastest, so each of the 2Q streams is coalesced.
#pragma once

#include <utility>

#include "lbm_args.hpp"
#include "lbm_ibb.hpp"

namespace lbm {

enum { COLL_BGK = 0, COLL_TRT = 1, COLL_MRT = 2 };


// Pull of cell n: population i arrives from x - e_i (raw stored values; the
// conversion to the compute type happens in sweep_relax, so the loads of
// several cells can all be in flight together).
// IDX32: the arrays hold fewer than 2^32 values, so offsets are formed in 32
// bits (a 24-bit multiply-add instead of a 64-bit one per gather: FP16,
// whose sweep is bound by instructions, gains 2-4 %, FP32 and FP64 under 1 %).
template <int Q, typename S, int IDX32>
__device__ __forceinline__ void sweep_pull(const S *__restrict__ A, const SweepArgs &a, uint32_t n, S (&r)[Q]) {
  using L = Lat<Q>;
  const uint32_t yz = fdiv(n, a.fx);
  const uint32_t x = n - yz * a.nx;
  const uint32_t z = (Q == 9) ? 0u : fdiv(yz, a.fy);
  const uint32_t y = yz - z * a.ny;
  const uint32_t xm = x == 0 ? a.nx - 1 : x - 1, xp = x + 1 == a.nx ? 0 : x + 1;
  const uint32_t ym = y == 0 ? a.ny - 1 : y - 1, yp = y + 1 == a.ny ? 0 : y + 1;
  const uint32_t zm = z == 0 ? a.nz - 1 : z - 1, zp = z + 1 == a.nz ? 0 : z + 1;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const uint32_t sx = L::ex(i) > 0 ? xm : (L::ex(i) < 0 ? xp : x);
    const uint32_t sy = L::ey(i) > 0 ? ym : (L::ey(i) < 0 ? yp : y);
    const uint32_t sz = L::ez(i) > 0 ? zm : (L::ez(i) < 0 ? zp : z);
    const uint32_t src = sx + a.nx * (sy + a.ny * sz);
    if constexpr (IDX32 != 0) r[i] = A[pidx32<Q>(i, src)];
    else r[i] = A[pidx<Q>(i, src)];
  }
}

// Pull of cell n on a bounded domain: each direction from where bnd_src
// keeps it.  Returns the mask of directions that take the inlet term; uo_at
// is the cell's index in the outlet plane (y + ny z), or ~0u.
template <int Q, typename S, int IDX32>
__device__ __forceinline__ uint32_t sweep_pull_bnd(const S *__restrict__ A, const SweepArgs &a, uint32_t n,
                                                   S (&r)[Q], uint32_t &uo_at) {
  using L = Lat<Q>;
  const uint32_t yz = fdiv(n, a.fx);
  const int x = (int)(n - yz * a.nx);
  const int z = (Q == 9) ? 0 : (int)fdiv(yz, a.fy);
  const int y = (int)yz - z * (int)a.ny;
  uint32_t inl = 0;
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const BndSrc s = bnd_src(L::ex(i), L::ey(i), L::ez(i), x, y, z, (int)a.nx, (int)a.ny, (int)a.nz, a.bc);
    if constexpr (IDX32 != 0) r[i] = A[pidx32<Q>(bnd_dir<Q>(i, s), s.cell)];
    else r[i] = A[pidx<Q>(bnd_dir<Q>(i, s), s.cell)];
    if (s.inlet) inl |= 1u << i;
  }
  uo_at = (a.bc[0] == BND_OPEN && x == (int)a.nx - 1) ? yz : ~0u;
  return inl;
}

// Row K of M times v, over the nonzero entries in ascending i.
template <int Q, int K, typename C, int... I>
__device__ __forceinline__ C mrt_row_dot(const C (&v)[Q], std::integer_sequence<int, I...>) {
  C s = C(0);
  ((s = (mrow<Q>(K, I) != 0) ? s + C(mrow<Q>(K, I)) * v[I] : s), ...);
  return s;
}
// Column I of M^T times dm (the back transform of one direction), ascending k.
template <int Q, int I, typename C, int... K>
__device__ __forceinline__ C mrt_col_dot(const C (&dm)[Q], std::integer_sequence<int, K...>) {
  C s = C(0);
  ((s = (mrow<Q>(K, I) != 0) ? s + C(mrow<Q>(K, I)) * dm[K] : s), ...);
  return s;
}
// dm of one row: conserved rows carry the force (momentum) or nothing
// (density); the others relax with their own rate, scaled by 1/|M_k|^2.
template <int Q, int K, typename C>
__device__ __forceinline__ C mrt_row(const C (&fneq)[Q], const C (&Fh)[Q], const SweepArgs &a, C Fx, C Fy, C Fz) {
  if constexpr (conserved<Q>(K)) {
    const C invn = C(1.0 / mnorm<Q>(K));
    return K == 0 ? C(0) : (K == 3 ? Fx : (K == 5 ? Fy : Fz)) * invn;
  } else {
    const auto seq = std::make_integer_sequence<int, Q>{};
    const C mn = mrt_row_dot<Q, K, C>(fneq, seq);
    const C mf = mrt_row_dot<Q, K, C>(Fh, seq);
    return (C)a.sA[K] * mn + (C)a.sB[K] * mf;
  }
}
template <int Q, typename C, int... K>
__device__ __forceinline__ void mrt_rows(const C (&fneq)[Q], const C (&Fh)[Q], const SweepArgs &a, C Fx, C Fy, C Fz,
                                         C (&dmn)[Q], std::integer_sequence<int, K...>) {
  ((dmn[K] = mrt_row<Q, K, C>(fneq, Fh, a, Fx, Fy, Fz)), ...);
}
template <int Q, typename C, int... I>
__device__ __forceinline__ void mrt_cols(const C (&dmn)[Q], C (&h)[Q], std::integer_sequence<int, I...>) {
  const auto seq = std::make_integer_sequence<int, Q>{};
  ((h[I] += mrt_col_dot<Q, I, C>(dmn, seq)), ...);
}

// Relaxation of one cell (Eq. 1 or Eq. 3 with the forcing of Sec. 2.1) and
// the store of its post-collision values (KEEP: also to keep[0 .. Q-2] for
// directions 1 .. Q-1, when keep is not null).  BND: the directions in inl
// take the inlet term (bnd_src) and a cell of the outlet plane (uo_at) keeps
// its u_x for the outflow condition.
template <int Q, int COLL, typename S, int FLAGS, int NT, int IDX32, bool KEEP = false, bool BND = false>
__device__ __forceinline__ void sweep_relax(S *__restrict__ B, const SweepArgs &a, uint32_t n, uint8_t fl,
                                            const S (&r)[Q], S *keep = nullptr, uint32_t inl = 0u,
                                            uint32_t uo_at = ~0u) {
  using C = typename Store<S>::C;
  using L = Lat<Q>;
  C h[Q];
#pragma unroll
  for (int i = 0; i < Q; i++) h[i] = (C)r[i];
  if constexpr (BND) {
    // inlet (Eq. 10 form): 2 w_i rho0 e_i.u_w / c_s^2 with u_w = (U_in, 0, 0), rho0 = 1
    if (inl) {
      const C U = (C)a.uin;
#pragma unroll
      for (int i = 0; i < Q; i++)
        if (L::ex(i) > 0 && (inl & (1u << i))) h[i] += C(6) * C(wgt<Q>(i)) * (C(L::ex(i)) * U);
    }
  }
  // Directions come in opposite pairs (i, i+1), i odd.  Pair sums and
  // differences give the moments: rho = 1 + drho, j = sum h e (sum w e = 0).
  constexpr int NP = (Q - 1) / 2;
  C Ps[NP], Md[NP];
#pragma unroll
  for (int k = 0; k < NP; k++) {
    Ps[k] = h[2 * k + 1] + h[2 * k + 2];
    Md[k] = h[2 * k + 1] - h[2 * k + 2];
  }
  C drho = h[0], jx = 0, jy = 0, jz = 0;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const int i = 2 * k + 1;
    drho += Ps[k];
    if (L::ex(i)) jx += L::ex(i) > 0 ? Md[k] : -Md[k];
    if (L::ey(i)) jy += L::ey(i) > 0 ? Md[k] : -Md[k];
    if (L::ez(i)) jz += L::ez(i) > 0 ? Md[k] : -Md[k];
  }
  const C rho = C(1) + drho;
  C Fx = 0, Fy = 0, Fz = 0;
  if (!FLAGS || !(fl & F_NOBODY)) {
    Fx = (C)a.g[0];
    Fy = (C)a.g[1];
    Fz = (C)a.g[2];
  }
  if (FLAGS && (fl & F_IBM)) {
    const C *fb = reinterpret_cast<const C *>(a.fibm);
    Fx += fb[n];
    Fy += fb[a.stride + n];
    if (Q == 19) Fz += fb[2 * a.stride + n];
  }
  const C inv = C(1) / rho;
  const C ux = (jx + C(0.5) * Fx) * inv, uy = (jy + C(0.5) * Fy) * inv, uz = (jz + C(0.5) * Fz) * inv;
  const C uu = ux * ux + uy * uy + uz * uz;
  const C uF = ux * Fx + uy * Fy + uz * Fz;
  if constexpr (BND) {
    if (uo_at != ~0u) static_cast<C *>(a.uo)[uo_at] = ux;
  }

  if (COLL == COLL_BGK || COLL == COLL_TRT) {
    // Eq. 3 with one rate on every even and one on every odd non-conserved
    // moment (BGK, Eq. 1: both rates 1/tau): M^-1 S M acts as sp on the part
    // of each pair that is even under e -> -e and as sm on the odd part.
    // With f_eq and Guo's term split the same way, per pair of direction e:
    //   even f_eq Se = w (drho - 1.5 rho u.u + 4.5 rho (e.u)^2),  odd Ao = 3 w rho e.u,
    //   even force FS = w (9 (e.u)(e.F) - 3 u.F),                 odd FA = 3 w e.F.
    const C sp = COLL == COLL_BGK ? (C)a.omega : (C)a.sp;
    const C sm = COLL == COLL_BGK ? (C)a.omega : (C)a.sm;
    const C kp = C(1) - C(0.5) * sp, km = C(1) - C(0.5) * sm;
    const C base = drho - C(1.5) * rho * uu;
    const C w0 = (C)wgt<Q>(0);
    h[0] += -sp * (h[0] - w0 * base) + kp * (w0 * (C(-3) * uF));
#pragma unroll
    for (int k = 0; k < NP; k++) {
      const int i = 2 * k + 1;
      const C w = (C)wgt<Q>(i);
      const C eu = C(L::ex(i)) * ux + C(L::ey(i)) * uy + C(L::ez(i)) * uz;
      const C eF = C(L::ex(i)) * Fx + C(L::ey(i)) * Fy + C(L::ez(i)) * Fz;
      const C Se = w * (base + C(4.5) * rho * eu * eu);
      const C Ao = w * (C(3) * rho * eu);
      const C FS = w * (C(9) * eu * eF - C(3) * uF);
      const C FA = w * (C(3) * eF);
      const C dp = -sp * (C(0.5) * Ps[k] - Se) + kp * FS;
      const C dm = -sm * (C(0.5) * Md[k] - Ao) + km * FA;
      h[i] += dp + dm;
      h[i + 1] += dp - dm;
    }
  } else {
    // non-equilibrium part and Guo's forcing term per direction
    C fneq[Q], Fh[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) {
      const C eu = C(L::ex(i)) * ux + C(L::ey(i)) * uy + C(L::ez(i)) * uz;
      const C eF = C(L::ex(i)) * Fx + C(L::ey(i)) * Fy + C(L::ez(i)) * Fz;
      const C w = (C)wgt<Q>(i);
      const C heq = w * (drho + rho * (C(3) * eu + C(4.5) * eu * eu - C(1.5) * uu));
      fneq[i] = h[i] - heq;
      Fh[i] = w * (C(3) * (eF - uF) + C(9) * eu * eF);
    }
    // general diagonal S: dm_k = -s_k (m - m_eq)_k + (1 - s_k/2) (M F)_k,
    // conserved rows: density 0, momentum F; then h += M^-1 dm.  The sparse
    // integer products are expanded at compile time (mrt_rows, mrt_cols):
    // only the nonzero entries of M become multiply-adds.
    C dmn[Q];
    mrt_rows<Q, C>(fneq, Fh, a, Fx, Fy, Fz, dmn, std::make_integer_sequence<int, Q>{});
    mrt_cols<Q, C>(dmn, h, std::make_integer_sequence<int, Q>{});
  }

  // The relaxation is compiled with contraction allowed; an empty asm makes
  // every post-collision value opaque, so that what follows (the store, and
  // in one variant a copy to LDS) cannot change how the compiler fuses the
  // arithmetic before it: every sweep variant rounds the same way.
#pragma unroll
  for (int i = 0; i < Q; i++) asm("" : "+v"(h[i]));
  // the block writes Q contiguous runs of kTile values per tile
  uint64_t base;
  if constexpr (IDX32 != 0) base = pidx32<Q>(0, n);
  else base = pidx<Q>(0, n);
  bool sr = false;
  uint32_t hsr = 0;
  if constexpr (sizeof(S) == 2) {
    sr = a.sr != 0;
    if (sr) hsr = hash32(n ^ a.seed);
  }
#pragma unroll
  for (int i = 0; i < Q; i++) {
    const S sv = store_value<S, C>(h[i], sr, sr ? sr_bits(hsr, i) : 0u);
    if (NT) __builtin_nontemporal_store(sv, B + base + (uint64_t)i * kTile);
    else B[base + (uint64_t)i * kTile] = sv;
    if (KEEP && i > 0 && keep) keep[i - 1] = sv;
  }
}

// Record of the lane's link j (< total) of this wavefront's CPT segments.
template <typename C, int CPT>
__device__ __forceinline__ uint32_t link_pos(const uint32_t (&first)[CPT], const uint32_t (&cnt)[CPT], uint32_t j,
                                             int &c) {
  c = 0;
  if (CPT == 2 && j >= cnt[0]) {
    c = 1;
    return first[CPT - 1] + (j - cnt[0]);
  }
  return first[0] + j;
}

// One link of sweep_links: lane link at record p, addressing words hd,
// segment c.  The populations are gathered first and the rest of the record
// is read after them, so that no wait separates the gathers from the pulls.
template <int Q, typename S, int CPT>
__device__ __forceinline__ void sweep_link_one(const S *A, const SweepLinkArgs &la, uint32_t p, uint4 hd, int c,
                                               S (*tab)[64 * (Q - 1)], uint32_t (*mask)[64]) {
  using C = typename Store<S>::C;
  const LinkRec<C> *rec = static_cast<const LinkRec<C> *>(la.rec);
  C *io = static_cast<C *>(la.io);
  S *dst = const_cast<S *>(A);
  const uint32_t rn = hd.x, rnff = hd.y, rnfff = hd.z;
  const int kind = (int)(hd.w & 255u), i = (int)(hd.w >> 8), ib = opp(i);
  const C hb_f = Store<S>::ld(A + pidx<Q>(ib, rn));
  const C hb_ff =
      (kind == LK_Q2_NEAR || kind == LK_Q1_NEAR || kind == LK_YU) ? Store<S>::ld(A + pidx<Q>(ib, rnff)) : C(0);
  const C hb_fff = (kind == LK_Q2_NEAR || kind == LK_YU) ? Store<S>::ld(A + pidx<Q>(ib, rnfff)) : C(0);
  const C hs_f = (kind == LK_Q2_FAR || kind == LK_Q1_FAR || kind == LK_YU) ? Store<S>::ld(A + pidx<Q>(i, rn)) : C(0);
  const C hs_ff = (kind == LK_Q2_FAR || kind == LK_YU) ? Store<S>::ld(A + pidx<Q>(i, rnff)) : C(0);
  const LinkRec<C> &r = rec[p];
  const LinkCoef<C> k{kind, r.k1, r.k2, r.k3, r.k4, 1.0};
  // (no Zhao-Yong links here: the table never holds them)
  const S v = store_value<S, C>(link_value<C>(k, r.B, hb_f, hb_ff, hb_fff, hs_f, hs_ff, C(0)), la.sr != 0,
                                la.sr ? hash32((r.nb * 32u + (uint32_t)i) ^ la.lseed) >> 19 : 0u);
  if (la.ghost) dst[pidx<Q>(i, r.nb)] = v;
  io[r.l] = (C)v;
  io[la.stride + r.l] = hb_f;
  const uint32_t o = rn & 63u;
  tab[c][o * (Q - 1) + (i - 1)] = v;
  atomicOr(&mask[c][o], 1u << i);
}

// Boundary links of this wavefront's cells (CPT segments of 64 cells, one
// cell of each per lane; the link records of segment c are rec[first[c] ..
// first[c] + cnt[c] - 1]): the lanes take the links one each and evaluate them
// on the source array; each value goes to the owning lane through LDS (tab,
// one row of Q-1 directions per cell, and a direction mask) and replaces the
// pulled value there (the solid-node slot it was pulled from is stale).  With
// la.ghost it is also written to that slot (read by no other node in this
// sweep), and the link's incoming and outgoing values are kept for its force.
// first, cnt, total are wavefront-uniform.  head0: the addressing words of the
// lane's first link, fetched before the cells' pulls were issued (loads
// complete in order, so a record read after the pulls would hold the link
// loads back until every pull had arrived).
template <int Q, typename S, int CPT>
__device__ __forceinline__ void sweep_links(const S *A, const SweepLinkArgs &la, const uint32_t (&first)[CPT],
                                            const uint32_t (&cnt)[CPT], uint32_t total, uint4 head0,
                                            S (&h)[CPT][Q], S (*tab)[64 * (Q - 1)], uint32_t (*mask)[64]) {
  using C = typename Store<S>::C;
  const int lane = threadIdx.x & 63;
  const LinkRec<C> *rec = static_cast<const LinkRec<C> *>(la.rec);
#pragma unroll
  for (int c = 0; c < CPT; c++) mask[c][lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  // the first 64 links from the addressing words fetched before the pulls (a
  // branch joining them with a later load would make the compiler wait for
  // every pull before the first gather); further ones, rare, one load each
  if ((uint32_t)lane < total) {
    int c;
    const uint32_t p = link_pos<C, CPT>(first, cnt, (uint32_t)lane, c);
    sweep_link_one<Q, S, CPT>(A, la, p, head0, c, tab, mask);
  }
  for (uint32_t b = 64; b < total; b += 64) {
    const uint32_t j = b + lane;
    if (j < total) {
      int c;
      const uint32_t p = link_pos<C, CPT>(first, cnt, j, c);
      sweep_link_one<Q, S, CPT>(A, la, p, LinkRec<C>::head(rec + p), c, tab, mask);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int c = 0; c < CPT; c++) {
    const uint32_t m = mask[c][lane];
    if (m) {
#pragma unroll
      for (int d = 1; d < Q; d++)
        if (m & (1u << d)) h[c][d] = tab[c][lane * (Q - 1) + (d - 1)];
    }
  }
}

// Zhao-Yong links of this wavefront's cells at the step this sweep computes
// (Eq. 16 reads x_f only): once the wavefront's cells are relaxed, the lanes
// take the links one each, read the post-collision h_i(x_f) and h_ibar(x_f)
// from the cells' LDS rows (tab: Q-1 stored values per cell, as written to B)
// and h_ibar(x_f) before the collision from A at x_ff (the value the cell
// pulled; no one writes A during the sweep), and write the unknown into the
// solid node's slot of B, which the next sweep pulls.  These are the values
// the bounce-back kernel reads, so both give the same bits.
template <int Q, typename S, int CPT>
__device__ __forceinline__ void sweep_links_zy(const S *A, S *B, const SweepLinkArgs &la, const uint32_t (&first)[CPT],
                                               const uint32_t (&cnt)[CPT], uint32_t total,
                                               const S (*tab)[64 * (Q - 1)]) {
  using C = typename Store<S>::C;
  const int lane = threadIdx.x & 63;
  const LinkRec<C> *rec = static_cast<const LinkRec<C> *>(la.rec);
  C *io = static_cast<C *>(la.io);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint32_t b = 0; b < total; b += 64) {
    const uint32_t j = b + lane;
    if (j < total) {
      int c;
      const uint32_t p = link_pos<C, CPT>(first, cnt, j, c);
      const LinkRec<C> r = rec[p];
      const int kind = (int)(r.kind_dir & 255u), i = (int)(r.kind_dir >> 8), ib = opp(i);
      const uint32_t o = r.n & 63u;
      const C hs_f = (C)tab[c][o * (Q - 1) + (i - 1)];
      const C hb_f = (C)tab[c][o * (Q - 1) + (ib - 1)];
      const C hpre = Store<S>::ld(A + pidx<Q>(ib, r.nff));
      const LinkCoef<C> k{kind, r.k1, r.k2, r.k3, r.k4, 1.0};
      const S v = store_value<S, C>(link_value<C>(k, r.B, hb_f, C(0), C(0), hs_f, C(0), hpre), la.sr != 0,
                                    la.sr ? hash32((r.nb * 32u + (uint32_t)i) ^ la.lseed) >> 19 : 0u);
      B[pidx<Q>(i, r.nb)] = v;
      io[r.l] = (C)v;
      io[la.stride + r.l] = hb_f;
    }
  }
}

// One block sweeps sweep_cpt tiles (group blk): every thread pulls its cell
// of each tile before relaxing any, so that half-precision storage keeps as
// many bytes in flight per wavefront as single precision.  INL: 0 no link
// evaluation, 1 the links of the previous step replace pulled values, 2 the
// Zhao-Yong links of this step follow the relaxation.
template <int Q, int COLL, typename S, int FLAGS, int NT, int INL, int IDX32 = 0, int BND = 0>
__device__ __forceinline__ void sweep_body(const S *__restrict__ A, S *__restrict__ B, const SweepArgs &a,
                                           const SweepLinkArgs *la, uint32_t blk) {
  constexpr int CPT = sweep_cpt_of<S>();
  uint32_t n[CPT];
  uint8_t fl[CPT];
  bool act[CPT];
#pragma unroll
  for (int c = 0; c < CPT; c++) {
    n[c] = (blk * CPT + c) * kBlock + threadIdx.x;
    act[c] = n[c] < a.N;
    fl[c] = (FLAGS && act[c]) ? a.flags[n[c]] : (uint8_t)0;
  }
  uint32_t first[CPT], cnt[CPT], total = 0;
  if constexpr (INL != 0) {
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < CPT; c++) {
      const uint32_t seg = __builtin_amdgcn_readfirstlane((blk * CPT + c) * (kBlock / 64) + (uint32_t)w);
      SegLink sg{0u, 0u};
      if (seg < la->nseg) sg = load_uniform(&la->seg_link[seg]);
      first[c] = sg.first;
      cnt[c] = sg.count;
      total += sg.count;
    }
  }
  // the addressing words of each lane's first link, ahead of the pulls
  uint4 head0 = {0u, 0u, 0u, 0u};
  if constexpr (INL == 1) {
    const uint32_t lane = threadIdx.x & 63u;
    if (lane < total) {
      int c;
      head0 = LinkRec<typename Store<S>::C>::head(
          static_cast<const LinkRec<typename Store<S>::C> *>(la->rec) +
          link_pos<typename Store<S>::C, CPT>(first, cnt, lane, c));
    }
  }
  // the loads are not predicated (a branch around them would make the
  // compiler wait for one cell's loads before issuing the next cell's):
  // cells past the end load cell N-1, solid nodes load and discard
  S r[CPT][Q];
  uint32_t inm[CPT], uo_at[CPT];
#pragma unroll
  for (int c = 0; c < CPT; c++) {
    if constexpr (BND != 0) inm[c] = sweep_pull_bnd<Q, S, IDX32>(A, a, act[c] ? n[c] : a.N - 1, r[c], uo_at[c]);
    else {
      sweep_pull<Q, S, IDX32>(A, a, act[c] ? n[c] : a.N - 1, r[c]);
      inm[c] = 0u;
      uo_at[c] = ~0u;
    }
  }
#pragma unroll
  for (int c = 0; c < CPT; c++) act[c] = act[c] && !(fl[c] & F_SOLID);  // nothing is stored for solid nodes
  if constexpr (INL == 1) {
    __shared__ S tab[kBlock / 64][CPT][64 * (Q - 1)];
    __shared__ uint32_t msk[kBlock / 64][CPT][64];
    const int w = threadIdx.x >> 6;
    if (total) sweep_links<Q, S, CPT>(A, *la, first, cnt, total, head0, r, tab[w], msk[w]);
  }
  if constexpr (INL == 2) {
    // wavefronts with links keep every cell's stored values in LDS for them
    __shared__ S ztab[kBlock / 64][CPT][64 * (Q - 1)];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < CPT; c++)
      if (act[c])
        sweep_relax<Q, COLL, S, FLAGS, NT, IDX32, true, BND != 0>(
            B, a, n[c], fl[c], r[c], total ? &ztab[w][c][lane * (Q - 1)] : nullptr, inm[c], uo_at[c]);
    if (total) sweep_links_zy<Q, S, CPT>(A, B, *la, first, cnt, total, ztab[w]);
  } else {
#pragma unroll
    for (int c = 0; c < CPT; c++)
      if (act[c]) sweep_relax<Q, COLL, S, FLAGS, NT, IDX32, false, BND != 0>(B, a, n[c], fl[c], r[c], nullptr, inm[c], uo_at[c]);
  }
}

// Waves per SIMD the sweep keeps when it also evaluates boundary links: the
// occupancy of the plain two-rate sweep, which the link branch must not
// lower (the general-rate relaxation has no such bound).
template <typename S, int COLL, int INL>
constexpr int sweep_min_waves() {
  return (!INL || COLL == COLL_MRT) ? 1 : (sizeof(S) == 4 ? 8 : (sizeof(S) == 2 ? 5 : 4));
}

template <int Q, int COLL, typename S, int FLAGS, int NT, int INL, int IDX32, int BND = 0>
__global__ __launch_bounds__(kBlock, (sweep_min_waves<S, COLL, INL>())) void k_sweep(const S *__restrict__ A,
                                                                             S *__restrict__ B, SweepArgs a,
                                                                             SweepLinkArgs la) {
  // leading blocks, dispatched first and finished long before the sweep's tail:
  // bounce-back force sums of earlier steps, or the IBM force of this one
  // policy: XCD-contiguous tile order (workgroups are dealt to the 8 XCDs
  // round-robin; this gives each XCD's L2 a contiguous range of tiles)
  uint32_t blk = a.xcd ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  if (blk < a.rblocks) {
    ft_reduce_waves(a.ft, blk);
    return;
  }
  blk -= a.rblocks;
  if (INL) {
    if (blk < la.cblocks) {
      chunk_sum_waves<Q>(la.cs, blk);
      return;
    }
    blk -= la.cblocks;
  }
  if (blk < a.iblocks) {
    ibm_ft_body(a.ift, (int)blk);
    return;
  }
  sweep_body<Q, COLL, S, FLAGS, NT, INL, IDX32, BND>(A, B, a, &la, blk - a.iblocks);
}

}  // namespace lbm
