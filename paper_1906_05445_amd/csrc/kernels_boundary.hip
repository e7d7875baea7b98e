// kernels_boundary.hip -- node classification, boundary-link builder,
// interpolated bounce-back with momentum-exchange force/torque, refill of
// uncovered nodes (Sec. 2.2, Eq. 10, Eq. 11, Eq. 17, Sec. 3.2).
//
// Links are built per solid over the solid's bounding box (all cells within
// R + 2 of its centre), so each solid's links are contiguous; the box is
// walked in a fixed order, which makes the link list, and every reduction
// over it, deterministic.  A link (x_f, i) joins a fluid node x_f to the
// solid node x_b = x_f - e_i; the bounce-back kernel writes the unknown
// f_i(x_f, t+1) into slot i of x_b, exactly where the next pull sweep at x_f
// looks for population i.  For fixed solids the sweep evaluates most steps'
// links itself, from per-segment link lists and a per-call link table built
// here (the same link arithmetic, lbm_ibb.hpp).
#include <algorithm>

#include "lbm_args.hpp"
#include "lbm_ibb.hpp"

namespace lbm {


__device__ inline void xyz_of(uint32_t n, const GeoArgs &a, int &x, int &y, int &z) {
  const uint32_t yz = fdiv(n, a.fx);
  x = (int)(n - yz * (uint32_t)a.b.nx);
  z = (int)fdiv(yz, a.fy);
  y = (int)(yz - (uint32_t)z * (uint32_t)a.b.ny);
}
__device__ inline uint32_t id_of(int x, int y, int z, const GeoArgs &a) {
  return (uint32_t)wrapi(x, a.b.nx) +
         (uint32_t)a.b.nx * ((uint32_t)wrapi(y, a.b.ny) + (uint32_t)a.b.ny * (uint32_t)wrapi(z, a.b.nz));
}

// Direction i (runtime) of the velocity set.
template <int Q>
__device__ inline void dir_of(int i, int &ex, int &ey, int &ez) {
  ex = ey = ez = 0;
#pragma unroll
  for (int k = 1; k < Q; k++)
    if (k == i) {
      ex = Lat<Q>::ex(k);
      ey = Lat<Q>::ey(k);
      ez = Lat<Q>::ez(k);
    }
}

// Box of solid s at time t: cell (lx, ly, lz) of the box -> lattice cell.
// Also returns the centre at t.
__device__ inline void box_origin(const DevSolid &s, const GeoArgs &a, int o[3], double c[3]) {
  solid_centre(s, a.t, a.b, c);
  if (!s.moving) {
    o[0] = s.box0[0];
    o[1] = s.box0[1];
    o[2] = s.box0[2];
    return;
  }
  for (int k = 0; k < 3; k++) o[k] = s.full[k] ? 0 : (int)floor(c[k] - s.R) - 2;
}

// Half-widths of the surface bands: a node changes classification between
// t and t+1 only within |U| of the surface, and the previous step's changes
// lie within 2|U| of the surface at t+1; a link (x_f, i) has its solid node
// x_f - e_i inside, so x_f lies within |e_i| <= sqrt(2) of the surface.
__device__ inline double move_band(const DevSolid &s) {
  return 2.0 * sqrt(s.U[0] * s.U[0] + s.U[1] * s.U[1] + s.U[2] * s.U[2]) + 0.5;
}
constexpr double kLinkBand = 1.5;
__device__ inline bool box_cell(const DevSolid &s, const int o[3], uint32_t bi, const GeoArgs &a, int &x, int &y,
                                int &z) {
  if (bi >= s.box_cells) return false;
  const uint32_t r = fdiv(bi, s.fex), lz = fdiv(bi, s.fexy);
  const uint32_t lx = bi - r * (uint32_t)s.ext[0], ly = r - lz * (uint32_t)s.ext[1];
  x = wrapi(o[0] + (int)lx, a.b.nx);
  y = wrapi(o[1] + (int)ly, a.b.ny);
  z = wrapi(o[2] + (int)lz, a.b.nz);
  return true;
}

// classification of one cell against all solids (first match wins)
__device__ inline int classify_cell(const GeoArgs &a, int x, int y, int z) {
  for (int k = 0; k < a.nsolid; k++) {
    const DevSolid s = load_uniform(&a.solids[k]);
    double c[3];
    solid_centre(s, a.t, a.b, c);
    if (inside_solid(s, c, x, y, z, a.b)) return k;
  }
  return -1;
}
__device__ inline uint8_t flags_for(const GeoArgs &a, int k, uint8_t old_ibm) {
  uint8_t f = old_ibm;
  if (k >= 0) {
    if (a.ibb) f |= F_SOLID;
    if (a.fluid_only) f |= F_NOBODY;
  }
  return f;
}

// Full classification (setup): previous geometry := current.
__global__ void k_classify_full(uint8_t *flags, uint16_t *owner, uint16_t *owner_prev, GeoArgs a) {
  const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= a.N) return;
  int x, y, z;
  xyz_of(n, a, x, y, z);
  const int k = classify_cell(a, x, y, z);
  uint8_t f = flags_for(a, k, flags[n] & F_IBM);
  if (f & F_SOLID) f |= F_WAS_SOLID;
  flags[n] = f;
  owner[n] = k < 0 ? 0xFFFF : (uint16_t)k;
  owner_prev[n] = owner[n];
}

// Moving solids, phase 1 over their boxes: remember the current geometry.
// (The refill list of a step starts empty: the link emit pass of the step
// before, the last reader of its count misc[3], clears it.  The overflow flag
// misc[4] stays set until lbm_set_solids.)
__device__ inline void classify_keep_body(const LinkArgs &a, uint32_t bx, int s) {
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  if (!sd.moving) return;
  int o[3], x, y, z;
  double c[3];
  box_origin(sd, a.g, o, c);
  if (!box_cell(sd, o, bx * blockDim.x + threadIdx.x, a.g, x, y, z)) return;
  if (!near_surface(sd, c, x, y, z, a.g.b, move_band(sd))) return;  // unchanged since the last step
  const uint32_t n = id_of(x, y, z, a.g);
  const uint8_t f = a.flags[n];
  a.flags[n] = (f & F_SOLID) ? (f | F_WAS_SOLID) : (uint8_t)(f & ~F_WAS_SOLID);
  a.owner_prev[n] = a.owner[n];
}
// Moving solids, phase 2 over their boxes: classify at the new time.
__device__ inline void classify_box_body(const LinkArgs &a, uint32_t bx, int s) {
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  if (!sd.moving) return;
  int o[3], x, y, z;
  double c[3];
  box_origin(sd, a.g, o, c);
  if (!box_cell(sd, o, bx * blockDim.x + threadIdx.x, a.g, x, y, z)) return;
  if (!near_surface(sd, c, x, y, z, a.g.b, move_band(sd))) return;  // cannot change this step
  const uint32_t n = id_of(x, y, z, a.g);
  const int k = classify_cell(a.g, x, y, z);
  const uint8_t old = a.flags[n];
  const uint8_t now = (uint8_t)(flags_for(a.g, k, old & F_IBM) | (old & F_WAS_SOLID));
  a.flags[n] = now;
  a.owner[n] = k < 0 ? 0xFFFF : (uint16_t)k;
  // uncovered by solid s (the box of its previous owner lists it once): refill
  if ((now & F_WAS_SOLID) && !(now & F_SOLID) && a.owner_prev[n] == (uint16_t)s) {
    const uint32_t at = atomicAdd(&a.misc[3], 1u);
    if (at < a.max_refill) a.refill_list[at] = ((uint64_t)(uint32_t)s << 32) | n;
    else a.misc[4] = 1u;
  }
  // covered by solid s (its box lists it once): its momentum goes to s
  if (a.cu && !(now & F_WAS_SOLID) && (now & F_SOLID) && k == s) {
    const uint32_t at = atomicAdd(&a.misc[3], 1u);
    if (at < a.max_refill) a.refill_list[at] = (1ull << 63) | ((uint64_t)(uint32_t)s << 32) | n;
    else a.misc[4] = 1u;
  }
}
__global__ void k_classify_keep(LinkArgs a) { classify_keep_body(a, blockIdx.x, blockIdx.y); }
__global__ void k_classify_box(LinkArgs a) { classify_box_body(a, blockIdx.x, blockIdx.y); }
// One solid: no other solid's box can meet this one's, so each box cell is one
// thread's in both phases, which then run back to back in that thread.
__global__ void k_classify_one(LinkArgs a) {
  classify_keep_body(a, blockIdx.x, 0);
  classify_box_body(a, blockIdx.x, 0);
}

void launch_classify(lbm_ctx *c, int64_t t, bool full);

// ----------------------------------------------------------------------------
// link builder
// ----------------------------------------------------------------------------

// Links of cell n whose solid node belongs to solid s; bit i of the result.
template <int Q>
__device__ inline uint32_t link_mask(const LinkArgs &a, int s, int x, int y, int z) {
  // all 2(Q-1) loads are independent: issue them together
  uint8_t f[Q];
  uint16_t o[Q];
#pragma unroll
  for (int i = 1; i < Q; i++) {
    const uint32_t nb = id_of(x - Lat<Q>::ex(i), y - Lat<Q>::ey(i), z - Lat<Q>::ez(i), a.g);
    f[i] = a.flags[nb];
    o[i] = a.owner[nb];
  }
  uint32_t m = 0;
#pragma unroll
  for (int i = 1; i < Q; i++)
    if ((f[i] & F_SOLID) && o[i] == (uint16_t)s) m |= 1u << i;
  return m;
}

// Refill of a node uncovered this step (Sec. 3.2): f = f_eq(rho_bar, u_w)
// with rho_bar the mean density at t of the neighbours that are fluid
// before and after the move (1 if none); written into the slots the node
// pulls from, P_i(x - e_i).  One wavefront per node, lane i gathering the
// density of neighbour x + e_i.  Refills touch disjoint slots (a node's own
// pull slots belong to other cells than those its neighbours' densities are
// gathered from), so the list order does not matter.
// Fixed-point add of a solid's covering / uncovering force m and torque r x m
// (sign -1: taken from the solid).
__device__ inline void cu_add(unsigned long long *cu, int s, const double m[3], const double r[3], double sign) {
  const double v[6] = {m[0], m[1], m[2], r[1] * m[2] - r[2] * m[1], r[2] * m[0] - r[0] * m[2],
                       r[0] * m[1] - r[1] * m[0]};
  for (int k = 0; k < 6; k++)
    atomicAdd(cu + (uint64_t)s * 6 + k, (unsigned long long)__double2ll_rn(sign * v[k] * cu_scale(k)));
}

// A node the solid covered this step (list entry with bit 63): its momentum,
// sum_i f_i e_i of the populations that streamed into it (pulled from the
// post-collision array, ghost values included), goes to the solid, with the
// torque about the solid's centre at t+1.  One wavefront, lane i pulling f_i.
template <int Q, typename S>
__device__ void cover_wave(const LinkArgs &a, int s, uint32_t n) {
  using L = Lat<Q>;
  const S *P = static_cast<const S *>(a.post);
  int x, y, z;
  xyz_of(n, a.g, x, y, z);
  const int lane = (int)(threadIdx.x & 63);
  double m[3] = {0.0, 0.0, 0.0};
  if (lane < Q) {
    int ex, ey, ez;
    dir_of<Q>(lane, ex, ey, ez);
    const double h = (double)Store<S>::ld(P + pidx<Q>(lane, id_of(x - ex, y - ey, z - ez, a.g)));
    m[0] = ex * h;  // sum_i h_i e_i = sum_i f_i e_i (sum_i w_i e_i = 0)
    m[1] = ey * h;
    m[2] = ez * h;
  }
  for (int k = 0; k < 3; k++) m[k] = __shfl(wave_sum(m[k]), 0, 64);
  if (lane != 0) return;
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  double c[3], r[3];
  solid_centre(sd, a.g.t, a.g.b, c);
  lever_arm(sd, c, (double)x, (double)y, (double)z, a.g.b, r);
  cu_add(a.cu, s, m, r, 1.0);
}

template <int Q, typename S>
__device__ void refill_wave(const LinkArgs &a, uint64_t entry) {
  using L = Lat<Q>;
  S *P = static_cast<S *>(a.post);
  const int s = __builtin_amdgcn_readfirstlane((int)((entry >> 32) & 0x7fffffffull));
  const uint32_t n = (uint32_t)entry;
  if (entry >> 63) {
    cover_wave<Q, S>(a, s, n);
    return;
  }
  int x, y, z;
  xyz_of(n, a.g, x, y, z);
  const int lane = (int)(threadIdx.x & 63);
  double r = 0.0;
  bool use = false;
  if (lane >= 1 && lane < Q) {
    int ex, ey, ez;
    dir_of<Q>(lane, ex, ey, ez);
    const int yx = x + ex, yy = y + ey, yzz = z + ez;
    use = !(a.flags[id_of(yx, yy, yzz, a.g)] & (F_SOLID | F_WAS_SOLID));
    if (use) {
#pragma unroll
      for (int j = 0; j < Q; j++)
        r += (double)Store<S>::ld(P + pidx<Q>(j, id_of(yx - L::ex(j), yy - L::ey(j), yzz - L::ez(j), a.g)));
    }
  }
  const int cnt = __popcll(__ballot(use));
  const double sum = __shfl(wave_sum(use ? r : 0.0), 0, 64);  // density deviations rho - 1
  const double drb = cnt ? sum / cnt : 0.0, rb = 1.0 + drb;
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  double c[3], lv[3], uw[3];
  solid_centre(sd, a.g.t, a.g.b, c);
  lever_arm(sd, c, (double)x, (double)y, (double)z, a.g.b, lv);
  wall_vel(sd, lv, uw);
  if (lane < Q) {
    int ex, ey, ez;
    dir_of<Q>(lane, ex, ey, ez);
    const double uu = uw[0] * uw[0] + uw[1] * uw[1] + uw[2] * uw[2];
    const double eu = ex * uw[0] + ey * uw[1] + ez * uw[2];
    double w = 0.0;
#pragma unroll
    for (int k = 0; k < Q; k++)
      if (k == lane) w = wgt<Q>(k);
    const double heq = w * (drb + rb * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
    Store<S>::st(P + pidx<Q>(lane, id_of(x - ex, y - ey, z - ez, a.g)), (typename Store<S>::C)heq);
  }
  // uncovering: the refilled momentum rho_bar u_w comes out of the solid
  if (a.cu && lane == 0) {
    const double m[3] = {rb * uw[0], rb * uw[1], rb * uw[2]};
    cu_add(a.cu, s, m, lv, -1.0);
  }
}

template <int Q>
__device__ inline void link_count_body(const LinkArgs &a, uint32_t bx, int s) {
  __shared__ double lds[16];
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  int o[3], x, y, z;
  double c[3];
  box_origin(sd, a.g, o, c);
  uint32_t m = 0;
  const uint32_t bi = bx * kBlock + threadIdx.x;
  const bool in = box_cell(sd, o, bi, a.g, x, y, z);
  if (in && near_surface(sd, c, x, y, z, a.g.b, kLinkBand)) {
    const uint32_t n = id_of(x, y, z, a.g);
    const uint8_t f = a.flags[n];
    if (!(f & F_SOLID)) m = link_mask<Q>(a, s, x, y, z);
  }
  if (a.masks && in) a.masks[sd.mask_off + bi] = m;  // read back by the emit pass
  const double tot = block_sum((double)__popc(m), lds);
  if (threadIdx.x == 0 && bx < a.max_box_chunks) a.box_counts[(uint64_t)s * a.max_box_chunks + bx] = (uint32_t)tot;
}
template <int Q>
__global__ __launch_bounds__(kBlock) void k_link_count(LinkArgs a) {
  link_count_body<Q>(a, blockIdx.x, blockIdx.y);
}

// Refill and link count of a single context in one launch: both read only the
// finished classification (the refill writes populations, the count flags and
// owners it does not touch).  Blocks 0 .. kRefillBlocks-1 walk the refill list,
// the others are the count pass's (box chunk, solid) units.
constexpr uint32_t kRefillBlocks = 64;
template <int Q, typename S>
__global__ __launch_bounds__(kBlock) void k_refill_count(LinkArgs a) {
  if (blockIdx.x < kRefillBlocks) {
    const uint32_t cnt = min(a.misc[3], a.max_refill);
    for (uint32_t e = blockIdx.x * 4 + (threadIdx.x >> 6); e < cnt; e += kRefillBlocks * 4)
      refill_wave<Q, S>(a, a.refill_list[e]);
    return;
  }
  const uint32_t u = blockIdx.x - kRefillBlocks, per = a.max_box_chunks;
  link_count_body<Q>(a, u % per, (int)(u / per));
}

// One block: exclusive scan of the per-(solid, box chunk) counts, then the
// per-solid link ranges and chunk bases of the bounce-back kernel.
__device__ inline void link_scan_body(const LinkArgs &a, int nsolid) {
  __shared__ uint32_t part[1024];
  const uint32_t total = (uint32_t)nsolid * a.max_box_chunks;
  const uint32_t per = (total + blockDim.x - 1) / blockDim.x;
  const uint32_t b0 = threadIdx.x * per, b1 = min(total, b0 + per);
  uint32_t s = 0;
  for (uint32_t k = b0; k < b1; k++) s += a.box_counts[k];
  // exclusive scan of the per-thread sums over the block (integer: any order
  // gives the same offsets): inclusive within each wavefront, then the
  // wavefront totals
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t inc = s;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t v = __shfl_up(inc, off, 64);
    if (lane >= off) inc += v;
  }
  if (lane == 63) part[wv] = inc;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int k = 0; k < nw; k++) {
    const uint32_t v = part[k];
    if (k < wv) base += v;
    all += v;
  }
  if (threadIdx.x == 0) {
    a.misc[0] = all;
    a.misc[1] = all > a.max_links ? 1u : 0u;
  }
  uint32_t run = base + inc - s;
  for (uint32_t k = b0; k < b1; k++) {
    const uint32_t v = a.box_counts[k];
    a.box_offsets[k] = run;
    run += v;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t cb = 0;
    for (int sd = 0; sd < nsolid; sd++) {
      const uint32_t first = a.box_offsets[(uint64_t)sd * a.max_box_chunks];
      const uint32_t last = sd + 1 < nsolid ? a.box_offsets[(uint64_t)(sd + 1) * a.max_box_chunks] : a.misc[0];
      SolidLinks L;
      L.start = first;
      L.count = last - first;
      L.chunk_base = cb;
      L.nchunks = (L.count + kLinkChunk - 1) / kLinkChunk;
      cb += L.nchunks;
      a.sl[sd] = L;
    }
  }
}
__global__ void k_link_scan(LinkArgs a, int nsolid) { link_scan_body(a, nsolid); }

// Exclusive prefix sum over the threads of a 256-thread block, in thread
// order; *total receives the block sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds4, uint32_t *total) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  __syncthreads();  // lds4 free (previous use finished)
  if (lane == 63) lds4[wv] = inc;
  __syncthreads();
  uint32_t base = 0, all = 0;
  for (int k = 0; k < kBlock / 64; k++) {
    if (k < wv) base += lds4[k];
    all += lds4[k];
  }
  *total = all;
  return base + inc - v;
}

constexpr int kEmitWindow = 1024;  // links of one unit staged in LDS at a time

// Links of one unit (256 box cells): each thread stages its links (cell,
// direction) in LDS at their place in the unit's order (by cell, then
// direction), then the whole block computes q and the x_ff / x_fff bits, one
// link per thread, and writes them.
// Sum over the threads of a 256-thread block (every thread gets it).
__device__ inline uint32_t block_sum_u32(uint32_t v, uint32_t *lds4) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if (lane == 0) lds4[wv] = v;
  __syncthreads();
  uint32_t all = 0;
  for (int k = 0; k < kBlock / 64; k++) all += lds4[k];
  return all;
}

// ONE: a context with a single solid, whose link offsets need no scan pass:
// each block sums the counts of the box chunks before its own, and block 0
// also writes the solid's link range and the total (what the scan writes).
template <int Q, bool ONE = false>
__device__ inline void link_emit_body(const LinkArgs &a, uint32_t bx, int s) {
  if (bx == 0 && s == 0 && threadIdx.x == 0) a.misc[3] = 0;  // the next step's refill list starts empty
  __shared__ uint32_t wsum[kBlock / 64];
  __shared__ uint32_t wsum2[kBlock / 64];
  __shared__ uint32_t st_cell[kEmitWindow];
  __shared__ uint8_t st_dir[kEmitWindow];
  const DevSolid sd = load_uniform(&a.g.solids[s]);
  int o[3], x = 0, y = 0, z = 0;
  double c[3];
  box_origin(sd, a.g, o, c);
  uint32_t m = 0, n = 0;
  const uint32_t bi = bx * kBlock + threadIdx.x;
  if (a.masks) {  // the count pass stored every box cell's mask
    if (box_cell(sd, o, bi, a.g, x, y, z)) {
      m = a.masks[sd.mask_off + bi];
      if (m) n = id_of(x, y, z, a.g);
    }
  } else if (box_cell(sd, o, bi, a.g, x, y, z) && near_surface(sd, c, x, y, z, a.g.b, kLinkBand)) {
    n = id_of(x, y, z, a.g);
    if (!(a.flags[n] & F_SOLID)) m = link_mask<Q>(a, s, x, y, z);
  }
  uint32_t total;
  const uint32_t before = block_exclusive_scan((uint32_t)__popc(m), wsum, &total);
  if (bx >= a.max_box_chunks) return;  // uniform over the block
  uint64_t base;
  if constexpr (ONE) {
    const uint32_t lim = bx == 0 ? a.max_box_chunks : bx;
    uint32_t v = 0;
    for (uint32_t k = threadIdx.x; k < lim; k += kBlock) v += a.box_counts[k];
    const uint32_t sum = block_sum_u32(v, wsum2);
    base = bx == 0 ? 0 : sum;
    if (bx == 0 && threadIdx.x == 0) {
      SolidLinks L;
      L.start = 0;
      L.count = sum;
      L.chunk_base = 0;
      L.nchunks = (sum + kLinkChunk - 1) / kLinkChunk;
      a.sl[0] = L;
      a.misc[0] = sum;
      a.misc[1] = sum > a.max_links ? 1u : 0u;
    }
  } else {
    base = a.box_offsets[(uint64_t)s * a.max_box_chunks + bx];
  }
  for (uint32_t w0 = 0; w0 < total; w0 += kEmitWindow) {
    uint32_t k = before, mm = m;
    while (mm) {
      const int i = __ffs(mm) - 1;
      mm &= mm - 1;
      if (k >= w0 && k < w0 + kEmitWindow) {
        st_cell[k - w0] = n;
        st_dir[k - w0] = (uint8_t)i;
      }
      k++;
    }
    __syncthreads();
    const uint32_t cnt = min(total - w0, (uint32_t)kEmitWindow);
    for (uint32_t j = threadIdx.x; j < cnt; j += kBlock) {
      const uint64_t pos = base + w0 + j;
      if (pos >= a.max_links) continue;
      const uint32_t cell = st_cell[j];
      const int i = st_dir[j];
      int ex, ey, ez, lx, ly, lz;
      dir_of<Q>(i, ex, ey, ez);
      xyz_of(cell, a.g, lx, ly, lz);
      const uint32_t ok1 = (a.flags[id_of(lx + ex, ly + ey, lz + ez, a.g)] & F_SOLID) ? 0u : 1u;
      const uint32_t ok2 = (a.flags[id_of(lx + 2 * ex, ly + 2 * ey, lz + 2 * ez, a.g)] & F_SOLID) ? 0u : 1u;
      a.link_cell[pos] = cell;
      a.link_meta[pos] = (uint32_t)i | (ok1 << 5) | (ok2 << 6) | ((uint32_t)s << 8);
      a.link_q[pos] = link_fraction(sd, c, lx, ly, lz, ex, ey, ez, a.g.b);
    }
    __syncthreads();
  }
}
template <int Q>
__global__ __launch_bounds__(kBlock) void k_link_emit(LinkArgs a) {
  link_emit_body<Q>(a, blockIdx.x, blockIdx.y);
}
template <int Q>
__global__ __launch_bounds__(kBlock) void k_link_emit_one(LinkArgs a) {
  link_emit_body<Q, true>(a, blockIdx.x, 0);
}

// ----------------------------------------------------------------------------
// interpolated bounce-back + momentum exchange (one thread per link)
// ----------------------------------------------------------------------------

// One wavefront per chunk of kLinkChunk links of one solid; each wave writes
// the chunk's force/torque partial (summed per solid in chunk order later).
// P: post-collision array of step t (receives the ghost values); pre: the
// array that step's sweep pulled from, where h_ibar(x_f, t) before the
// collision sits at x_ff (Zhao-Yong only; a fluid value, or the ghost value
// the previous step left there when x_ff is solid).
template <int Q, typename S>
__device__ inline void ibb_body(S *__restrict__ P, const S *__restrict__ pre, const IbbArgs &a, int64_t t,
                                uint32_t bx, int s) {
  const SolidLinks sl = a.sl[s];
  const int lane = threadIdx.x;
  const bool active = bx < sl.nchunks && (uint64_t)sl.chunk_base + bx < a.max_partials;
  if (active) {
    const uint32_t li = bx * kLinkChunk + lane;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // capacity overflow (reported by the host after the step) must not read out of bounds
    if (li < sl.count && (uint64_t)sl.start + li < a.max_links) {
      using C = typename Store<S>::C;
      const uint64_t l = (uint64_t)sl.start + li;
      const uint32_t n = a.link_cell[l], meta = a.link_meta[l];
      const double q = a.link_q[l];
      const int i = (int)(meta & 31u), ib = opp(i);
      const bool ffok = (meta >> 5) & 1u, fffok = (meta >> 6) & 1u;
      int x, y, z;
      xyz_of(n, a.g, x, y, z);
      const DevSolid sd = load_uniform(&a.g.solids[s]);
      double c[3];
      solid_centre(sd, t, a.g.b, c);
      const LinkGeo g = link_geo<Q>(i, q, sd, c, x, y, z, a.g.b);
      const LinkCoef<C> k = link_coef<C>(a.method, q, ffok, fffok);
      const C hb_f = Store<S>::ld(P + pidx<Q>(ib, n));
      const C hb_ff = ffok ? Store<S>::ld(P + pidx<Q>(ib, g.nff)) : C(0);
      const C hb_fff = fffok ? Store<S>::ld(P + pidx<Q>(ib, g.nfff)) : C(0);
      const C hs_f = Store<S>::ld(P + pidx<Q>(i, n));
      const C hs_ff = ffok ? Store<S>::ld(P + pidx<Q>(i, g.nff)) : C(0);
      const C hpre = k.kind == LK_ZY ? Store<S>::ld(pre + pidx<Q>(ib, g.nff)) : C(0);
      const S v = store_value<S, C>(link_value<C>(k, link_wall<C>(k, g.B), hb_f, hb_ff, hb_fff, hs_f, hs_ff, hpre),
                                    a.sr != 0, a.sr ? hash32((g.nb * 32u + (uint32_t)i) ^ sr_seed(t)) >> 19 : 0u);
      P[pidx<Q>(i, g.nb)] = v;
      link_ft((double)(C)v, (double)hb_f, g.a, g.b, g.d, g.r, acc);
    }
    for (int k = 0; k < 6; k++) {
      const double tot = wave_sum(acc[k]);
      if (lane == 0) a.partials[(uint64_t)(sl.chunk_base + bx) * 6 + k] = tot;
    }
  }
}
template <int Q, typename S>
__global__ __launch_bounds__(64) void k_ibb(S *__restrict__ P, const S *__restrict__ pre, IbbArgs a) {
  ibb_body<Q, S>(P, pre, a, a.g.t, blockIdx.x, blockIdx.y);
}

// Free solid k (Eq. 20, fluid density rho0 = 1, dt = 1) after the force and
// torque FT of step t are known: v' = v + (F + (rho_p - 1) V_p g) /
// (rho_p V_p), w' = w + T / I_p, centre' = centre + (v + v')/2 wrapped into
// the box; the state of step t is kept in cp, Up, Wp (the geometry of the
// collision at t, for the macroscopic readout).  Vector stores; kernels
// launched after it read the new table.  flag: set when a velocity component
// reaches half a cell per step.
__device__ inline void free_update_with(const DevSolid &s, DevSolid *solids, int k, const double FT[6],
                                        const Box3 &b, int64_t t, uint32_t *flag) {
#pragma clang fp contract(off)
  if (!s.free) return;
  const double m = s.rho_p * s.Vp;
  double c[3], vn[3], wn[3], cn[3];
  solid_centre(s, t, b, c);
  for (int a = 0; a < 3; a++) {
    if (s.fm) {
      // Eq. 23 (rho_f = 1, dt = 1): the inner fluid's inertia from the velocities of the step before
      vn[a] = s.U[a] + (s.Vp * (s.U[a] - s.Up[a]) + FT[a] + (s.rho_p - 1.0) * s.Vp * s.grav[a]) / m;
      wn[a] = s.W[a] + (s.Ip / s.rho_p * (s.W[a] - s.Wp[a]) + FT[3 + a]) / s.Ip;
    } else {
      vn[a] = s.U[a] + (FT[a] + (s.rho_p - 1.0) * s.Vp * s.grav[a]) / m;
      wn[a] = s.W[a] + FT[3 + a] / s.Ip;
    }
  }
  if (b.D == 2) {
    vn[2] = 0.0;
    wn[0] = 0.0;
    wn[1] = 0.0;
  }
  double dn[3];
  for (int a = 0; a < 3; a++) {
    cn[a] = c[a];
    dn[a] = s.dsp[a];
    if (a < b.D) {
      dn[a] = s.dsp[a] + 0.5 * (s.U[a] + vn[a]);
      const double L = (double)box_dim(b, a);
      double y = c[a] + 0.5 * (s.U[a] + vn[a]);
      if (!(y >= 0.0 && y < L)) {
        y = fmod(y, L);
        if (y < 0.0) y = y + L;
      }
      cn[a] = y;
    }
    if (fabs(vn[a]) >= 0.5) flag[0] = 1u;
  }
  DevSolid &o = solids[k];
  for (int a = 0; a < 3; a++) {
    o.cp[a] = c[a];
    o.Up[a] = s.U[a];
    o.Wp[a] = s.W[a];
    o.c0[a] = cn[a];
    o.U[a] = vn[a];
    o.W[a] = wn[a];
    o.dsp[a] = dn[a];
  }
  o.tref = t + 1;
}
__device__ inline void free_update_one(DevSolid *solids, int k, const double FT[6], const Box3 &b, int64_t t,
                                       uint32_t *flag) {
  const DevSolid s = solids[k];
  free_update_with(s, solids, k, FT, b, t, flag);
}

// IBM force/torque of step t of a free IBM solid (one block of 1024 threads
// per solid: the sum is latency-bound) and, by the thread that wrote them,
// its motion to t + 1 by Eq. 23.
constexpr int kFtFreeBlock = 1024;
// The solid's record is copied to LDS while the points are summed, the six
// sums share one pass of wave shuffles, and the totals reach the updating
// thread through LDS.
__global__ __launch_bounds__(kFtFreeBlock) void k_ibm_ft_free(IbmFtArgs f, DevSolid *solids, uint32_t *flag) {
#pragma clang fp contract(off)
  static_assert(sizeof(DevSolid) % 8 == 0 && sizeof(DevSolid) / 8 <= kFtFreeBlock, "solid record copy");
  __shared__ DevSolid sd;
  __shared__ double part[kFtFreeBlock / 64][6];
  __shared__ double tot[6];
  const int s = (int)blockIdx.x;
  if (threadIdx.x < sizeof(DevSolid) / 8)
    reinterpret_cast<uint64_t *>(&sd)[threadIdx.x] = reinterpret_cast<const uint64_t *>(solids + s)[threadIdx.x];
  double c[3] = {0.0, 0.0, 0.0};
  if (!f.mv) solid_centre(solids[s], f.t, f.b, c);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  const int64_t l0 = f.start[s], l1 = l0 + f.count[s];
  for (int64_t l = l0 + threadIdx.x; l < l1; l += blockDim.x) {
    double r[3], F[3];
    if (f.mv)
      for (int k = 0; k < 3; k++) r[k] = f.wts[l * 24 + 16 + k];
    else
      lever_arm(solids[s], c, f.X[l * 3], f.X[l * 3 + 1], f.X[l * 3 + 2], f.b, r);
    for (int k = 0; k < 3; k++) F[k] = -f.Fsum[l * 3 + k] * f.dV[l];
    acc[0] += F[0];
    acc[1] += F[1];
    acc[2] += F[2];
    acc[3] += r[1] * F[2] - r[2] * F[1];
    acc[4] += r[2] * F[0] - r[0] * F[2];
    acc[5] += r[0] * F[1] - r[1] * F[0];
  }
  for (int k = 0; k < 6; k++)
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_down(acc[k], off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0)
    for (int k = 0; k < 6; k++) part[wv][k] = acc[k];
  __syncthreads();
  if (threadIdx.x < 6) {
    double v = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); w++) v += part[w][threadIdx.x];
    tot[threadIdx.x] = v;
    f.hist[(uint64_t)s * 6 + threadIdx.x] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double FT[6];
  for (int k = 0; k < 6; k++) FT[k] = tot[k];
  free_update_with(sd, solids, s, FT, f.b, f.t, flag);
}

void launch_ibm_ft_free(lbm_ctx *c, int64_t t) {
  hipLaunchKernelGGL(k_ibm_ft_free, dim3((uint32_t)c->nsolid), dim3(kFtFreeBlock), 0, c->stream, ibm_ft_args_of(c, t),
                     c->at<DevSolid>(c->L.solids), c->at<uint32_t>(c->L.misc) + 6);
}

// Force/torque of step t per solid (as k_ft_reduce) and, by the lane that
// wrote them, the free motion of that solid from the same values.
__global__ __launch_bounds__(256) void k_ft_reduce_free(FtReduceArgs r, DevSolid *solids, Box3 b, int64_t t,
                                                        uint32_t *flag) {
  ft_reduce_waves(r, blockIdx.x);
  const int s = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
  if ((threadIdx.x & 63) != 0 || s >= r.nsolid) return;
  double FT[6];
  for (int k = 0; k < 6; k++) FT[k] = r.hist[(uint64_t)s * 6 + k];  // this thread's own stores
  free_update_one(solids, s, FT, b, t, flag);
}

// Per-solid force/torque: one wavefront per solid sums that solid's chunk
// partials in chunk order into the history slot (used for the last step of an
// lbm_step call; earlier steps are reduced inside the next sweep launch).
__global__ __launch_bounds__(256) void k_ft_reduce(FtReduceArgs r) {
  ft_reduce_waves(r, blockIdx.x);
}

// Chunk partials from per-link force terms (the sweep's bounce-back of fixed
// solids); 256 threads, one chunk unit per wavefront.
template <int Q>
__global__ __launch_bounds__(256) void k_chunk_sum(ChunkSumArgs a) {
  chunk_sum_waves<Q>(a, blockIdx.x);
}

// Link lists of fixed solids by sweep segment (64 cells): count the links of
// every segment (and flag their fluid nodes F_LINK), give each segment with
// links a range of the cell list, fill the ranges with link indices.  The
// order inside a range does not matter: every link writes its own direction
// and its own slots.
__global__ __launch_bounds__(64) void k_seg_link_count(LinkArgs a, SegLink *seg) {
  const SolidLinks sl = a.sl[blockIdx.y];
  const uint32_t li = blockIdx.x * 64 + threadIdx.x;
  if (li >= sl.count || (uint64_t)sl.start + li >= a.max_links) return;
  const uint32_t n = a.link_cell[(uint64_t)sl.start + li];
  atomicAdd(&seg[n >> 6].count, 1u);
  a.flags[n] = (uint8_t)(a.flags[n] | F_LINK);  // every writer sets the same bit
}
__global__ __launch_bounds__(256) void k_seg_link_alloc(SegLink *seg, uint32_t nseg, uint32_t *cursor) {
  const uint32_t s = blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const uint32_t v = s < nseg ? seg[s].count : 0u;
  uint32_t inc = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(inc, off, 64);
    if (lane >= off) inc += t;
  }
  const uint32_t tot = __shfl(inc, 63, 64);
  uint32_t base = 0;
  if (lane == 63 && tot) base = atomicAdd(cursor, tot);
  base = __shfl(base, 63, 64);
  if (v) seg[s] = SegLink{base + inc - v, 0u};
}
__global__ __launch_bounds__(64) void k_seg_link_fill(LinkArgs a, SegLink *seg, uint32_t *cell_list) {
  const SolidLinks sl = a.sl[blockIdx.y];
  const uint32_t li = blockIdx.x * 64 + threadIdx.x;
  if (li >= sl.count || (uint64_t)sl.start + li >= a.max_links) return;
  const uint64_t l = (uint64_t)sl.start + li;
  SegLink *g = &seg[a.link_cell[l] >> 6];
  const uint64_t pos = (uint64_t)g->first + atomicAdd(&g->count, 1u);
  if (pos < a.max_links) cell_list[pos] = (uint32_t)l;
}

// Link table of fixed solids for the sweep, one thread per cell-list entry
// (sweep-segment order): the link's cells, formula and coefficients
// (LinkRec at the entry) and the FP64 constants of Eq. 17 ([12][stride]: a,
// b, d, r at the link index), from the same functions the bounce-back kernel
// evaluates each step.  Bits 8.. of a link's meta word hold its solid.
template <int Q, typename S>
__global__ __launch_bounds__(64) void k_link_table(LinkArgs a, const uint32_t *cell_list, uint32_t nlinks, int method,
                                                   void *rec_, uint64_t stride) {
  using C = typename Store<S>::C;
  const uint32_t pos = blockIdx.x * 64 + threadIdx.x;
  if (pos >= nlinks) return;
  const uint32_t l = cell_list[pos];
  if ((uint64_t)l >= stride || (uint64_t)l >= a.max_links) return;
  const uint32_t n = a.link_cell[l], meta = a.link_meta[l];
  const double q = a.link_q[l];
  const int i = (int)(meta & 31u);
  const int s = (int)(meta >> 8);
  int x, y, z;
  xyz_of(n, a.g, x, y, z);
  const DevSolid sd = a.g.solids[s];
  double c[3];
  solid_centre(sd, a.g.t, a.g.b, c);
  const LinkGeo g = link_geo<Q>(i, q, sd, c, x, y, z, a.g.b);
  const LinkCoef<C> k = link_coef<C>(method, q, (meta >> 5) & 1u, (meta >> 6) & 1u);
  LinkRec<C> r{};
  r.n = n;
  r.nb = g.nb;
  r.nff = g.nff;
  r.nfff = g.nfff;
  r.kind_dir = (uint32_t)k.kind | ((uint32_t)i << 8);
  r.l = l;
  r.k1 = k.k1;
  r.k2 = k.k2;
  r.k3 = k.k3;
  r.k4 = k.k4;
  r.B = link_wall<C>(k, g.B);
  static_cast<LinkRec<C> *>(rec_)[pos] = r;
}

// ----------------------------------------------------------------------------
// batched forms: the same bodies over the members of a work list, each at its
// own time t = t0 + k and state parity (k: the batch step counter)
// ----------------------------------------------------------------------------
__device__ inline int64_t slot_time(const BatchSlot *slots, int m, int64_t k) { return SLOT(m, t0) + k; }
__device__ inline void *slot_post(const BatchSlot *slots, int m, int64_t k) {
  return SLOT(m, P[(SLOT(m, cur0) ^ (int)(k & 1)) ^ 1]);
}
__device__ inline const void *slot_pre(const BatchSlot *slots, int m, int64_t k) {
  return SLOT(m, P[SLOT(m, cur0) ^ (int)(k & 1)]);
}

// bounce-back on the post-collision array of this step; unit = (solid, chunk)
template <int Q, typename S>
__global__ __launch_bounds__(64) void k_ibb_batch(const BatchSlot *__restrict__ slots, const WorkList *__restrict__ wl,
                                                   const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const uint32_t per = (uint32_t)SLOT(m, k5_chunks);
    const int s = (int)(u / per);
    const IbbArgs a = SLOT(m, ib);
    ibb_body<Q, S>(static_cast<S *>(slot_post(slots, m, k)), static_cast<const S *>(slot_pre(slots, m, k)), a,
                   slot_time(slots, m, k), u - (uint32_t)s * per, s);
  });
}

// per-solid force/torque of this step into the lattice's history ring
__global__ __launch_bounds__(256) void k_ft_batch(const BatchSlot *__restrict__ slots, const WorkList *__restrict__ wl,
                                                  const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    FtReduceArgs r = SLOT(m, ft);
    r.hist = SLOT(m, hist) + (uint64_t)(slot_time(slots, m, k) % kHistCap) * (uint64_t)SLOT(m, max_solids) * 6;
    ft_reduce_waves(r, u);
  });
}

// translating solids move to t + 1: keep and classify, count, scan with
// refill, emit -- over the (solid, box chunk) units of the moving members, or
// one unit per member
__device__ inline LinkArgs move_args(const BatchSlot *slots, int m, int64_t k) {
  LinkArgs a = SLOT(m, lk);
  a.g.t = slot_time(slots, m, k) + 1;
  a.post = slot_post(slots, m, k);
  return a;
}
// (a member with one solid classifies in the same pass: no other box can meet
// its box, so each box cell is one thread's in both phases; members with
// several solids classify in k_classify_box_batch, over their own work list)
__global__ __launch_bounds__(kBlock) void k_classify_keep_batch(const BatchSlot *__restrict__ slots,
                                                                const WorkList *__restrict__ wl,
                                                                const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const LinkArgs a = move_args(slots, m, k);
    const int s = (int)(u / a.max_box_chunks);
    const uint32_t bx = u - (uint32_t)s * a.max_box_chunks;
    classify_keep_body(a, bx, s);
    if (SLOT(m, nsolid) == 1) classify_box_body(a, bx, s);
  });
}
__global__ __launch_bounds__(kBlock) void k_classify_box_batch(const BatchSlot *__restrict__ slots,
                                                               const WorkList *__restrict__ wl,
                                                               const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const LinkArgs a = move_args(slots, m, k);
    const int s = (int)(u / a.max_box_chunks);
    classify_box_body(a, u - (uint32_t)s * a.max_box_chunks, s);
  });
}
// (the box units are latency-bound chains of loads; at most 64 registers, no
// spills, let 8 waves per SIMD overlap them)
template <int Q>
__global__ __launch_bounds__(kBlock, 8) void k_link_count_batch(const BatchSlot *__restrict__ slots,
                                                             const WorkList *__restrict__ wl,
                                                             const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const LinkArgs a = move_args(slots, m, k);
    const int s = (int)(u / a.max_box_chunks);
    link_count_body<Q>(a, u - (uint32_t)s * a.max_box_chunks, s);
  });
}
// One unit per member: the link scan, which also folds the capacity checks
// into the member's status words, then the refill of the nodes its solids
// uncovered, the block's 16 wavefronts walking the refill list.  The refill
// reads only the finished classification and writes populations, which
// neither the scan nor the count and emit passes touch; it rides here rather
// than in the count pass, whose occupancy its registers would lower.
template <int Q, typename S>
__global__ __launch_bounds__(1024) void k_scan_refill_batch(const BatchSlot *__restrict__ slots,
                                                            const WorkList *__restrict__ wl,
                                                            const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t) {
    const LinkArgs a = move_args(slots, m, k);
    const int nsolid = SLOT(m, nsolid);
    link_scan_body(a, nsolid);
    if (threadIdx.x == 0) {
      uint32_t bad = a.misc[1] ? (uint32_t)BS_LINKS_OVERFLOW : 0u;
      if (a.misc[4]) bad |= BS_REFILL_OVERFLOW;
      const uint32_t k5 = (uint32_t)SLOT(m, k5_chunks);
      for (int s = 0; s < nsolid; s++)
        if (a.sl[s].nchunks > k5) bad |= BS_CHUNKS_OVERFLOW;
      uint32_t *st = SLOT(m, status);
      st[0] |= bad;
      st[1] = a.misc[0];
    }
    const uint32_t cnt = min(a.misc[3], a.max_refill);
    for (uint32_t e = threadIdx.x >> 6; e < cnt; e += blockDim.x >> 6) refill_wave<Q, S>(a, a.refill_list[e]);
    __syncthreads();
  });
}
// (5 waves per SIMD is the most its registers allow without spills)
template <int Q>
__global__ __launch_bounds__(kBlock, 5) void k_link_emit_batch(const BatchSlot *__restrict__ slots,
                                                            const WorkList *__restrict__ wl,
                                                            const int64_t *__restrict__ step) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t u) {
    const LinkArgs a = move_args(slots, m, k);
    const int s = (int)(u / a.max_box_chunks);
    link_emit_body<Q>(a, u - (uint32_t)s * a.max_box_chunks, s);
  });
}

// Relative change |a - b| / |a| of a solid's force (3 values each): 0 for two
// zero forces, infinity from zero to non-zero, NaN when either is not finite
// (a diverged member).
__device__ inline double force_rel_change(const double *a, const double *b) {
  double d2 = 0.0, n2 = 0.0, m2 = 0.0;
  for (int c = 0; c < 3; c++) {
    d2 += (a[c] - b[c]) * (a[c] - b[c]);
    n2 += a[c] * a[c];
    m2 += b[c] * b[c];
  }
  if (!isfinite(n2) || !isfinite(m2) || !isfinite(d2)) return __builtin_nan("");
  return n2 > 0.0 ? sqrt(d2 / n2) : (d2 > 0.0 ? INFINITY : 0.0);
}
// max that keeps a NaN
__device__ inline double max_keep_nan(double x, double y) { return (x != x || y != y) ? __builtin_nan("") : fmax(x, y); }

// Serving convergence check: per member, the largest relative change of a
// solid's force over `lag` steps, |F(t-1) - F(t-1-lag)| / |F(t-1)| with t the
// member's time (NaN if a force is not finite); -1 while fewer than lag + 1
// steps are in its history.
__global__ __launch_bounds__(64) void k_force_change(const BatchSlot *__restrict__ slots,
                                                     const WorkList *__restrict__ wl,
                                                     const int64_t *__restrict__ step, int64_t lag, double *out) {
  const int64_t k = *step;
  batch_units(wl, 0, [&](int m, uint32_t) {
    const double *hist = SLOT(m, hist);
    const int nsolid = SLOT(m, nsolid);
    const int max_solids = SLOT(m, max_solids);
    const int s = (int)threadIdx.x;
    const int64_t t = SLOT(m, t0) + k - 1;
    const bool ok = lag > 0 && lag < kHistCap && t - lag >= 0;
    double r = 0.0;
    if (ok && s < nsolid) {
      const uint64_t per = (uint64_t)max_solids * 6;
      const double *a = hist + (uint64_t)(t % kHistCap) * per + (uint64_t)s * 6;
      const double *b = hist + (uint64_t)((t - lag) % kHistCap) * per + (uint64_t)s * 6;
      r = force_rel_change(a, b);
    }
    for (int off = 32; off > 0; off >>= 1) r = max_keep_nan(r, __shfl_down(r, off, 64));
    for (int s0 = 64; s0 < nsolid; s0 += 64) {  // more than 64 solids: serial tail in lane 0
      if (threadIdx.x == 0 && ok) {
        for (int q = s0; q < min(nsolid, s0 + 64); q++) {
          const uint64_t per = (uint64_t)max_solids * 6;
          const double *a = hist + (uint64_t)(t % kHistCap) * per + (uint64_t)q * 6;
          const double *b = hist + (uint64_t)((t - lag) % kHistCap) * per + (uint64_t)q * 6;
          r = max_keep_nan(r, force_rel_change(a, b));
        }
      }
    }
    if (threadIdx.x == 0) out[m] = ok ? r : -1.0;
  });
}

void launch_force_change(const BatchLaunch &b, const WorkList *wl, int64_t lag, double *out, uint32_t grid) {
  hipLaunchKernelGGL(k_force_change, dim3(grid), dim3(64), 0, b.stream, b.slots, wl, b.step, lag, out);
}

void launch_ibb_batch(const BatchLaunch &b, const WorkList *wl, uint32_t grid) {
#define LBM_IBB(QQ, SS) hipLaunchKernelGGL((k_ibb_batch<QQ, SS>), dim3(grid), dim3(64), 0, b.stream, b.slots, wl, b.step)
  if (b.Q == 9) {
    if (b.storage == LBM_F64) LBM_IBB(9, double);
    else if (b.storage == LBM_F32_DEV) LBM_IBB(9, float);
    else LBM_IBB(9, _Float16);
  } else {
    if (b.storage == LBM_F64) LBM_IBB(19, double);
    else if (b.storage == LBM_F32_DEV) LBM_IBB(19, float);
    else LBM_IBB(19, _Float16);
  }
#undef LBM_IBB
}

void launch_ft_batch(const BatchLaunch &b, const WorkList *wl, uint32_t grid) {
  hipLaunchKernelGGL(k_ft_batch, dim3(grid), dim3(256), 0, b.stream, b.slots, wl, b.step);
}

void launch_move_batch(const BatchLaunch &b, const WorkList *box, const WorkList *boxm, const WorkList *one,
                       bool any_multi, uint32_t grid) {
  const dim3 g(grid), blk(kBlock), g1(std::min<uint32_t>(grid, 1024));
  hipLaunchKernelGGL(k_classify_keep_batch, g, blk, 0, b.stream, b.slots, box, b.step);
  if (any_multi) hipLaunchKernelGGL(k_classify_box_batch, g, blk, 0, b.stream, b.slots, boxm, b.step);
  if (b.Q == 9) hipLaunchKernelGGL(k_link_count_batch<9>, g, blk, 0, b.stream, b.slots, box, b.step);
  else hipLaunchKernelGGL(k_link_count_batch<19>, g, blk, 0, b.stream, b.slots, box, b.step);
#define LBM_SR(QQ, SS) \
  hipLaunchKernelGGL((k_scan_refill_batch<QQ, SS>), g1, dim3(1024), 0, b.stream, b.slots, one, b.step)
  if (b.Q == 9) {
    if (b.storage == LBM_F64) LBM_SR(9, double);
    else if (b.storage == LBM_F32_DEV) LBM_SR(9, float);
    else LBM_SR(9, _Float16);
  } else {
    if (b.storage == LBM_F64) LBM_SR(19, double);
    else if (b.storage == LBM_F32_DEV) LBM_SR(19, float);
    else LBM_SR(19, _Float16);
  }
#undef LBM_SR
  if (b.Q == 9) hipLaunchKernelGGL(k_link_emit_batch<9>, g, blk, 0, b.stream, b.slots, box, b.step);
  else hipLaunchKernelGGL(k_link_emit_batch<19>, g, blk, 0, b.stream, b.slots, box, b.step);
}

// ----------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------
static GeoArgs geo_args(const lbm_ctx *c, int64_t t) {
  GeoArgs g{};
  g.b = Box3{c->p.nx, c->p.ny, c->p.nz, c->D};
  g.N = (uint32_t)c->N;
  g.fx = c->fx;
  g.fy = c->fy;
  g.stride = c->L.stride;
  g.solids = c->at<DevSolid>(c->L.solids);
  g.nsolid = c->nsolid;
  g.ibb = c->method != LBM_IBM;
  g.fluid_only = c->p.body_force_fluid_only;
  g.t = t;
  return g;
}

static LinkArgs link_args(const lbm_ctx *c, int64_t t) {
  LinkArgs a{};
  a.g = geo_args(c, t);
  a.flags = c->at<uint8_t>(c->L.flags);
  a.owner = c->at<uint16_t>(c->L.owner0);
  a.owner_prev = c->at<uint16_t>(c->L.owner1);
  a.box_counts = c->at<uint32_t>(c->L.box_counts);
  a.box_offsets = c->at<uint32_t>(c->L.box_offsets);
  a.max_box_chunks = (uint32_t)c->max_box_chunks;
  a.link_cell = c->at<uint32_t>(c->L.link_cell);
  a.link_meta = c->at<uint32_t>(c->L.link_meta);
  a.link_q = c->at<double>(c->L.link_q);
  a.max_links = (uint64_t)c->L.max_links;
  a.sl = c->at<SolidLinks>(c->L.solid_links);
  a.misc = c->at<uint32_t>(c->L.misc);
  a.refill_list = c->at<uint64_t>(c->L.refill);
  a.max_refill = (uint32_t)c->L.max_refill;
  a.masks = c->mask_cells > 0 ? c->at<uint32_t>(c->L.staging) : nullptr;
  a.cu = c->p.cover_momentum ? c->at<unsigned long long>(c->L.cu) : nullptr;
  return a;
}

void fill_link_args(lbm_ctx *c, LinkArgs *a) { *a = link_args(c, c->t); }

void fill_ibb_args(lbm_ctx *c, IbbArgs *ap) {
  IbbArgs &a = *ap;
  a = IbbArgs{};
  a.g = geo_args(c, c->t);
  a.link_cell = c->at<uint32_t>(c->L.link_cell);
  a.link_meta = c->at<uint32_t>(c->L.link_meta);
  a.link_q = c->at<double>(c->L.link_q);
  a.sl = c->at<SolidLinks>(c->L.solid_links);
  a.partials = c->at<double>(c->L.partials);
  a.method = c->method;
  a.sr = c->p.storage == LBM_F16_SR ? 1 : 0;
  a.max_links = (uint64_t)c->L.max_links;
  a.max_partials = (uint64_t)c->L.max_partials;
}

void launch_classify(lbm_ctx *c, int64_t t, bool full) {
  if (full) {
    GeoArgs g = geo_args(c, t);
    hipLaunchKernelGGL(k_classify_full, dim3((uint32_t)((c->N + 255) / 256)), dim3(256), 0, c->stream,
                       c->at<uint8_t>(c->L.flags), c->at<uint16_t>(c->L.owner0), c->at<uint16_t>(c->L.owner1), g);
    return;
  }
  LinkArgs a = link_args(c, t);
  if (c->nsolid == 1) {
    hipLaunchKernelGGL(k_classify_one, dim3((uint32_t)c->max_box_chunks), dim3(kBlock), 0, c->stream, a);
    return;
  }
  const dim3 grid((uint32_t)c->max_box_chunks, (uint32_t)c->nsolid);
  hipLaunchKernelGGL(k_classify_keep, grid, dim3(kBlock), 0, c->stream, a);
  hipLaunchKernelGGL(k_classify_box, grid, dim3(kBlock), 0, c->stream, a);
}

void launch_refill_count(lbm_ctx *c, int64_t t, void *post) {
  LinkArgs a = link_args(c, t);
  a.post = post;
  const dim3 grid(kRefillBlocks + (uint32_t)c->max_box_chunks * (uint32_t)c->nsolid);
#define LBM_RC(QQ, SS) hipLaunchKernelGGL((k_refill_count<QQ, SS>), grid, dim3(kBlock), 0, c->stream, a)
  if (c->Q == 9) {
    if (c->p.storage == LBM_F64) LBM_RC(9, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_RC(9, float);
    else LBM_RC(9, _Float16);
  } else {
    if (c->p.storage == LBM_F64) LBM_RC(19, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_RC(19, float);
    else LBM_RC(19, _Float16);
  }
#undef LBM_RC
}

void launch_link_count(lbm_ctx *c, int64_t t) {
  LinkArgs a = link_args(c, t);
  const dim3 grid((uint32_t)c->max_box_chunks, (uint32_t)c->nsolid);
  if (c->Q == 9) hipLaunchKernelGGL(k_link_count<9>, grid, dim3(kBlock), 0, c->stream, a);
  else hipLaunchKernelGGL(k_link_count<19>, grid, dim3(kBlock), 0, c->stream, a);
}

void launch_link_scan(lbm_ctx *c) {
  LinkArgs a = link_args(c, 0);
  hipLaunchKernelGGL(k_link_scan, dim3(1), dim3(1024), 0, c->stream, a, c->nsolid);
}

void launch_link_emit(lbm_ctx *c, int64_t t) {
  LinkArgs a = link_args(c, t);
  if (c->nsolid == 1) {  // offsets formed in the emit pass itself (no scan launch)
    const dim3 g1((uint32_t)c->max_box_chunks);
    if (c->Q == 9) hipLaunchKernelGGL(k_link_emit_one<9>, g1, dim3(kBlock), 0, c->stream, a);
    else hipLaunchKernelGGL(k_link_emit_one<19>, g1, dim3(kBlock), 0, c->stream, a);
    return;
  }
  const dim3 grid((uint32_t)c->max_box_chunks, (uint32_t)c->nsolid);
  if (c->Q == 9) hipLaunchKernelGGL(k_link_emit<9>, grid, dim3(kBlock), 0, c->stream, a);
  else hipLaunchKernelGGL(k_link_emit<19>, grid, dim3(kBlock), 0, c->stream, a);
}

void launch_ibb(lbm_ctx *c, void *P, const void *pre, int64_t t) {
  if (c->k5_chunks <= 0) return;
  IbbArgs a;
  fill_ibb_args(c, &a);
  a.g.t = t;
  a.partials = partials_of(c, t);
  const dim3 grid((uint32_t)c->k5_chunks, (uint32_t)c->nsolid);
#define LBM_IBB(QQ, SS) \
  hipLaunchKernelGGL((k_ibb<QQ, SS>), grid, dim3(64), 0, c->stream, static_cast<SS *>(P), static_cast<const SS *>(pre), a)
  if (c->Q == 9) {
    if (c->p.storage == LBM_F64) LBM_IBB(9, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_IBB(9, float);
    else LBM_IBB(9, _Float16);
  } else {
    if (c->p.storage == LBM_F64) LBM_IBB(19, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_IBB(19, float);
    else LBM_IBB(19, _Float16);
  }
#undef LBM_IBB
}

FtReduceArgs ft_reduce_args(lbm_ctx *c, int64_t t) {
  FtReduceArgs r{};
  r.partials = c->at<double>(c->L.partials);
  r.sl = c->at<SolidLinks>(c->L.solid_links);
  r.hist = c->at<double>(c->L.hist) + (uint64_t)(t % kHistCap) * c->L.max_solids * 6;
  r.nsolid = c->nsolid;
  r.max_partials = (uint64_t)c->L.max_partials;
  r.cu = (c->p.cover_momentum && c->any_moving) ? c->at<unsigned long long>(c->L.cu) : nullptr;
  return r;
}

void launch_ft_reduce(lbm_ctx *c, int64_t t) {
  if (c->k5_chunks <= 0) return;
  FtReduceArgs r = ft_reduce_args(c, t);
  r.partials = partials_of(c, t);
  hipLaunchKernelGGL(k_ft_reduce, dim3((uint32_t)((c->nsolid + 3) / 4)), dim3(256), 0, c->stream, r);
}

// Free solids: the force reduction of step t and the motion update in one launch
// (a solid without links gets zero force and moves under its weight alone).
void launch_ft_reduce_free(lbm_ctx *c, int64_t t) {
  FtReduceArgs r = ft_reduce_args(c, t);
  r.partials = partials_of(c, t);
  const Box3 b{c->p.nx, c->p.ny, c->p.nz, c->D};
  hipLaunchKernelGGL(k_ft_reduce_free, dim3((uint32_t)((c->nsolid + 3) / 4)), dim3(256), 0, c->stream, r,
                     c->at<DevSolid>(c->L.solids), b, t, c->at<uint32_t>(c->L.misc) + 6);
}

double *partials_of(lbm_ctx *c, int64_t t) { return c->at<double>((t & 1) ? c->L.partials2 : c->L.partials); }

// Staging region while an lbm_step call applies the bounce-back in the sweep:
// the link records and, per step parity, the stored incoming and outgoing
// values of every link ([2][stride] compute type).
static size_t link_rec_bytes(const lbm_ctx *c) { return c->store_bytes == 8 ? sizeof(LinkRec<double>) : sizeof(LinkRec<float>); }
static size_t link_c_bytes(const lbm_ctx *c) { return c->store_bytes == 8 ? 8 : 4; }
static size_t link_io_offset(const lbm_ctx *c, int64_t t) {
  return c->L.staging + c->link_stride * link_rec_bytes(c) + (size_t)(t & 1) * 2 * c->link_stride * link_c_bytes(c);
}
bool link_table_fits(const lbm_ctx *c, uint64_t stride) {
  const size_t per = link_rec_bytes(c) + 4 * link_c_bytes(c);
  return stride * per <= (size_t)4 * c->N * 8;
}

void *link_io_of(lbm_ctx *c, int64_t t) { return c->ws + link_io_offset(c, t); }
const void *link_rec_of(lbm_ctx *c) { return c->ws + c->L.staging; }

ChunkSumArgs chunk_sum_args(lbm_ctx *c, int64_t t) {
  ChunkSumArgs a{};
  a.io = link_io_of(c, t);
  a.cbytes = (int)link_c_bytes(c);
  a.lcell = c->at<uint32_t>(c->L.link_cell);
  a.lmeta = c->at<uint32_t>(c->L.link_meta);
  a.lq = c->at<double>(c->L.link_q);
  a.solids = c->at<DevSolid>(c->L.solids);
  a.nx = c->p.nx;
  a.ny = c->p.ny;
  a.nz = c->p.nz;
  a.D = c->D;
  a.fx = c->fx;
  a.fy = c->fy;
  a.stride = c->link_stride;
  a.sl = c->at<SolidLinks>(c->L.solid_links);
  a.partials = partials_of(c, t);
  a.max_links = (uint64_t)c->L.max_links;
  a.max_partials = (uint64_t)c->L.max_partials;
  a.per = (uint32_t)c->k5_chunks;
  a.nsolid = c->nsolid;
  return a;
}

void launch_link_table(lbm_ctx *c) {
  if (!c->link_lists) return;
  const LinkArgs a = link_args(c, c->t);
  const uint32_t nl = (uint32_t)c->nlinks;
  const dim3 grid((nl + 63) / 64);
  const uint32_t *list = c->at<uint32_t>(c->L.cell_list);
  void *rec = c->ws + c->L.staging;
  const uint64_t st = c->link_stride;
#define LBM_LT(QQ, SS) \
  hipLaunchKernelGGL((k_link_table<QQ, SS>), grid, dim3(64), 0, c->stream, a, list, nl, c->method, rec, st)
  if (c->Q == 9) {
    if (c->p.storage == LBM_F64) LBM_LT(9, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_LT(9, float);
    else LBM_LT(9, _Float16);
  } else {
    if (c->p.storage == LBM_F64) LBM_LT(19, double);
    else if (c->p.storage == LBM_F32_DEV) LBM_LT(19, float);
    else LBM_LT(19, _Float16);
  }
#undef LBM_LT
}

uint32_t chunk_sum_blocks(const lbm_ctx *c) {
  return (uint32_t)(((int64_t)c->k5_chunks * c->nsolid + 3) / 4);
}

void launch_chunk_sum(lbm_ctx *c, int64_t t) {
  if (c->k5_chunks <= 0) return;
  if (c->Q == 9)
    hipLaunchKernelGGL(k_chunk_sum<9>, dim3(chunk_sum_blocks(c)), dim3(256), 0, c->stream, chunk_sum_args(c, t));
  else
    hipLaunchKernelGGL(k_chunk_sum<19>, dim3(chunk_sum_blocks(c)), dim3(256), 0, c->stream, chunk_sum_args(c, t));
}

// Builds the link lists by sweep segment of a context whose solids are all
// fixed; without them (translating solids, IBM, capacity limits) the
// bounce-back stays a kernel of its own after every sweep.
hipError_t build_link_lists(lbm_ctx *c) {
  c->link_lists = false;
  c->link_stride = 0;
  if (c->method == LBM_IBM || c->any_moving || c->nsolid <= 0 || c->nlinks <= 0 || c->k5_chunks <= 0)
    return hipSuccess;
  const uint64_t stride = ((uint64_t)c->nlinks + 63) / 64 * 64;
  // the per-call link table must fit the staging region
  if (!link_table_fits(c, stride)) return hipSuccess;
  const uint32_t nseg = (uint32_t)((c->N + 63) / 64);
  SegLink *seg = c->at<SegLink>(c->L.seg_link);
  uint32_t *cursor = c->at<uint32_t>(c->L.misc) + 12;
  hipError_t e = hipMemsetAsync(seg, 0, (size_t)nseg * sizeof(SegLink), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(cursor, 0, 4, c->stream);
  if (e != hipSuccess) return e;
  const LinkArgs a = link_args(c, c->t);
  const dim3 grid((uint32_t)c->k5_chunks, (uint32_t)c->nsolid);
  hipLaunchKernelGGL(k_seg_link_count, grid, dim3(64), 0, c->stream, a, seg);
  hipLaunchKernelGGL(k_seg_link_alloc, dim3((nseg + 255) / 256), dim3(256), 0, c->stream, seg, nseg, cursor);
  hipLaunchKernelGGL(k_seg_link_fill, grid, dim3(64), 0, c->stream, a, seg, c->at<uint32_t>(c->L.cell_list));
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  c->link_stride = stride;
  c->link_lists = true;
  return hipSuccess;
}

}  // namespace lbm
