// lbm_args.hpp -- per-lattice argument blocks of the kernels.  The same
// blocks are passed by value to the single-lattice kernels and stored in
// device memory, one per lattice, for the batched kernels.
#pragma once

#include "lbm_geom.hpp"

namespace lbm {

struct GeoArgs {
  Box3 b;
  uint32_t N;
  FastDiv fx, fy;
  uint64_t stride;
  const DevSolid *solids;
  int nsolid;
  int ibb;         // 1 = solids remove nodes from the fluid (IBB), 0 = IBM
  int fluid_only;  // body force only outside solids
  int64_t t;       // geometry time
};

struct LinkArgs {
  GeoArgs g;
  uint8_t *flags;
  uint16_t *owner, *owner_prev;
  uint32_t *box_counts;    // [nsolid][max_box_chunks]
  uint32_t *box_offsets;   // exclusive scan of box_counts
  uint32_t max_box_chunks;
  uint32_t *link_cell, *link_meta;
  double *link_q;
  uint64_t max_links;
  SolidLinks *sl;
  uint32_t *misc;          // [0] total links, [1] overflow flag
  void *post;              // refill: post-collision array of step t-1 -> t
  uint64_t *refill_list;   // nodes uncovered this step: (solid << 32) | cell; with cu also the
                           // nodes covered, marked by bit 63
  unsigned long long *cu;  // covering / uncovering momentum [solid][6] in fixed point (cu_scale), or null
  uint32_t max_refill;     // misc[3] counts them, misc[4] flags an overflow
  uint32_t *masks;         // link mask of every box cell (solid s at solids[s].mask_off), written by
                           // the count pass, read by the emit pass; null: emit recomputes them
};

struct IbbArgs {
  GeoArgs g;
  const uint32_t *link_cell, *link_meta;
  const double *link_q;
  const SolidLinks *sl;
  double *partials;  // [chunk][6]
  uint64_t max_links, max_partials;
  int method;        // LBM_BB, LBM_IBB_LINEAR, LBM_IBB_QUADRATIC, LBM_IBB_YU, LBM_IBB_ZHAO_YONG
  int sr;            // FP16 stochastic rounding of the link values (seed from the step)
};

// Per-solid IBM force and torque of one step (Sec. 3.1, App. B).
struct IbmFtArgs {
  Box3 b;
  const DevSolid *solids;
  int mv;              // moving solid: lever arms from wts (see IbmArgs)
  const double *wts;
  const double *X, *dV, *Fsum;
  const int64_t *start, *count;  // points of each solid
  double *hist;                  // history slot of the step
  int64_t t;
};

struct SweepArgs {
  uint32_t N, nx, ny, nz;
  FastDiv fx, fy;
  uint64_t stride;
  const uint8_t *flags;
  const void *fibm;  // [3][stride] compute type, read where F_IBM is set
  double g[3];
  double omega;          // BGK
  double sp, sm;         // two-rate MRT: even and odd non-conserved rates
  double sA[kMaxQ];      // general MRT: -s_k / |M_k|^2
  double sB[kMaxQ];      //              (1 - s_k/2) / |M_k|^2
  uint32_t rblocks;      // leading blocks that reduce the previous step's force partials
  FtReduceArgs ft;
  uint32_t iblocks;      // next blocks: IBM force/torque of this step, one per solid
  IbmFtArgs ift;
  uint32_t xcd;          // 1: blocks take tiles in XCD-contiguous order
  uint32_t sr;           // FP16 storage with stochastic rounding
  uint32_t seed;         // sr_seed of the step the sweep computes
  int32_t bc[3];         // domain boundaries per axis (BND_*), bounded-domain sweeps only
  double uin;            // inflow velocity of an open x axis
  void *uo;              // [ny nz] compute type: u_x of the last x layer's collisions (open x)
};

// Bounce-back of the previous step applied inside the sweep (fixed solids).
// The wavefront that sweeps cells 64 s .. 64 s + 63 evaluates the links of
// those cells (seg_link[s] into cell_list, one link per lane; LinkRec records
// of the compute type in rec) on the source array, which holds the
// post-collision values of the previous step.  Each value replaces the pulled
// value of its direction in the owning lane (through LDS) and is written to
// the solid-node slot it stands for; the link's incoming and outgoing values
// (io, [2][stride]) are kept for Eq. 17.  Leading blocks form the chunk
// partials of the step before.
struct SweepLinkArgs {
  const SegLink *seg_link;
  const uint32_t *cell_list;
  uint32_t nseg;
  const void *rec;
  void *io;
  uint64_t stride;
  uint32_t cblocks;
  ChunkSumArgs cs;
  uint32_t sr, lseed;  // FP16 stochastic rounding of the link values; sr_seed of the links' step
  uint32_t ghost;      // links evaluated from A also store their values in A's solid-node slots
};

// IBM spreading: lanes per shell cell (each takes every kSpreadLanes-th entry
// of the cell's list) and shell cells per 256-thread block or batch unit.
constexpr int kSpreadLanes = 16;
constexpr int kSpreadCellsPerBlock = 256 / kSpreadLanes;

struct IbmArgs {
  Box3 b;
  uint32_t N;
  FastDiv fx, fy;
  uint64_t stride;
  int64_t nlag, nshell;
  const double *X, *dV;
  const int32_t *sid;
  double *Ud;            // [nlag][3]
  const int32_t *base;   // [nlag][3] floor(X) - 1
  double *wts;           // [nlag][12] per-axis weights
  const uint32_t *idx;   // [nlag][64] shell index of each stencil slot
  double *Fsum;          // [nlag][3] FP64 total boundary force of the step
  void *Fk;              // [nlag][3] compute type, force of the current iteration
  const uint32_t *shell_cell, *rowptr, *ent;
  void *ushell, *fshell; // [3][nshell] compute type
  void *fibm;            // [3][stride] compute type
  uint8_t *flags;
  const DevSolid *solids;
  double g[3];
  int64_t t;
  int delta;             // points of the delta function: 4 (Eq. 6), 3 or 2
  // moving solid: 5-node boxes (idx [nlag][128], ent = point << 7 | slot,
  // wts [nlag][24] = 3 x 5 weights, pad, lever arm at 16..18); shell cells
  // are where they were at placement, moved by the whole-cell shift, kept
  // for the step t in shift[4 (t & 1) + axis]
  int mv;
  int32_t *shift;
  // fixed solids, forcing iterations in point space: row l of the point
  // coupling A is nrow[l * nw .. l * nw + nw - 1] (IbmEntry of the compute
  // type; nptr[l] of them are the row, the rest padding with value 0 and
  // column l); the interpolated velocity U~ [nlag][3]; the force of an
  // iteration in Fk / Fk2 as [nlag] x 4 (x, y, z, 0) of the compute type; idx
  // holds the cell (not the shell index) of each stencil slot
  const uint32_t *nptr;
  void *nrow;
  int nw;
  int poly;  // the rows hold P (one product replaces the iterations), else A
  void *Ut;
  void *Fk2;
};

// One entry of a row of the point coupling: column (a point) and value.
template <typename C>
struct IbmEntry;
template <>
struct alignas(8) IbmEntry<float> {
  uint32_t col;
  float val;
};
template <>
struct alignas(16) IbmEntry<double> {
  uint32_t col, pad;
  double val;
};
// A point force of one iteration, padded to four components (one vector load).
template <typename C>
struct alignas(4 * sizeof(C)) IbmF4 {
  C x, y, z, w;
};

__device__ __host__ inline IbmFtArgs ibm_ft_args(const IbmArgs &a, int64_t t, const int64_t *start,
                                                 const int64_t *count, double *hist) {
  IbmFtArgs f;
  f.b = a.b;
  f.solids = a.solids;
  f.mv = a.mv;
  f.wts = a.wts;
  f.X = a.X;
  f.dV = a.dV;
  f.Fsum = a.Fsum;
  f.start = start;
  f.count = count;
  f.hist = hist;
  f.t = t;
  return f;
}

// Force -sum F_l dV_l and torque -sum (X_l - Y) x F_l dV_l on solid s; one
// block of kBlock threads (every caller uses that size, so the summation
// order, and the result, is the same in the sweep launch and the batched
// kernel).
__device__ inline void ibm_ft_body(const IbmFtArgs &a, int s) {
  __shared__ double lds[16];
  const DevSolid &sd = a.solids[s];
  double c[3];
  solid_centre(sd, a.t, a.b, c);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int64_t l = a.start[s] + threadIdx.x; l < a.start[s] + a.count[s]; l += blockDim.x) {
    double r[3], F[3];
    if (a.mv)
      for (int k = 0; k < 3; k++) r[k] = a.wts[l * 24 + 16 + k];
    else
      lever_arm(sd, c, a.X[l * 3], a.X[l * 3 + 1], a.X[l * 3 + 2], a.b, r);
    for (int k = 0; k < 3; k++) F[k] = -a.Fsum[l * 3 + k] * a.dV[l];
    acc[0] += F[0];
    acc[1] += F[1];
    acc[2] += F[2];
    acc[3] += r[1] * F[2] - r[2] * F[1];
    acc[4] += r[2] * F[0] - r[0] * F[2];
    acc[5] += r[0] * F[1] - r[1] * F[0];
  }
  for (int k = 0; k < 6; k++) {
    const double tot = block_sum(acc[k], lds);
    if (threadIdx.x == 0) a.hist[(uint64_t)s * 6 + k] = tot;
  }
}

// Cell indexing of the per-cell helper kernels.
struct CellArgs {
  uint32_t N, nx, ny, nz;
  FastDiv fx, fy;
  uint64_t stride;
  int32_t bnd;     // some axis is not periodic: gathers follow bnd_src
  int32_t bc[3];   // domain boundaries per axis (BND_*)
  double uin;      // inflow velocity of an open x axis
};

// Macroscopic-field kernel arguments.
struct MacroArgs {
  CellArgs ca;
  const uint8_t *flags;
  const uint16_t *owner;
  const DevSolid *solids;
  const void *fibm;
  double g[3];
  int64_t t_geom;
  int D;
  int initial;
  int moved;  // solids translated after the collision: its geometry is the previous one
  int nsolid;
  uint8_t solid_bit;
};

// Strain rate of the last collision (Eq. 19): the rates of the second-order
// moment rows (trace |e|^2, then 3e_x^2 - |e|^2 and e_y^2 - e_z^2 (D3Q19) or
// e_x^2 - e_y^2 (D2Q9), then e_x e_y, e_y e_z, e_x e_z), the viscosity of
// Eq. 2, and which half of the output a launch writes.
struct StrainArgs {
  MacroArgs m;
  double s[6];
  double nu;
  int part;  // 0: s_xx, s_yy, s_zz, eps; 1: s_xy, s_yz, s_xz
};

// One lattice of a batch as the batched kernels see it.  Its time and state
// parity advance with the batch step counter: at counter value k the lattice
// is at t = t0 + k and its current state is P[cur0 ^ (k & 1)].
struct BatchSlot {
  void *P[2];
  int32_t cur0;
  int32_t method;
  int32_t nsolid;
  int32_t n_iter;
  int32_t k5_chunks;
  int32_t max_box_chunks;
  int32_t max_solids;
  int32_t tiles;
  int64_t t0;
  double *hist;      // force/torque history ring of the lattice
  uint32_t *status;  // [0] sticky capacity-overflow flags, [1] link count
  const int64_t *lag_start, *lag_count;
  SweepArgs sw;
  IbbArgs ib;
  LinkArgs lk;
  IbmArgs im;
  FtReduceArgs ft;
};

// Status bits of a batched lattice.
enum { BS_LINKS_OVERFLOW = 1, BS_CHUNKS_OVERFLOW = 2, BS_REFILL_OVERFLOW = 4 };

// The units (tiles, link chunks, ...) of one batched launch: member k owns
// units start[k] .. start[k+1]-1 and is lattice slot[k] of the batch.  Kept
// in device memory, so a captured launch follows changes of the batch.
// Units of a batched launch: member j owns units start[j] .. start[j+1]-1
// and is batch slot slot[j]; bucket[b] is the member that owns the first unit
// u with u * kWlBuckets / total = b, where a lookup starts.
constexpr uint32_t kWlBuckets = 1024;
struct WorkList {
  uint32_t total;
  int32_t n;
  const uint32_t *start;
  const int32_t *slot;
  const uint16_t *bucket;
};

// Load of a block-uniform value from the batch tables through the constant
// address space: the tables are written only by the host between launches,
// so the value can come through the scalar cache into scalar registers (only
// the fields that are used are loaded).  The address must be block-uniform.
template <typename T>
__device__ __forceinline__ T load_uniform(const T *p) {
  T v;
  __builtin_memcpy(&v, (const __attribute__((address_space(4))) T *)p, sizeof(T));
  return v;
}

// Member that owns unit `u` (< total): the last k with start[k] <= u, found
// from u's bucket (usually zero or one step onwards).
__device__ inline int batch_member_of(const WorkList &wl, uint32_t u) {
  const uint32_t b = (uint32_t)(((uint64_t)u * kWlBuckets) / wl.total);
  int k = load_uniform(wl.bucket + b);
  while (k + 1 < wl.n && load_uniform(wl.start + k + 1) <= u) k++;
  return k;
}

// Persistent walk over the units of a work list by blocks blk of nblk: order 0
// gives each block a contiguous share, order 1 deals the units out
// round-robin.  f(slot, local unit) is called with the same trip count by
// every thread of the block.
template <typename F>
__device__ inline void batch_units_in(const WorkList *wlp, int order, uint32_t blk, uint32_t nblk, F f) {
  const WorkList wl = load_uniform(wlp);
  const uint32_t total = wl.total;
  uint32_t u, end, inc;
  if (order == 0) {
    const uint32_t per = (total + nblk - 1) / nblk;
    u = blk * per;
    end = min(total, u + per);
    inc = 1;
  } else {
    u = blk;
    end = total;
    inc = nblk;
  }
  if (u >= end) return;
  int k = batch_member_of(wl, u);
  uint32_t lo = load_uniform(wl.start + k), hi = load_uniform(wl.start + k + 1);
  for (; u < end; u += inc) {
    while (u >= hi) {
      k++;
      lo = hi;
      hi = load_uniform(wl.start + k + 1);
    }
    f(load_uniform(wl.slot + k), u - lo);
  }
}
// ... by all blocks of the grid
template <typename F>
__device__ inline void batch_units(const WorkList *wlp, int order, F f) {
  batch_units_in(wlp, order, blockIdx.x, gridDim.x, f);
}

// Block-uniform field of member m.
#define SLOT(m, field) load_uniform(&slots[m].field)

// Host side of a batched launch.
struct BatchLaunch {
  const BatchSlot *slots;
  const int64_t *step;
  hipStream_t stream;
  int Q, storage;
};

// argument blocks of a context (host)
void fill_sweep_args(lbm_ctx *c, SweepArgs *a);
// kernels_sweep_bnd.hip: the sweep on a domain with bounded axes
void launch_sweep_bnd(lbm_ctx *c, const void *A, void *B, const SweepArgs &a, const SweepLinkArgs &la, int coll,
                      int inl, hipEvent_t e0, hipEvent_t e1);
void fill_macro_args(lbm_ctx *c, MacroArgs *m, int mode);
void fill_ibb_args(lbm_ctx *c, IbbArgs *a);
void fill_link_args(lbm_ctx *c, LinkArgs *a);
void fill_ibm_args(lbm_ctx *c, IbmArgs *a);
IbmFtArgs ibm_ft_args_of(lbm_ctx *c, int64_t t);

// batched launches (grid = persistent blocks)
void launch_sweep_batch(const BatchLaunch &b, const WorkList *wl, int coll, int nt, int order, uint32_t grid,
                        hipEvent_t e0, hipEvent_t e1);
void launch_tick(hipStream_t s, int64_t *step);
void launch_ibb_batch(const BatchLaunch &b, const WorkList *wl, uint32_t grid);
void launch_ft_batch(const BatchLaunch &b, const WorkList *wl, uint32_t grid);
void launch_force_change(const BatchLaunch &b, const WorkList *wl, int64_t lag, double *out, uint32_t grid);
void launch_move_batch(const BatchLaunch &b, const WorkList *wl_box, const WorkList *wl_box_multi,
                       const WorkList *wl_one, bool any_multi, uint32_t grid);
void launch_ibm_batch(const BatchLaunch &b, const WorkList *wl_spread, const WorkList *wl_lag, const WorkList *wl_ft,
                      int max_iter, uint32_t grid);

}  // namespace lbm
