// lbm_internal.hpp -- context layout and kernel launchers shared by the
// library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <array>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.hpp"

namespace lbm {

constexpr int kMaxQ = 19;
constexpr int kHistCap = 8192;  // steps of force/torque history kept on the device
constexpr int kBlock = 256;     // threads per block for per-cell kernels
constexpr int kLinkChunk = 64;  // links per wavefront of the bounce-back kernel
constexpr int kIbmNbr = 128;    // point-coupling entries per Lagrangian point of capacity

// Solid as the kernels see it.
struct DevSolid {
  int32_t kind, inverted, ax, sgn, moving;
  int32_t full[3];   // box spans the whole axis
  int32_t ext[3];    // box extent per axis
  int32_t box0[3];   // box origin of a fixed solid
  uint32_t box_cells;
  FastDiv fex, fexy;  // division by ext[0] and by ext[0] * ext[1]
  uint64_t mask_off;  // first box cell of this solid in the link-mask buffer
  double c0[3], R, U[3], W[3];
  // free motion (Eq. 20): the centre is c0 at time tref (0 for prescribed
  // motion), updated after every step; cp, Up, Wp hold the state of the step
  // before (the geometry of the last collision)
  int32_t free;
  int64_t tref;
  double rho_p, Vp, Ip, grav[3];
  double cp[3], Up[3], Wp[3];
  // IBM: displacement of the solid at time tref since its Lagrangian points
  // were placed (unwrapped; the points move rigidly with it), and free motion
  // by Eq. 23 (fluid inside the solid) instead of Eq. 20
  double dsp[3];
  int32_t fm;
};

// Where one solid's links sit in the link arrays, and its chunk partials.
struct SolidLinks {
  uint32_t start, count, chunk_base, nchunks;
};

// Regions carved out of the caller's workspace (byte offsets).
struct Layout {
  size_t A, B, flags, owner0, owner1, link_cell, link_meta, link_q, box_counts, box_offsets, solid_links,
      partials, partials2, seg_link, cell_list, solids, hist, staging, fibm, lag_X, lag_dV, lag_sid, lag_Ud, lag_base, lag_w, lag_idx, lag_Fsum,
      lag_Fk, lag_Fk2, lag_Ut, lag_nptr, lag_nrow, shell_cell, shell_rowptr, shell_ent, shell_u, shell_f,
      refill, uo, cu, misc, total;
  size_t stride;  // N rounded up to whole tiles; populations take Q * stride values
  int64_t max_links, max_lag, max_shell, max_box_chunks, max_partials, max_refill;
  int32_t max_solids;
};

bool make_layout(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lag, Layout *L);

// Per-solid reduction of the bounce-back chunk partials into a history slot.
struct FtReduceArgs {
  const double *partials;
  const SolidLinks *sl;
  double *hist;
  int nsolid;
  uint64_t max_partials;
  unsigned long long *cu;  // covering / uncovering momentum of the last move (added, then cleared), or null
};

// Covering / uncovering momentum (moving bounce-back solids) is summed in
// fixed point, so that the sum does not depend on the order the nodes come
// in: 2^56 per unit of force (|sum| < 128), 2^50 per unit of torque.
__host__ __device__ inline double cu_scale(int k) { return k < 3 ? 72057594037927936.0 : 1125899906842624.0; }

// Wave-wide sum of a double (64 lanes, fixed order); lane 0 holds the result.
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Links of the 64 cells n = 64 s .. 64 s + 63 (one wavefront of a sweep):
// entries first .. first + count - 1 of the cell list.
struct SegLink {
  uint32_t first, count;
};

// Chunk partials of the bounce-back force from tabulated links: io holds the
// stored incoming and outgoing value of every link ([2][stride], compute type
// of cbytes bytes), fc the FP64 constants of Eq. 17 ([12][stride]).
struct ChunkSumArgs {
  const void *io;
  int cbytes;
  // the links (cell, direction | solid << 8, q) and the geometry their Eq. 17
  // terms are formed from (fixed solids)
  const uint32_t *lcell, *lmeta;
  const double *lq;
  const DevSolid *solids;
  int32_t nx, ny, nz, D;
  FastDiv fx, fy;
  uint64_t stride;
  const SolidLinks *sl;
  double *partials;
  uint64_t max_links, max_partials;
  uint32_t per;  // chunk units per solid
  int nsolid;
};

// Block `blk` (256 threads) reduces solids 4*blk .. 4*blk+3, one per wavefront.
__device__ inline void ft_reduce_waves(const FtReduceArgs &r, uint32_t blk) {
  const int lane = threadIdx.x & 63;
  const int s = (int)(blk * 4 + (threadIdx.x >> 6));
  if (s >= r.nsolid) return;
  const SolidLinks L = r.sl[s];
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (uint32_t c = lane; c < L.nchunks; c += 64) {
    const uint64_t at = (uint64_t)L.chunk_base + c;
    if (at >= r.max_partials) break;
    for (int k = 0; k < 6; k++) v[k] += r.partials[at * 6 + k];
  }
  for (int k = 0; k < 6; k++) {
    double tot = wave_sum(v[k]);
    if (lane == 0) {
      if (r.cu) {
        unsigned long long *q = r.cu + (uint64_t)s * 6 + k;
        tot = tot + (double)(long long)*q / cu_scale(k);
        *q = 0ull;
      }
      r.hist[(uint64_t)s * 6 + k] = tot;
    }
  }
}

}  // namespace lbm

// The opaque context.
struct lbm_ctx {
  lbm_params p;
  double rates[lbm::kMaxQ];
  bool default_rates;
  int Q, D;
  int64_t N;
  int store_bytes;
  hipStream_t stream;
  char *ws;
  size_t ws_bytes;
  lbm::Layout L;
  lbm::FastDiv fx, fy;
  // state
  int cur;  // which of A/B holds the current state (0 = A)
  int64_t t;
  bool fresh;  // no step since create / set_f / set_state
  // solids
  int method;
  int nsolid;
  bool any_moving;  // IBB solids that translate or move freely
  bool any_free;
  bool ibm_moving;  // the IBM solid translates or moves freely (one solid)
  bool ibm_free;
  int64_t solids_t;  // t at lbm_set_solids
  std::vector<lbm_solid> solids;
  std::vector<lbm::DevSolid> dsolids;
  int32_t max_box_chunks;  // per solid, for the link-builder grid
  int32_t k5_chunks;       // grid.x of the bounce-back kernel
  int64_t nlinks;
  uint64_t mask_cells;     // box cells of all solids, when their link masks fit the staging region (else 0)
  // link lists of fixed solids by sweep segment built: the sweep can apply
  // the bounce-back of the previous step itself (per-call link table in the
  // staging region, link_stride entries per array)
  bool link_lists;
  uint64_t link_stride;
  // IBM
  int n_iter;
  int delta;  // points of the IBM delta function: 4, 3 or 2
  double retraction;
  int64_t nlag;
  int64_t nshell;
  int ibm_nw;  // row stride of the point coupling (fixed IBM solids)
  // the rows hold P = sum_{k < n_iter} (I - A)^k instead of A: the iterations
  // run as one product (single contexts whose P fits the row capacity)
  bool ibm_poly = false;
  std::vector<int64_t> lag_start, lag_count;
  std::vector<double> lag_X, lag_dV;
  bool lag_user;
  int32_t prof_every;       // record events around every prof_every-th sweep (0: off)
  int64_t prof_count;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pool;  // read, free for reuse
  int sweep_policy;        // autotuned sweep policy (bit 0: non-temporal stores, bit 1: XCD-contiguous tiles; -1: not tuned yet)
  struct TuneEvent {
    int policy;
    hipEvent_t e0, e1;
  };
  std::vector<TuneEvent> tune_events;
  uint64_t tuned_key;
  double tune_us[4];       // measured sweep time of the four policies
  int tune_skipped;         // sweeps run before tuning starts
  int tune_k;               // tuning sweeps run so far
  struct ProfSpan {
    hipEvent_t e0, e1;
    int64_t launches;  // stream-collide launches between the two events
  };
  std::vector<ProfSpan> prof_events;
  std::string err;
  // batches
  struct lbm_batch *batch;  // owning batch, or null
  uint64_t version;         // bumped by every call that changes the state or the geometry
  // lbm_create_noalloc: the device whose static scratch array holds the workspace
  // (the host struct then lives in static storage too); -1 otherwise
  int noalloc_dev;
  // helpers
  void *state() const { return ws + (cur == 0 ? L.A : L.B); }
  void *other() const { return ws + (cur == 0 ? L.B : L.A); }
  template <typename T>
  T *at(size_t off) const {
    return reinterpret_cast<T *>(ws + off);
  }
};

namespace lbm {

// some axis is not periodic (lbm_params.boundary)
inline bool bounded(const lbm_ctx *c) {
  return c->p.boundary[0] != BND_PERIODIC || c->p.boundary[1] != BND_PERIODIC || c->p.boundary[2] != BND_PERIODIC;
}

int collision_kind(const lbm_ctx *c, double *sp = nullptr, double *sm = nullptr);
lbm_status destroy_ctx(lbm_ctx *c);  // frees the host side of a context

// kernels_sweep.hip
// reduce_t >= 0: the launch also reduces the bounce-back force partials of step reduce_t;
// ibm_t >= 0: it also sums the IBM force/torque of step ibm_t (forcing already done)
// link_t >= 0: the sweep applies the bounce-back of step link_t (= the step
// whose post-collision values A holds) and stores the per-link force terms of
// that step; sum_t >= 0: it also forms the chunk partials of step sum_t.
// ghost (with link_t >= 0): the link values also go to the solid nodes' slots
// of A, which only a readout of A after the call (lbm_macros, lbm_strain)
// pulls, so the last sweep of a call stores them and the others need not.
// policy: bit 0 non-temporal stores, bit 1 XCD-contiguous tile order
void launch_sweep(lbm_ctx *c, const void *A, void *B, int policy, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                  int64_t reduce_t = -1, int64_t ibm_t = -1, int64_t link_t = -1, int64_t sum_t = -1,
                  bool ghost = true);
void launch_encode_shift(lbm_ctx *c, int dir, const double *src, void *A, bool raw);
// kernels_sweep_bnd.hip: bounded domains (lbm_params.boundary)
void launch_outflow(lbm_ctx *c, const void *A, void *B);
void launch_transfer_bnd(lbm_ctx *c, int dir, const double *f, void *A, bool encode, bool raw);
void launch_bnd_uniform(lbm_ctx *c, void *A, const double *h);
void launch_decode_gather(lbm_ctx *c, int dir, const void *A, double *dst, bool raw);
void launch_refill_count(lbm_ctx *c, int64_t t, void *post);
void launch_ft_reduce_free(lbm_ctx *c, int64_t t);
void launch_ibm_ft_free(lbm_ctx *c, int64_t t);
void launch_strain(lbm_ctx *c, const void *src, double *out, int part);
void launch_macros(lbm_ctx *c, const void *src, double *out, int mode);
void launch_fill_zero(lbm_ctx *c, void *A);
struct DirVals {
  double v[kMaxQ];
};
// every slot of direction i of A set to h[i] (a uniform state)
void launch_fill_uniform(lbm_ctx *c, void *A, const double *h);
int launch_check_finite(lbm_ctx *c, const void *A, uint32_t *flag);
void launch_copy_probe(const void *src, void *dst, size_t bytes, hipStream_t s);

// kernels_boundary.hip
void launch_classify(lbm_ctx *c, int64_t t, bool full);
void launch_link_count(lbm_ctx *c, int64_t t);
void launch_link_scan(lbm_ctx *c);
void launch_link_emit(lbm_ctx *c, int64_t t);
void launch_ibb(lbm_ctx *c, void *Bpost, const void *pre, int64_t t);
FtReduceArgs ft_reduce_args(lbm_ctx *c, int64_t t);
void launch_ft_reduce(lbm_ctx *c, int64_t t);
// single contexts alternate two chunk-partial buffers by step parity
double *partials_of(lbm_ctx *c, int64_t t);
// per-call link table of fixed solids (staging region) and the per-link
// values of step t (buffer t & 1)
bool link_table_fits(const lbm_ctx *c, uint64_t stride);
void launch_link_table(lbm_ctx *c);
const void *link_rec_of(lbm_ctx *c);
void *link_io_of(lbm_ctx *c, int64_t t);
ChunkSumArgs chunk_sum_args(lbm_ctx *c, int64_t t);
uint32_t chunk_sum_blocks(const lbm_ctx *c);
void launch_chunk_sum(lbm_ctx *c, int64_t t);
hipError_t build_link_lists(lbm_ctx *c);

// kernels_ibm.hip
void launch_ibm_setup(lbm_ctx *c);
void launch_ibm_step(lbm_ctx *c, const void *A, int64_t t, bool with_ft);

}  // namespace lbm
