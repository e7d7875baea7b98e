// batch.hip -- many independent lattices advanced together.
//
// A batch owns one caller-provided device pool.  Its head holds the device
// tables (one BatchSlot of kernel arguments per member, the work lists of
// every batched launch, the step counter, per-member status words); the rest
// is handed out, first fit, as the workspaces of member contexts, so a member
// is admitted by its footprint and released without touching the others.
//
// A batched step is one launch per stage over the units of all members (the
// tiles of the sweep, the link chunks of bounce-back, the box chunks of the
// link rebuild of translating solids, the shell cells and points of IBM).
// Launches are persistent: a fixed grid walks a work list kept in device
// memory, and each member's time and state parity follow a device step
// counter, so the step is captured once in a HIP graph and the same graph
// keeps serving while members come and go.  The sweep's grid size, unit
// order and store policy are chosen by timing the first steps of the batch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "lbm_args.hpp"

using namespace lbm;

namespace {

enum {
  WL_SWEEP = 0,  // + collision kind (BGK, two-rate MRT, general MRT)
  WL_IBB = 3,
  WL_FT,
  WL_BOX,        // (solid, box chunk) units of members with translating solids
  WL_ONE,        // one unit per member with translating solids
  WL_BOX_MULTI,  // the WL_BOX units of those members that hold several solids
  WL_IBM_SPREAD,  // kSpreadCellsPerBlock shell cells per unit (kSpreadLanes lanes per cell)
  WL_IBM_LAG,
  WL_IBM_FT,
  WL_SOLID,      // one unit per member with solids (convergence check)
  WL_COUNT
};

constexpr int kGraphSteps = 8;  // steps unrolled into the multi-step graph
constexpr int kTuneRounds = 2;  // timed steps per sweep candidate

struct Member {
  lbm_ctx *c = nullptr;
  size_t off = 0, bytes = 0;
  uint64_t version = 0;
};

// Sweep launch shape: store policy, unit order, and either a persistent grid
// of `mult` blocks per compute unit or (mult 0) one block per `tpb` tiles.
struct SweepCfg {
  int nt, order, mult, tpb;
};

const SweepCfg kCands[] = {{0, 0, 4, 0},  {0, 0, 8, 0},  {0, 0, 16, 0}, {0, 1, 4, 0},  {0, 1, 8, 0},  {0, 1, 16, 0},
                           {0, 0, 0, 1},  {0, 0, 0, 2},  {0, 0, 0, 4},  {1, 0, 4, 0},  {1, 0, 8, 0},  {1, 0, 16, 0},
                           {1, 1, 4, 0},  {1, 1, 8, 0},  {1, 1, 16, 0}, {1, 0, 0, 1},  {1, 0, 0, 2},  {1, 0, 0, 4}};
constexpr int kNumCands = (int)(sizeof(kCands) / sizeof(kCands[0]));

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// tuned sweep configuration per (lattice, storage, size class), process-wide:
// the chosen candidate and the mean time of every candidate (us)
struct TuneResult {
  int chosen;
  double us[kNumCands];
};
std::map<uint64_t, TuneResult> g_batch_tune;
std::mutex g_batch_tune_mutex;

}  // namespace

struct lbm_batch {
  int lattice = 0, storage = 0, Q = 19;
  hipStream_t stream = nullptr;
  bool own_stream = false;  // created by lbm_batch_create (the caller passed none)
  char *pool = nullptr;
  size_t pool_bytes = 0, table_bytes = 0;
  int32_t max_slots = 0;
  int cus = 256;
  std::map<size_t, size_t> free_;  // offset -> bytes
  std::vector<Member> mem;         // per slot
  // device tables
  BatchSlot *d_slots = nullptr;
  int64_t *d_step = nullptr;
  uint32_t *d_status = nullptr;
  WorkList *d_wl = nullptr;
  uint16_t *d_bucket = nullptr;  // [WL_COUNT][kWlBuckets]
  uint32_t *d_start = nullptr;
  int32_t *d_mem = nullptr;
  double *d_change = nullptr;
  // composition
  bool dirty = true;
  int nlive = 0;
  uint32_t coll_mask = 0;
  bool any_ibb = false, any_moving = false, any_multi = false, any_ibm = false;
  int max_iter = 0;
  uint64_t tiles = 0;
  // graphs
  hipGraphExec_t g1 = nullptr, gk = nullptr;
  uint64_t graph_key = 0;
  // sweep tuning
  int chosen = -1;
  double chosen_us = 0.0;
  double cand_us[kNumCands] = {0};
  uint32_t totals[WL_COUNT] = {0};  // units of every work list (host copy)
  uint64_t tune_key = 0;
  int tune_next = 0;
  struct Sample {
    int cand;
    hipEvent_t e0, e1;
  };
  std::vector<Sample> samples;
  std::string err;

  WorkList *wl(int k) const { return d_wl + k; }
};

namespace {

lbm_status berr(lbm_batch *b, lbm_status st, const std::string &msg) {
  if (b) b->err = msg;
  return st;
}

#define BHIP(expr)                                                                     \
  do {                                                                                 \
    hipError_t _e = (expr);                                                            \
    if (_e != hipSuccess) return berr(b, LBM_EDEVICE, std::string(#expr ": ") + hipGetErrorString(_e)); \
  } while (0)

void destroy_graphs(lbm_batch *b) {
  for (hipGraphExec_t *g : {&b->g1, &b->gk})
    if (*g) {
      (void)hipGraphExecDestroy(*g);
      *g = nullptr;
    }
  b->graph_key = 0;
}

void drop_samples(lbm_batch *b) {
  for (auto &s : b->samples) {
    (void)hipEventDestroy(s.e0);
    (void)hipEventDestroy(s.e1);
  }
  b->samples.clear();
}

// pool allocator (first fit, 256-byte granules, coalescing)
bool pool_take(lbm_batch *b, size_t bytes, size_t *off) {
  bytes = align256(bytes);
  for (auto it = b->free_.begin(); it != b->free_.end(); ++it) {
    if (it->second < bytes) continue;
    *off = it->first;
    const size_t rest = it->second - bytes;
    const size_t at = it->first + bytes;
    b->free_.erase(it);
    if (rest) b->free_[at] = rest;
    return true;
  }
  return false;
}

void pool_give(lbm_batch *b, size_t off, size_t bytes) {
  bytes = align256(bytes);
  auto it = b->free_.emplace(off, bytes).first;
  auto nx = std::next(it);
  if (nx != b->free_.end() && it->first + it->second == nx->first) {
    it->second += nx->second;
    b->free_.erase(nx);
  }
  if (it != b->free_.begin()) {
    auto pv = std::prev(it);
    if (pv->first + pv->second == it->first) {
      pv->second += it->second;
      b->free_.erase(it);
    }
  }
}

bool member_ibb(const lbm_ctx *c) { return c->method != LBM_IBM && c->nsolid > 0 && c->k5_chunks > 0; }
bool member_moving(const lbm_ctx *c) { return member_ibb(c) && c->any_moving; }
bool member_ibm(const lbm_ctx *c) { return c->method == LBM_IBM && c->nsolid > 0 && c->nlag > 0 && c->n_iter > 0; }

// Rebuild the device tables from the members' current host state; the step
// counter restarts at 0 with t0 = t and cur0 = cur of every member.
lbm_status rebuild(lbm_batch *b) {
  BHIP(hipStreamSynchronize(b->stream));
  const int S = b->max_slots;
  std::vector<BatchSlot> slots((size_t)S);
  std::vector<std::vector<uint32_t>> units(WL_COUNT);
  std::vector<std::vector<int32_t>> who(WL_COUNT);
  b->nlive = 0;
  b->coll_mask = 0;
  b->any_ibb = b->any_moving = b->any_multi = b->any_ibm = false;
  b->max_iter = 0;
  b->tiles = 0;
  for (int k = 0; k < S; k++) {
    Member &m = b->mem[(size_t)k];
    if (!m.c) continue;
    lbm_ctx *c = m.c;
    m.version = c->version;
    b->nlive++;
    BatchSlot &bs = slots[(size_t)k];
    bs.P[0] = c->ws + c->L.A;
    bs.P[1] = c->ws + c->L.B;
    bs.cur0 = c->cur;
    bs.t0 = c->t;
    bs.method = c->method;
    bs.nsolid = c->nsolid;
    bs.n_iter = c->n_iter;
    bs.k5_chunks = c->k5_chunks;
    bs.max_box_chunks = c->max_box_chunks;
    bs.max_solids = c->L.max_solids;
    const uint32_t tiles = (uint32_t)(c->L.stride / kTile);
    bs.tiles = (int32_t)tiles;
    bs.hist = c->at<double>(c->L.hist);
    bs.status = b->d_status + 2 * (size_t)k;
    bs.lag_start = c->at<int64_t>(c->L.misc + 64);
    bs.lag_count = c->at<int64_t>(c->L.misc + 64 + 8 * (size_t)c->L.max_solids);
    fill_sweep_args(c, &bs.sw);
    fill_ibb_args(c, &bs.ib);
    fill_link_args(c, &bs.lk);
    fill_ibm_args(c, &bs.im);
    bs.ft = ft_reduce_args(c, 0);
    auto add = [&](int l, uint64_t n) {
      if (n == 0) return;
      units[l].push_back((uint32_t)n);
      who[l].push_back(k);
    };
    const int coll = collision_kind(c);
    b->coll_mask |= 1u << coll;
    add(WL_SWEEP + coll, (tiles + sweep_cpt_storage(c->store_bytes) - 1) / sweep_cpt_storage(c->store_bytes));
    b->tiles += tiles;
    if (member_ibb(c)) {
      b->any_ibb = true;
      add(WL_IBB, (uint64_t)c->k5_chunks * c->nsolid);
      add(WL_FT, (uint64_t)(c->nsolid + 3) / 4);
      if (member_moving(c)) {
        b->any_moving = true;
        add(WL_BOX, (uint64_t)c->max_box_chunks * c->nsolid);
        add(WL_ONE, 1);
        if (c->nsolid > 1) {
          b->any_multi = true;
          add(WL_BOX_MULTI, (uint64_t)c->max_box_chunks * c->nsolid);
        }
      }
    }
    if (c->nsolid > 0) add(WL_SOLID, 1);
    if (member_ibm(c)) {
      b->any_ibm = true;
      b->max_iter = std::max(b->max_iter, c->n_iter);
      add(WL_IBM_SPREAD, (uint64_t)((c->nshell + kSpreadCellsPerBlock - 1) / kSpreadCellsPerBlock));
      add(WL_IBM_LAG, (uint64_t)((c->nlag + 3) / 4));  // four points (wavefronts) per block
      add(WL_IBM_FT, (uint64_t)c->nsolid);
    }
  }
  std::vector<WorkList> wl(WL_COUNT);
  std::vector<uint32_t> start((size_t)WL_COUNT * (S + 1), 0);
  std::vector<int32_t> slot((size_t)WL_COUNT * S, 0);
  std::vector<uint16_t> bucket((size_t)WL_COUNT * kWlBuckets, 0);
  for (int l = 0; l < WL_COUNT; l++) {
    uint64_t run = 0;
    uint32_t *st = start.data() + (size_t)l * (S + 1);
    for (size_t j = 0; j < units[l].size(); j++) {
      st[j] = (uint32_t)run;
      run += units[l][j];
      slot[(size_t)l * S + j] = who[l][j];
    }
    if (run >= (1ull << 32)) return berr(b, LBM_ENOMEM, "too many units in one batched launch");
    st[units[l].size()] = (uint32_t)run;
    wl[l].total = (uint32_t)run;
    b->totals[l] = (uint32_t)run;
    wl[l].n = (int32_t)units[l].size();
    wl[l].start = b->d_start + (size_t)l * (S + 1);
    wl[l].slot = b->d_mem + (size_t)l * S;
    wl[l].bucket = b->d_bucket + (size_t)l * kWlBuckets;
    // owner of the first unit of each bucket (bucket of u: u * kWlBuckets / total)
    uint16_t *bk = bucket.data() + (size_t)l * kWlBuckets;
    size_t k = 0;
    for (uint32_t q = 0; q < kWlBuckets && run > 0; q++) {
      const uint64_t first = ((uint64_t)q * run + kWlBuckets - 1) / kWlBuckets;
      while (k + 1 < units[l].size() && st[k + 1] <= first) k++;
      bk[q] = (uint16_t)k;
    }
  }
  std::vector<uint32_t> status((size_t)2 * S, 0);
  for (int k = 0; k < S; k++)
    if (b->mem[(size_t)k].c) status[2 * (size_t)k + 1] = (uint32_t)b->mem[(size_t)k].c->nlinks;
  const int64_t zero = 0;
  BHIP(hipMemcpyAsync(b->d_slots, slots.data(), sizeof(BatchSlot) * S, hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->d_wl, wl.data(), sizeof(WorkList) * WL_COUNT, hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->d_start, start.data(), sizeof(uint32_t) * start.size(), hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->d_mem, slot.data(), sizeof(int32_t) * slot.size(), hipMemcpyHostToDevice, b->stream));
  BHIP(hipMemcpyAsync(b->d_bucket, bucket.data(), sizeof(uint16_t) * bucket.size(), hipMemcpyHostToDevice,
                      b->stream));
  BHIP(hipMemcpyAsync(b->d_status, status.data(), sizeof(uint32_t) * status.size(), hipMemcpyHostToDevice,
                      b->stream));
  BHIP(hipMemcpyAsync(b->d_step, &zero, sizeof(zero), hipMemcpyHostToDevice, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  b->dirty = false;
  return LBM_OK;
}

uint32_t grid_of(const lbm_batch *b, int mult) { return (uint32_t)std::max(1, mult * b->cus); }

// One batched step (enqueue only); e0/e1 (optional) time the sweep launches.
void enqueue_step(lbm_batch *b, const SweepCfg &cfg, hipEvent_t e0, hipEvent_t e1) {
  const BatchLaunch bl{b->d_slots, b->d_step, b->stream, b->Q, b->storage};
  if (b->any_ibm)
    launch_ibm_batch(bl, b->wl(WL_IBM_SPREAD), b->wl(WL_IBM_LAG), b->wl(WL_IBM_FT), b->max_iter, grid_of(b, 4));
  int first = -1, lastc = -1;
  for (int k = 0; k < 3; k++)
    if (b->coll_mask & (1u << k)) {
      if (first < 0) first = k;
      lastc = k;
    }
  for (int k = 0; k < 3; k++)
    if (b->coll_mask & (1u << k))
      launch_sweep_batch(bl, b->wl(WL_SWEEP + k), k, cfg.nt, cfg.order,
                         cfg.mult ? grid_of(b, cfg.mult)
                                  : std::max<uint32_t>(1, (b->totals[WL_SWEEP + k] + cfg.tpb - 1) / cfg.tpb),
                         k == first ? e0 : nullptr, k == lastc ? e1 : nullptr);
  if (b->any_ibb) {
    launch_ibb_batch(bl, b->wl(WL_IBB), grid_of(b, 32));
    launch_ft_batch(bl, b->wl(WL_FT), std::min<uint32_t>(grid_of(b, 4), 1024));
    if (b->any_moving)
      launch_move_batch(bl, b->wl(WL_BOX), b->wl(WL_BOX_MULTI), b->wl(WL_ONE), b->any_multi, grid_of(b, 8));
  }
  launch_tick(b->stream, b->d_step);
}

uint64_t size_class(const lbm_batch *b) {
  uint64_t c = 0;
  while ((1ull << c) < b->tiles) c++;
  return ((uint64_t)b->Q * 8 + (uint64_t)b->storage) * 64 + c;
}

// composition summary that decides the captured graphs
uint64_t graph_key_of(const lbm_batch *b) {
  uint64_t k = 1;
  k = k * 8 + b->coll_mask;
  k = k * 2 + (b->any_ibb ? 1 : 0);
  k = k * 2 + (b->any_moving ? 1 : 0);
  k = k * 2 + (b->any_multi ? 1 : 0);
  k = k * 2 + (b->any_ibm ? 1 : 0);
  k = k * 64 + (uint64_t)b->max_iter;
  k = k * 64 + (uint64_t)b->chosen;
  if (b->chosen >= 0 && kCands[b->chosen].mult == 0)  // grid = tiles: re-capture when they change
    for (int l = WL_SWEEP; l < WL_SWEEP + 3; l++) k = k * 1000003ull + b->totals[l];
  return k;
}

lbm_status capture(lbm_batch *b, int steps, hipGraphExec_t *out) {
  hipGraph_t g = nullptr;
  BHIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  for (int s = 0; s < steps; s++) enqueue_step(b, kCands[b->chosen], nullptr, nullptr);
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (e != hipSuccess) return berr(b, LBM_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return berr(b, LBM_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
  return LBM_OK;
}

lbm_status ensure_graphs(lbm_batch *b) {
  const uint64_t key = graph_key_of(b);
  if (b->g1 && b->graph_key == key) return LBM_OK;
  destroy_graphs(b);
  lbm_status st = capture(b, 1, &b->g1);
  if (st == LBM_OK) st = capture(b, kGraphSteps, &b->gk);
  if (st != LBM_OK) {
    destroy_graphs(b);
    return st;
  }
  b->graph_key = key;
  return LBM_OK;
}

// Online tuning: the first steps of a size class run eagerly, each with one
// sweep candidate timed by events on its dispatches (round-robin, so drift
// hits every candidate alike); the fastest mean wins.  Every candidate
// computes the same values.
lbm_status tune_finish(lbm_batch *b) {
  BHIP(hipStreamSynchronize(b->stream));
  double sum[kNumCands] = {0};
  int cnt[kNumCands] = {0};
  for (auto &s : b->samples) {
    float ms = 0.0f;
    BHIP(hipEventElapsedTime(&ms, s.e0, s.e1));
    sum[s.cand] += ms;
    cnt[s.cand]++;
  }
  drop_samples(b);
  int best = 0;
  double best_us = 1e300;
  for (int k = 0; k < kNumCands; k++) {
    b->cand_us[k] = cnt[k] ? 1e3 * sum[k] / cnt[k] : -1.0;
    if (cnt[k] && b->cand_us[k] < best_us) {
      best_us = b->cand_us[k];
      best = k;
    }
  }
  b->chosen = best;
  b->chosen_us = best_us;
  TuneResult r;
  r.chosen = best;
  for (int k = 0; k < kNumCands; k++) r.us[k] = b->cand_us[k];
  std::lock_guard<std::mutex> g(g_batch_tune_mutex);
  g_batch_tune[b->tune_key] = r;
  return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_batch_table_bytes(int32_t max_slots) {
  if (max_slots <= 0) return 0;
  const size_t S = (size_t)max_slots;
  return align256(sizeof(BatchSlot) * S) + 256 + align256(8 * S) + align256(sizeof(WorkList) * WL_COUNT) +
         align256(4 * WL_COUNT * (S + 1)) + align256(4 * WL_COUNT * S) + align256(8 * S) +
         align256(2 * WL_COUNT * (size_t)kWlBuckets);
}

lbm_status lbm_batch_create(int32_t lattice, int32_t storage, int32_t max_slots, void *dev_pool, size_t pool_bytes,
                            void *hip_stream, lbm_batch **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  if ((lattice != LBM_D2Q9 && lattice != LBM_D3Q19) || storage < LBM_F64 || storage > LBM_F16_SR) return LBM_EINVAL;
  if (max_slots <= 0 || max_slots > 65536 || !dev_pool || ((uintptr_t)dev_pool & 255)) return LBM_EINVAL;
  const size_t tb = lbm_batch_table_bytes(max_slots);
  if (pool_bytes < tb + 256) return LBM_ENOMEM;
  lbm_batch *b = new (std::nothrow) lbm_batch();
  if (!b) return LBM_ENOMEM;
  b->lattice = lattice;
  b->storage = storage;
  b->Q = lattice == LBM_D2Q9 ? 9 : 19;
  b->pool = static_cast<char *>(dev_pool);
  b->pool_bytes = pool_bytes;
  b->table_bytes = tb;
  b->max_slots = max_slots;
  b->mem.resize((size_t)max_slots);
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
    b->cus = cus;
  // the caller's stream, else one of the batch's own (default priority); the
  // steps are captured as graphs, which the null stream cannot hold
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess) {
      delete b;
      return LBM_EDEVICE;
    }
    b->own_stream = true;
  }
  char *p = b->pool;
  const size_t S = (size_t)max_slots;
  b->d_slots = reinterpret_cast<BatchSlot *>(p);
  p += align256(sizeof(BatchSlot) * S);
  b->d_step = reinterpret_cast<int64_t *>(p);
  p += 256;
  b->d_status = reinterpret_cast<uint32_t *>(p);
  p += align256(8 * S);
  b->d_wl = reinterpret_cast<WorkList *>(p);
  p += align256(sizeof(WorkList) * WL_COUNT);
  b->d_start = reinterpret_cast<uint32_t *>(p);
  p += align256(4 * WL_COUNT * (S + 1));
  b->d_mem = reinterpret_cast<int32_t *>(p);
  p += align256(4 * WL_COUNT * S);
  b->d_change = reinterpret_cast<double *>(p);
  p += align256(8 * S);
  b->d_bucket = reinterpret_cast<uint16_t *>(p);
  b->free_[tb] = (pool_bytes - tb) & ~size_t(255);
  if (rebuild(b) != LBM_OK) {
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return LBM_EDEVICE;
  }
  *out = b;
  return LBM_OK;
}

lbm_status lbm_batch_admit(lbm_batch *b, const lbm_params *p, int32_t max_solids, int64_t max_links,
                           int64_t max_lagrangian, lbm_ctx **out) {
  if (!b || !p || !out) return LBM_EINVAL;
  *out = nullptr;
  if (p->lattice != b->lattice || p->storage != b->storage)
    return berr(b, LBM_EINVAL, "lattice and storage must match the batch");
  const size_t need = lbm_workspace_bytes(p, max_solids, max_links, max_lagrangian);
  if (!need) return berr(b, LBM_EINVAL, "invalid lattice parameters");
  if (p->boundary[0] != BND_PERIODIC || p->boundary[1] != BND_PERIODIC || p->boundary[2] != BND_PERIODIC)
    return berr(b, LBM_EUNSUPPORTED, "batches take periodic lattices");
  // the batched sweep forms offsets in 32 bits
  if ((double)p->nx * p->ny * p->nz * (p->lattice == LBM_D2Q9 ? 9 : 19) >= 2147483648.0)
    return berr(b, LBM_EINVAL, "a batch member holds fewer than 2^31 values per population array");
  int slot = -1;
  for (int k = 0; k < b->max_slots; k++)
    if (!b->mem[(size_t)k].c) {
      slot = k;
      break;
    }
  if (slot < 0) return berr(b, LBM_EAGAIN, "every slot of the batch is taken");
  size_t off = 0;
  if (!pool_take(b, need, &off)) return berr(b, LBM_EAGAIN, "not enough contiguous pool memory");
  lbm_ctx *c = nullptr;
  const lbm_status st = lbm_create(p, max_solids, max_links, max_lagrangian, b->pool + off, align256(need), b->stream,
                                   &c);
  if (st != LBM_OK) {
    pool_give(b, off, need);
    return berr(b, st, "member creation failed");
  }
  c->batch = b;
  Member &m = b->mem[(size_t)slot];
  m.c = c;
  m.off = off;
  m.bytes = need;
  m.version = c->version;
  b->dirty = true;
  *out = c;
  return LBM_OK;
}

lbm_status lbm_batch_release(lbm_batch *b, lbm_ctx *c) {
  if (!b || !c || c->batch != b) return LBM_EINVAL;
  for (auto &m : b->mem) {
    if (m.c != c) continue;
    BHIP(hipStreamSynchronize(b->stream));
    c->batch = nullptr;
    (void)destroy_ctx(c);
    pool_give(b, m.off, m.bytes);
    m = Member{};
    b->dirty = true;
    return LBM_OK;
  }
  return LBM_EINVAL;
}

lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps) {
  if (!b || nsteps < 0) return LBM_EINVAL;
  if (nsteps == 0) return LBM_OK;
  for (auto &m : b->mem)
    if (m.c && m.c->version != m.version) b->dirty = true;
  if (b->dirty) {
    const lbm_status st = rebuild(b);
    if (st != LBM_OK) return st;
  }
  if (b->nlive == 0) return LBM_OK;
  // sweep configuration of this size class: cached, or tuned on the first steps
  const uint64_t key = size_class(b);
  if (b->tune_key != key) {
    drop_samples(b);
    b->tune_key = key;
    b->tune_next = 0;
    b->chosen = -1;
    std::lock_guard<std::mutex> g(g_batch_tune_mutex);
    auto it = g_batch_tune.find(key);
    if (it != g_batch_tune.end()) {
      b->chosen = it->second.chosen;
      b->chosen_us = it->second.us[b->chosen];
      for (int k = 0; k < kNumCands; k++) b->cand_us[k] = it->second.us[k];
    }
  }
  int64_t done = 0;
  while (b->chosen < 0 && done < nsteps) {
    const int cand = b->tune_next % kNumCands;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    b->samples.push_back({cand, e0, e1});
    enqueue_step(b, kCands[cand], e0, e1);
    BHIP(hipGetLastError());
    b->tune_next++;
    done++;
    if (b->tune_next >= kNumCands * kTuneRounds) {
      const lbm_status st = tune_finish(b);
      if (st != LBM_OK) return st;
    }
  }
  if (done < nsteps) {
    lbm_status st = ensure_graphs(b);
    if (st != LBM_OK) return st;
    int64_t left = nsteps - done;
    for (; left >= kGraphSteps; left -= kGraphSteps) BHIP(hipGraphLaunch(b->gk, b->stream));
    for (; left > 0; left--) BHIP(hipGraphLaunch(b->g1, b->stream));
  }
  for (auto &m : b->mem) {
    if (!m.c) continue;
    m.c->t += nsteps;
    m.c->cur ^= (int)(nsteps & 1);
    m.c->fresh = false;
  }
  if (b->any_moving) {
    // capacity checks of the translating solids' rebuilt link tables
    std::vector<uint32_t> status((size_t)2 * b->max_slots);
    BHIP(hipMemcpyAsync(status.data(), b->d_status, sizeof(uint32_t) * status.size(), hipMemcpyDeviceToHost,
                        b->stream));
    BHIP(hipStreamSynchronize(b->stream));
    for (int k = 0; k < b->max_slots; k++) {
      lbm_ctx *c = b->mem[(size_t)k].c;
      if (!c || !member_moving(c)) continue;
      c->nlinks = status[2 * (size_t)k + 1];
      const uint32_t bad = status[2 * (size_t)k];
      if (bad & BS_LINKS_OVERFLOW) c->err = "more boundary links than max_links";
      else if (bad & BS_CHUNKS_OVERFLOW) c->err = "a translating solid outgrew its link headroom";
      if (bad) return berr(b, LBM_ENOMEM, "a member exceeded its link capacity: " + c->err);
    }
  }
  return LBM_OK;
}

lbm_status lbm_batch_sync(lbm_batch *b) {
  if (!b) return LBM_EINVAL;
  BHIP(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

lbm_status lbm_batch_info(lbm_batch *b, int32_t *members, size_t *bytes_free, size_t *largest_free,
                          int64_t *total_cells) {
  if (!b) return LBM_EINVAL;
  int32_t n = 0;
  int64_t cells = 0;
  for (auto &m : b->mem)
    if (m.c) {
      n++;
      cells += m.c->N;
    }
  size_t fr = 0, big = 0;
  for (auto &f : b->free_) {
    fr += f.second;
    big = std::max(big, f.second);
  }
  if (members) *members = n;
  if (bytes_free) *bytes_free = fr;
  if (largest_free) *largest_free = big;
  if (total_cells) *total_cells = cells;
  return LBM_OK;
}

lbm_status lbm_batch_tune_info(lbm_batch *b, int32_t *nontemporal, int32_t *order, int32_t *blocks,
                               int32_t *tiles_per_block, double *sweep_us) {
  if (!b) return LBM_EINVAL;
  if (b->chosen < 0) return berr(b, LBM_ESTATE, "the sweep is not tuned yet");
  const SweepCfg &c = kCands[b->chosen];
  if (nontemporal) *nontemporal = c.nt;
  if (order) *order = c.order;
  if (blocks) *blocks = c.mult ? (int32_t)grid_of(b, c.mult) : 0;
  if (tiles_per_block) *tiles_per_block = c.tpb;
  if (sweep_us) *sweep_us = b->chosen_us;
  return LBM_OK;
}

int32_t lbm_batch_tune_table(lbm_batch *b, int32_t cap, int32_t *nontemporal, int32_t *order, int32_t *blocks,
                             int32_t *tiles_per_block, double *sweep_us) {
  if (!b) return 0;
  const int n = std::min<int32_t>(cap, kNumCands);
  for (int k = 0; k < n; k++) {
    if (nontemporal) nontemporal[k] = kCands[k].nt;
    if (order) order[k] = kCands[k].order;
    if (blocks) blocks[k] = kCands[k].mult ? (int32_t)grid_of(b, kCands[k].mult) : 0;
    if (tiles_per_block) tiles_per_block[k] = kCands[k].tpb;
    if (sweep_us) sweep_us[k] = b->chosen >= 0 ? b->cand_us[k] : -1.0;
  }
  return kNumCands;
}

lbm_status lbm_batch_time_sweep(lbm_batch *b, int64_t nsteps, double *sweep_us) {
  if (!b || nsteps <= 0 || !sweep_us) return LBM_EINVAL;
  if (b->dirty) {
    const lbm_status st = rebuild(b);
    if (st != LBM_OK) return st;
  }
  for (auto &m : b->mem)
    if (m.c && m.c->version != m.version) return berr(b, LBM_ESTATE, "members changed since the last batch step");
  if (b->chosen < 0) return berr(b, LBM_ESTATE, "the sweep is not tuned yet");
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev((size_t)nsteps);
  for (auto &e : ev) {
    BHIP(hipEventCreate(&e.first));
    BHIP(hipEventCreate(&e.second));
  }
  for (int64_t s = 0; s < nsteps; s++)
    enqueue_step(b, kCands[b->chosen], ev[(size_t)s].first, ev[(size_t)s].second);
  BHIP(hipGetLastError());
  for (auto &m : b->mem) {
    if (!m.c) continue;
    m.c->t += nsteps;
    m.c->cur ^= (int)(nsteps & 1);
    m.c->fresh = false;
  }
  BHIP(hipStreamSynchronize(b->stream));
  double tot = 0.0;
  for (auto &e : ev) {
    float ms = 0.0f;
    BHIP(hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  *sweep_us = 1e3 * tot / (double)nsteps;
  return LBM_OK;
}

lbm_status lbm_batch_force_change(lbm_batch *b, int64_t lag, lbm_ctx **members, double *change) {
  if (!b || !members || !change || lag <= 0) return LBM_EINVAL;
  if (lag >= lbm_history_capacity()) return berr(b, LBM_EINVAL, "lag beyond the force history");
  for (auto &m : b->mem)
    if (m.c && m.c->version != m.version) b->dirty = true;
  if (b->dirty) {
    const lbm_status st = rebuild(b);
    if (st != LBM_OK) return st;
  }
  const BatchLaunch bl{b->d_slots, b->d_step, b->stream, b->Q, b->storage};
  launch_force_change(bl, b->wl(WL_SOLID), lag, b->d_change, std::min<uint32_t>(grid_of(b, 1), 1024));
  BHIP(hipGetLastError());
  std::vector<double> out((size_t)b->max_slots);
  BHIP(hipMemcpyAsync(out.data(), b->d_change, sizeof(double) * out.size(), hipMemcpyDeviceToHost, b->stream));
  BHIP(hipStreamSynchronize(b->stream));
  for (int k = 0; k < b->max_slots; k++) {
    lbm_ctx *c = b->mem[(size_t)k].c;
    members[k] = c;
    change[k] = (c && c->nsolid > 0) ? out[(size_t)k] : -1.0;
  }
  return LBM_OK;
}

lbm_status lbm_batch_poll(lbm_batch *b, int64_t lag, double tol, lbm_ctx **converged, int32_t cap, int32_t *n) {
  if (!b || !n || !(tol > 0.0) || cap < 0 || (cap > 0 && !converged)) return LBM_EINVAL;
  std::vector<lbm_ctx *> members((size_t)b->max_slots);
  std::vector<double> change((size_t)b->max_slots);
  const lbm_status st = lbm_batch_force_change(b, lag, members.data(), change.data());
  if (st != LBM_OK) return st;
  int32_t k = 0;
  for (int s = 0; s < b->max_slots; s++)
    if (members[(size_t)s] && change[(size_t)s] >= 0.0 && change[(size_t)s] < tol) {
      if (k < cap) converged[k] = members[(size_t)s];
      k++;
    }
  *n = k;
  return LBM_OK;
}

void *lbm_batch_stream(lbm_batch *b) { return b ? (void *)b->stream : nullptr; }

const char *lbm_batch_last_error(const lbm_batch *b) { return b ? b->err.c_str() : "null batch"; }

lbm_status lbm_batch_destroy(lbm_batch *b) {
  if (!b) return LBM_EINVAL;
  (void)hipStreamSynchronize(b->stream);
  for (auto &m : b->mem)
    if (m.c) {
      m.c->batch = nullptr;
      (void)destroy_ctx(m.c);
      m = Member{};
    }
  destroy_graphs(b);
  drop_samples(b);
  if (b->own_stream) (void)hipStreamDestroy(b->stream);
  delete b;
  return LBM_OK;
}

}  // extern "C"
