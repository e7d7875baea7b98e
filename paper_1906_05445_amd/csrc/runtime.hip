// runtime.hip -- host side of liblbm.so: the C ABI of include/lbm.h.
//
// The context lives in a caller-owned device workspace carved into fixed
// regions (populations A/B, node flags, solid ownership, boundary links,
// Lagrangian data, force history, staging); the library itself never
// allocates device memory.  Every call enqueues work on the caller's stream;
// only the readout calls synchronise it.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>

#include "lbm_internal.hpp"

using namespace lbm;

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// bytes of the static workspace array behind lbm_create_noalloc
constexpr size_t kNoAllocBytes = size_t(64) << 20;

int csize_of(int storage) { return storage == LBM_F64 ? 8 : 4; }
int ssize_of(int storage) { return storage == LBM_F64 ? 8 : (storage == LBM_F32_DEV ? 4 : 2); }

FastDiv make_div(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) s++;
  f.s = s;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << s) - d)) / d) + 1);
  return f;
}

bool set_err(lbm_ctx *c, const char *msg) {
  if (c) c->err = msg;
  return false;
}

lbm_status hip_check(lbm_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return LBM_OK;
  if (c) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return LBM_EDEVICE;
}

#define HIPCALL(expr)                                    \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return hip_check(c, _e, #expr); \
  } while (0)

int qof(int lattice) { return lattice == LBM_D2Q9 ? 9 : 19; }

bool valid_params(const lbm_params *p) {
  if (!p) return false;
  if (p->lattice != LBM_D2Q9 && p->lattice != LBM_D3Q19) return false;
  if (p->collision != LBM_BGK && p->collision != LBM_MRT) return false;
  if (p->storage < LBM_F64 || p->storage > LBM_F16_SR) return false;
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return false;
  if (p->lattice == LBM_D2Q9 && p->nz != 1) return false;
  // cell indices are 32-bit (and sums of two of them stay below 2^32); offsets
  // into the population arrays are 64-bit where Q * cells reaches 2^32
  const double N = (double)p->nx * p->ny * p->nz;
  if (N >= 2147483648.0) return false;
  if (!(p->tau > 0.5) || !std::isfinite(p->tau)) return false;
  for (int k = 0; k < 3; k++)
    if (!std::isfinite(p->body_force[k])) return false;
  // domain boundaries (Sec. 3.4): OPEN on x only, D2Q9 keeps z periodic
  for (int k = 0; k < 3; k++) {
    if (p->boundary[k] < BND_PERIODIC || p->boundary[k] > BND_OPEN) return false;
    if (p->boundary[k] == BND_OPEN && k != 0) return false;
  }
  if (p->lattice == LBM_D2Q9 && p->boundary[2] != BND_PERIODIC) return false;
  if (p->boundary[0] == BND_OPEN && p->nx < 8) return false;
  if (!std::isfinite(p->inflow) || std::fabs(p->inflow) >= 0.3) return false;
  if (p->cover_momentum != 0 && p->cover_momentum != 1) return false;
  return true;
}

// Default relaxation rates of the MRT collision (the paper does not print
// S): 1/tau on every even non-conserved moment, s_odd on the odd ones with
// (tau - 1/2)(1/s_odd - 1/2) = 3/16; conserved rows 1 (no effect).
void default_rates(int Q, double tau, double *r) {
  const double snu = 1.0 / tau;
  const double sodd = 1.0 / (0.5 + (3.0 / 16.0) / (tau - 0.5));
  for (int k = 0; k < Q; k++) {
    const bool cons = Q == 9 ? conserved<9>(k) : conserved<19>(k);
    const bool odd = Q == 9 ? odd_row<9>(k) : odd_row<19>(k);
    r[k] = cons ? 1.0 : (odd ? sodd : snu);
  }
}

}  // namespace

namespace lbm {

bool make_layout(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lag, Layout *L) {
  if (!valid_params(p)) return false;
  const int Q = qof(p->lattice);
  const int64_t N = (int64_t)p->nx * p->ny * p->nz;
  const int s = ssize_of(p->storage), cs = csize_of(p->storage);
  if (max_solids <= 0) max_solids = 1;
  if (max_solids > 65534) return false;
  if (max_links <= 0) max_links = std::max<int64_t>(65536, N / 2);
  if (max_lag < 0) max_lag = 0;  // no IBM space
  else if (max_lag == 0) max_lag = std::max<int64_t>(1024, N / 64);
  if (max_links >= (1ll << 32) || max_lag >= (1ll << 26)) return false;
  Layout l{};
  l.stride = (size_t)((N + kTile - 1) / kTile * kTile);  // whole tiles
  l.max_links = max_links;
  l.max_lag = max_lag;
  // cells in the points' delta supports: 16 per point of capacity (a mesh of
  // about one point per unit area, Sec. 2.1, takes 4 to 8)
  l.max_shell = std::min<int64_t>(N, 16 * max_lag);
  l.max_box_chunks = (N + kBlock - 1) / kBlock;
  l.max_partials = (max_links + kLinkChunk - 1) / kLinkChunk + max_solids;
  l.max_solids = max_solids;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align256(o + bytes);
    return at;
  };
  l.A = take((size_t)Q * l.stride * s);
  l.B = take((size_t)Q * l.stride * s);
  l.flags = take((size_t)N);
  l.owner0 = take((size_t)N * 2);
  l.owner1 = take((size_t)N * 2);
  l.link_cell = take((size_t)max_links * 4);
  l.link_meta = take((size_t)max_links * 4);
  l.link_q = take((size_t)max_links * 8);
  l.box_counts = take((size_t)max_solids * l.max_box_chunks * 4);
  l.box_offsets = take((size_t)max_solids * l.max_box_chunks * 4);
  l.solid_links = take((size_t)max_solids * sizeof(SolidLinks));
  l.partials = take((size_t)l.max_partials * 6 * 8);
  l.partials2 = take((size_t)l.max_partials * 6 * 8);
  l.seg_link = take((size_t)((N + 63) / 64) * 8);
  l.cell_list = take((size_t)max_links * 4);
  l.solids = take((size_t)max_solids * sizeof(DevSolid));
  l.hist = take((size_t)kHistCap * max_solids * 6 * 8);
  l.staging = take((size_t)4 * N * 8);
  l.fibm = take(max_lag > 0 ? (size_t)3 * l.stride * cs : 0);
  l.lag_X = take((size_t)max_lag * 24);
  l.lag_dV = take((size_t)max_lag * 8);
  l.lag_sid = take((size_t)max_lag * 4);
  l.lag_Ud = take((size_t)max_lag * 24);
  l.lag_base = take((size_t)max_lag * 12);
  l.lag_w = take((size_t)max_lag * 96);
  l.lag_idx = take((size_t)max_lag * 256);
  l.lag_Fsum = take((size_t)max_lag * 24);
  l.lag_Fk = take((size_t)max_lag * 4 * cs);
  l.lag_Fk2 = take((size_t)max_lag * 4 * cs);
  l.lag_Ut = take((size_t)max_lag * 3 * cs);
  l.lag_nptr = take((size_t)max_lag * 4);
  l.lag_nrow = take((size_t)max_lag * kIbmNbr * (cs == 8 ? 16 : 8));
  l.shell_cell = take((size_t)l.max_shell * 4);
  l.shell_rowptr = take((size_t)(l.max_shell + 1) * 4);
  l.shell_ent = take((size_t)max_lag * 64 * 4);
  l.shell_u = take((size_t)3 * l.max_shell * cs);
  l.shell_f = take((size_t)3 * l.max_shell * cs);
  l.max_refill = std::max<int64_t>(4096, N / 16);
  l.refill = take((size_t)l.max_refill * 8);
  l.uo = take(p->boundary[0] == BND_OPEN ? (size_t)p->ny * p->nz * cs : 0);
  l.cu = take((size_t)max_solids * 6 * 8);
  l.misc = take((size_t)64 + 16 * (size_t)max_solids + 64);
  l.total = o;
  *L = l;
  return true;
}

}  // namespace lbm

// ----------------------------------------------------------------------------
// Lagrangian meshes (Sec. 2.1): geodesic sphere with about one point per unit
// area, circles and rings with spacing about 1.
// ----------------------------------------------------------------------------
namespace {

struct V3 {
  double x, y, z;
};

void icosphere(const double c[3], double R, std::vector<double> &X, double &dV) {
  const double ph = (1.0 + std::sqrt(5.0)) / 2.0;
  std::vector<V3> v;
  for (double a : {-1.0, 1.0})
    for (double b : {-ph, ph}) {
      v.push_back({0.0, a, b});
      v.push_back({a, b, 0.0});
      v.push_back({b, 0.0, a});
    }
  std::sort(v.begin(), v.end(), [](const V3 &p, const V3 &q) {
    if (p.x != q.x) return p.x < q.x;
    if (p.y != q.y) return p.y < q.y;
    return p.z < q.z;
  });
  const int nv = (int)v.size();
  auto d2 = [&](int i, int j) {
    const double dx = v[i].x - v[j].x, dy = v[i].y - v[j].y, dz = v[i].z - v[j].z;
    return dx * dx + dy * dy + dz * dz;
  };
  std::vector<std::pair<int, int>> edges;
  for (int i = 0; i < nv; i++)
    for (int j = i + 1; j < nv; j++)
      if (std::fabs(d2(i, j) - 4.0) < 1e-9) edges.push_back({i, j});
  auto adj = [&](int i, int j) { return std::fabs(d2(i, j) - 4.0) < 1e-9; };
  std::vector<std::array<int, 3>> faces;
  for (auto &e : edges)
    for (int k = e.second + 1; k < nv; k++)
      if (adj(e.first, k) && adj(e.second, k)) faces.push_back({e.first, e.second, k});
  const int n = std::max(1, (int)std::nearbyint(R * std::sqrt(4.0 * M_PI / 10.0)));
  std::vector<V3> P(v.begin(), v.end());
  for (auto &e : edges)
    for (int k = 1; k < n; k++) {
      const V3 &a = v[e.first], &b = v[e.second];
      P.push_back({((n - k) * a.x + k * b.x) / n, ((n - k) * a.y + k * b.y) / n, ((n - k) * a.z + k * b.z) / n});
    }
  for (auto &f : faces)
    for (int i = 1; i < n; i++)
      for (int j = 1; j < n - i; j++) {
        const int k = n - i - j;
        const V3 &a = v[f[0]], &b = v[f[1]], &cc = v[f[2]];
        P.push_back({(i * a.x + j * b.x + k * cc.x) / n, (i * a.y + j * b.y + k * cc.y) / n,
                     (i * a.z + j * b.z + k * cc.z) / n});
      }
  X.clear();
  for (auto &p : P) {
    const double nr = std::sqrt(p.x * p.x + p.y * p.y + p.z * p.z);
    X.push_back(c[0] + R * (p.x / nr));
    X.push_back(c[1] + R * (p.y / nr));
    X.push_back(c[2] + R * (p.z / nr));
  }
  dV = 4.0 * M_PI * R * R / (double)P.size();
}

void circle(const double c[3], double R, double z, std::vector<double> &X, double &dV) {
  const int n = std::max(3, (int)std::nearbyint(2.0 * M_PI * R));
  for (int l = 0; l < n; l++) {
    const double a = 2.0 * M_PI * l / n;
    X.push_back(c[0] + R * std::cos(a));
    X.push_back(c[1] + R * std::sin(a));
    X.push_back(z);
  }
  dV = 2.0 * M_PI * R / n;
}

}  // namespace

// ----------------------------------------------------------------------------
// C ABI
// ----------------------------------------------------------------------------
// ----------------------------------------------------------------------------
// lbm_create_noalloc: the workspace of one context per device in a file-scope
// device array.  In host code `scratch` names a host-side stand-in, not device
// memory; its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// used.  The host struct of the context lives in static storage, so the call
// allocates nothing on the device or the host.
// ----------------------------------------------------------------------------
static __device__ __align__(256) char scratch[kNoAllocBytes];

namespace {
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mutex;
char *g_scratch_ptr[kNoAllocDevices];  // device address of `scratch` per device (null: not taken yet)
bool g_noalloc_busy[kNoAllocDevices];  // a context lives in that device's array
alignas(lbm_ctx) unsigned char g_noalloc_ctx[kNoAllocDevices][sizeof(lbm_ctx)];
}  // namespace

// Releases the static slot of a context made by lbm_create_noalloc (the host
// struct is destroyed in place).
static void release_noalloc(lbm_ctx *c) {
  const int dev = c->noalloc_dev;
  c->~lbm_ctx();
  std::lock_guard<std::mutex> g(g_noalloc_mutex);
  g_noalloc_busy[dev] = false;
}

lbm_status lbm::destroy_ctx(lbm_ctx *c) {
  (void)hipStreamSynchronize(c->stream);
  for (auto &e : c->prof_events) {
    (void)hipEventDestroy(e.e0);
    (void)hipEventDestroy(e.e1);
  }
  for (auto &e : c->prof_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (auto &t : c->tune_events) {
    (void)hipEventDestroy(t.e0);
    (void)hipEventDestroy(t.e1);
  }
  if (c->noalloc_dev >= 0) release_noalloc(c);
  else delete c;
  return LBM_OK;
}

extern "C" {

const char *lbm_status_string(lbm_status st) {
  switch (st) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace or capacity too small";
    case LBM_EDEVICE: return "HIP runtime error";
    case LBM_EDIVERGED: return "non-finite populations";
    case LBM_EUNSUPPORTED: return "unsupported combination";
    case LBM_ESTATE: return "call out of order";
    case LBM_EAGAIN: return "admission deferred";
    default: return "unknown status";
  }
}

const char *lbm_last_error(const lbm_ctx *c) { return c ? c->err.c_str() : "null context"; }

int64_t lbm_history_capacity(void) { return kHistCap; }

int64_t lbm_time(const lbm_ctx *c) { return c ? c->t : -1; }

size_t lbm_workspace_bytes(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian) {
  Layout L;
  if (!make_layout(p, max_solids, max_links, max_lagrangian, &L)) return 0;
  return L.total;
}

// Parameters checked and the workspace layout of a context (lbm_create and
// lbm_create_noalloc).
static lbm_status check_create(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian,
                               Layout *L) {
  if (!p || !make_layout(p, max_solids, max_links, max_lagrangian, L)) return LBM_EINVAL;
  if (p->collision == LBM_MRT && p->rates)
    for (int k = 0; k < qof(p->lattice); k++)
      if (!std::isfinite(p->rates[k]) || p->rates[k] < 0.0 || p->rates[k] >= 2.0) return LBM_EINVAL;
  return LBM_OK;
}

// A new context in the host storage `c` over the device workspace ws: the
// rest state, cleared flags and no owner (every byte of the workspace that is
// read before it is written is set here, so a reused workspace carries
// nothing over).
static lbm_status init_ctx(lbm_ctx *c, const lbm_params *p, const Layout &L, void *dev_workspace, size_t ws_bytes,
                           void *hip_stream) {
  c->p = *p;
  c->p.rates = nullptr;
  c->Q = qof(p->lattice);
  c->D = p->lattice == LBM_D2Q9 ? 2 : 3;
  c->N = (int64_t)p->nx * p->ny * p->nz;
  c->store_bytes = ssize_of(p->storage);
  c->default_rates = !(p->collision == LBM_MRT && p->rates);
  if (c->default_rates) default_rates(c->Q, p->tau, c->rates);
  else
    for (int k = 0; k < c->Q; k++) c->rates[k] = p->rates[k];
  c->stream = static_cast<hipStream_t>(hip_stream);
  c->ws = static_cast<char *>(dev_workspace);
  c->ws_bytes = ws_bytes;
  c->L = L;
  c->fx = make_div((uint32_t)p->nx);
  c->fy = make_div((uint32_t)p->ny);
  c->cur = 0;
  c->t = 0;
  c->method = LBM_BB;
  c->nsolid = 0;
  c->any_moving = false;
  c->any_free = false;
  c->ibm_moving = false;
  c->ibm_free = false;
  c->solids_t = 0;
  c->max_box_chunks = 0;
  c->k5_chunks = 0;
  c->nlinks = 0;
  c->n_iter = 5;
  c->delta = 4;
  c->retraction = 0.0;
  c->nlag = 0;
  c->nshell = 0;
  c->ibm_nw = 64;
  c->lag_user = false;
  c->prof_every = 0;
  c->prof_count = 0;
  c->sweep_policy = -1;
  c->tuned_key = 0;
  for (double &u : c->tune_us) u = 0.0;
  c->fresh = true;
  c->batch = nullptr;
  c->version = 0;
  c->noalloc_dev = -1;
  // rest state, cleared flags and ownership
  hipError_t e = hipMemsetAsync(c->ws, 0, L.total, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.owner0, 0xFF, (size_t)c->N * 2, c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(c->ws + L.owner1, 0xFF, (size_t)c->N * 2, c->stream);
  if (e == hipSuccess && bounded(c)) {
    // the rest state f = w: the inlet slots hold its values less the inlet term
    const double zero[kMaxQ] = {};
    launch_bnd_uniform(c, c->state(), zero);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  return e == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

lbm_status lbm_create(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian,
                      void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_ctx **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  Layout L;
  const lbm_status st = check_create(p, max_solids, max_links, max_lagrangian, &L);
  if (st != LBM_OK) return st;
  if (!dev_workspace || ws_bytes < L.total) return LBM_ENOMEM;
  if (((uintptr_t)dev_workspace & 255) != 0) return LBM_EINVAL;
  lbm_ctx *c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_ENOMEM;
  if (init_ctx(c, p, L, dev_workspace, ws_bytes, hip_stream) != LBM_OK) {
    delete c;
    return LBM_EDEVICE;
  }
  *out = c;
  return LBM_OK;
}

lbm_status lbm_create_noalloc(const lbm_params *p, int32_t max_solids, int64_t max_links, int64_t max_lagrangian,
                              void *hip_stream, lbm_ctx **out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  Layout L;
  const lbm_status st = check_create(p, max_solids, max_links, max_lagrangian, &L);
  if (st != LBM_OK) return st;
  if (L.total > kNoAllocBytes) return LBM_ENOMEM;  // the lattice does not fit the static array
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocDevices) return LBM_EDEVICE;
  std::lock_guard<std::mutex> g(g_noalloc_mutex);
  if (g_noalloc_busy[dev]) return LBM_ESTATE;  // one context per device shares the array
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LBM_EDEVICE;
    g_scratch_ptr[dev] = static_cast<char *>(ptr);
  }
  lbm_ctx *c = new (g_noalloc_ctx[dev]) lbm_ctx();
  if (init_ctx(c, p, L, g_scratch_ptr[dev], kNoAllocBytes, hip_stream) != LBM_OK) {
    c->~lbm_ctx();
    return LBM_EDEVICE;
  }
  c->noalloc_dev = dev;
  g_noalloc_busy[dev] = true;
  *out = c;
  return LBM_OK;
}

size_t lbm_noalloc_capacity(void) { return kNoAllocBytes; }


lbm_status lbm_destroy(lbm_ctx *c) {
  if (!c) return LBM_EINVAL;
  if (c->batch) return set_err(c, "a batch member is released through its batch"), LBM_ESTATE;
  return lbm::destroy_ctx(c);
}

// A pair of profiling events: from the pool of read ones, else new.
static hipError_t take_prof_events(lbm_ctx *c, hipEvent_t *e0, hipEvent_t *e1) {
  if (!c->prof_pool.empty()) {
    *e0 = c->prof_pool.back().first;
    *e1 = c->prof_pool.back().second;
    c->prof_pool.pop_back();
    return hipSuccess;
  }
  hipError_t e = hipEventCreate(e0);
  if (e == hipSuccess) e = hipEventCreate(e1);
  return e;
}

lbm_status lbm_profile(lbm_ctx *c, int32_t every) {
  if (!c || every < 0) return LBM_EINVAL;
  c->prof_every = every;
  c->prof_count = 0;
  return LBM_OK;
}

lbm_status lbm_profile_read(lbm_ctx *c, double *sweep_ms, int64_t *launches) {
  if (!c) return LBM_EINVAL;
  HIPCALL(hipStreamSynchronize(c->stream));
  double tot = 0.0;
  int64_t n = 0;
  for (auto &e : c->prof_events) {
    float ms = 0.0f;
    HIPCALL(hipEventElapsedTime(&ms, e.e0, e.e1));
    tot += ms;
    n += e.launches;
    c->prof_pool.push_back({e.e0, e.e1});  // reused by later recordings
  }
  if (sweep_ms) *sweep_ms = tot;
  if (launches) *launches = n;
  c->prof_events.clear();
  return LBM_OK;
}

static lbm_status build_ibm(lbm_ctx *c);
static lbm_status ibm_polynomial(lbm_ctx *c, const std::vector<uint32_t> &rlen);
static lbm_status clear_solids(lbm_ctx *c, lbm_status st);

static bool coord_axis(const double a[3], int *ax, int *sg) {
  int k = -1, cnt = 0;
  for (int i = 0; i < 3; i++)
    if (a[i] != 0.0) {
      k = i;
      cnt++;
    }
  if (cnt != 1 || std::fabs(a[k]) != 1.0) return false;
  *ax = k;
  *sg = a[k] > 0 ? 1 : -1;
  return true;
}

static int dim_of(const lbm_ctx *c, int a) { return a == 0 ? c->p.nx : (a == 1 ? c->p.ny : c->p.nz); }

lbm_status lbm_set_solids(lbm_ctx *c, const lbm_solid *s, int32_t n, int32_t method, const lbm_ibm_opts *opts) {
  if (c) c->version++;
  if (!c) return LBM_EINVAL;
  if (n < 0 || n > c->L.max_solids || (n > 0 && !s)) return set_err(c, "solid count"), LBM_EINVAL;
  if (method < LBM_BB || method > LBM_IBB_ZHAO_YONG) return set_err(c, "method"), LBM_EINVAL;
  std::vector<DevSolid> ds((size_t)std::max(n, 1));
  bool moving = false;
  int32_t mbc = 0;
  uint64_t mask_total = 0;  // box cells of the solids so far (link-mask buffer offsets)
  bool any_free = false;
  for (int k = 0; k < n; k++) {
    const lbm_solid &q = s[k];
    DevSolid &d = ds[k];
    std::memset(&d, 0, sizeof(d));
    d.kind = q.kind;
    d.inverted = q.inverted ? 1 : 0;
    d.R = q.radius;
    for (int a = 0; a < 3; a++) {
      d.c0[a] = q.centre[a];
      d.U[a] = q.velocity[a];
      d.W[a] = q.omega[a];
      if (!std::isfinite(q.centre[a]) || !std::isfinite(q.velocity[a]) || !std::isfinite(q.omega[a]))
        return set_err(c, "non-finite solid data"), LBM_EINVAL;
    }
    if (c->D == 2) d.U[2] = 0.0;
    if (q.kind < LBM_SPHERE || q.kind > LBM_PLANE) return set_err(c, "solid kind"), LBM_EINVAL;
    int ax = 2, sg = 1;
    if (q.kind != LBM_SPHERE && !coord_axis(q.axis, &ax, &sg))
      return set_err(c, "axis must be a coordinate unit vector"), LBM_EINVAL;
    if (c->D == 2 && q.kind == LBM_CYLINDER && ax != 2) return set_err(c, "2D cylinders lie along z"), LBM_EINVAL;
    if (c->D == 2 && q.kind == LBM_PLANE && ax == 2) return set_err(c, "2D plane normal in the xy plane"), LBM_EINVAL;
    d.ax = ax;
    d.sgn = sg;
    d.moving = (d.U[0] != 0.0 || d.U[1] != 0.0 || d.U[2] != 0.0) ? 1 : 0;
    if (q.density != 0.0) {
      // free motion (Eq. 20)
      if (!(q.density > 0.0) || !std::isfinite(q.density) || !std::isfinite(q.gravity[0]) ||
          !std::isfinite(q.gravity[1]) || !std::isfinite(q.gravity[2]))
        return set_err(c, "free solid: density must be positive, gravity finite"), LBM_EINVAL;
      if (q.kind == LBM_PLANE || q.inverted || (q.kind == LBM_CYLINDER && c->D != 2) || c->batch)
        return set_err(c, "free solids need a sphere or 2D cylinder, not inverted, outside a batch"),
               LBM_EUNSUPPORTED;
      d.fm = method == LBM_IBM ? 1 : 0;  // Eq. 23 with the fluid inside the solid, else Eq. 20
      const double pi = 3.14159265358979323846, R = q.radius;
      d.free = 1;
      d.moving = 1;
      d.rho_p = q.density;
      for (int a = 0; a < 3; a++) d.grav[a] = (c->D == 2 && a == 2) ? 0.0 : q.gravity[a];
      d.Vp = q.kind == LBM_SPHERE ? 4.0 / 3.0 * pi * R * R * R : pi * R * R;
      d.Ip = (q.kind == LBM_SPHERE ? 0.4 : 0.5) * q.density * d.Vp * R * R;
      any_free = true;
    }
    for (int a = 0; a < 3; a++) {
      d.cp[a] = d.c0[a];
      d.Up[a] = d.U[a];
      d.Wp[a] = d.W[a];
    }
    if (bounded(c)) {
      // fixed spheres and cylinders along periodic axes, clear of the bounded faces
      if (d.moving || d.free || q.kind == LBM_PLANE || q.inverted ||
          (q.kind == LBM_CYLINDER && c->p.boundary[ax] != BND_PERIODIC))
        return set_err(c, "a bounded domain takes fixed spheres and cylinders along periodic axes"),
               LBM_EUNSUPPORTED;
      const int nn[3] = {c->p.nx, c->p.ny, c->p.nz};
      for (int a = 0; a < c->D; a++) {
        if (c->p.boundary[a] == BND_PERIODIC || (q.kind == LBM_CYLINDER && a == ax)) continue;
        if (!(q.centre[a] - q.radius - 4.0 >= 0.0 && q.centre[a] + q.radius + 4.0 <= nn[a] - 1.0))
          return set_err(c, "a solid must stay 4 nodes clear of the bounded faces"), LBM_EINVAL;
      }
    }
    if (d.moving && q.kind == LBM_PLANE)
      return set_err(c, "translating solids need a sphere or cylinder"), LBM_EUNSUPPORTED;
    if (d.moving && method == LBM_IBM) {
      const bool g = c->p.body_force[0] != 0.0 || c->p.body_force[1] != 0.0 || c->p.body_force[2] != 0.0;
      if (n != 1 || q.inverted || (q.kind == LBM_CYLINDER && c->D != 2) || c->batch ||
          (g && c->p.body_force_fluid_only))
        return set_err(c, "a moving IBM solid: the only solid, a sphere or 2D cylinder, not inverted, outside a "
                          "batch, with no fluid-only body force"),
               LBM_EUNSUPPORTED;
    }
    if (d.moving) {
      for (int a = 0; a < 3; a++)
        if (std::fabs(d.U[a]) >= 1.0) return set_err(c, "solid speed must be below one cell per step"), LBM_EINVAL;
    }
    moving |= d.moving != 0;
    if (q.kind != LBM_PLANE) {
      if (!(q.radius > 0.0)) return set_err(c, "radius must be positive"), LBM_EINVAL;
      for (int a = 0; a < c->D; a++) {
        if (q.kind == LBM_CYLINDER && a == ax) continue;
        if (!(q.centre[a] >= 0.0 && q.centre[a] < (double)dim_of(c, a)))
          return set_err(c, "centre must lie inside the box"), LBM_EINVAL;
        if (!(2.0 * q.radius < (double)dim_of(c, a))) return set_err(c, "solid wider than the box"), LBM_EINVAL;
      }
    }
    // bounding box: every cell within R + 2 of the centre (planes: 2 cells each side)
    uint64_t cells = 1;
    for (int a = 0; a < 3; a++) {
      const int La = dim_of(c, a);
      int ext;
      if (a >= c->D) ext = La;
      else if (q.kind == LBM_PLANE) ext = (a == ax) ? 6 : La;
      else if (q.kind == LBM_CYLINDER && a == ax) ext = La;
      else ext = (int)std::ceil(2.0 * q.radius) + 6;
      if (ext >= La) {
        d.full[a] = 1;
        d.ext[a] = La;
        d.box0[a] = 0;
      } else {
        d.full[a] = 0;
        d.ext[a] = ext;
        const double lo = q.kind == LBM_PLANE ? q.centre[a] : q.centre[a] - q.radius;
        d.box0[a] = (int)std::floor(lo) - 2;
      }
      cells *= (uint64_t)d.ext[a];
    }
    d.box_cells = (uint32_t)cells;
    d.mask_off = mask_total;
    mask_total += cells;
    d.fex = make_div((uint32_t)d.ext[0]);
    d.fexy = make_div((uint32_t)d.ext[0] * (uint32_t)d.ext[1]);
    mbc = std::max<int32_t>(mbc, (int32_t)((cells + kBlock - 1) / kBlock));
  }
  // ordinary spheres / cylinders must not overlap
  for (int a = 0; a < n; a++)
    for (int b = a + 1; b < n; b++) {
      if (s[a].kind == LBM_PLANE || s[b].kind == LBM_PLANE || s[a].inverted || s[b].inverted) continue;
      if (ds[a].moving || ds[b].moving) continue;
      double d2 = 0.0;
      for (int k = 0; k < c->D; k++) {
        if ((s[a].kind == LBM_CYLINDER && k == ds[a].ax) || (s[b].kind == LBM_CYLINDER && k == ds[b].ax)) continue;
        double d = s[a].centre[k] - s[b].centre[k];
        const double L = dim_of(c, k);
        d -= L * std::nearbyint(d / L);
        d2 += d * d;
      }
      if (std::sqrt(d2) < s[a].radius + s[b].radius) return set_err(c, "solids overlap"), LBM_EINVAL;
    }
  if (method == LBM_IBM)
    for (int k = 0; k < n; k++) {
      if (s[k].kind == LBM_PLANE) return set_err(c, "IBM needs spheres or cylinders"), LBM_EUNSUPPORTED;
      if (c->D == 3 && s[k].kind == LBM_CYLINDER && ds[k].ax != 2)
        return set_err(c, "IBM cylinders lie along z"), LBM_EUNSUPPORTED;
    }
  // the IBM options are checked before anything is written: a rejected call
  // leaves the context exactly as it was
  const int n_iter = opts ? opts->n_iter : 5;
  const int delta = (opts && opts->delta) ? opts->delta : 4;
  const double retraction = opts ? opts->retraction : 0.0;
  if (n_iter < 0 || !std::isfinite(retraction) || delta < 2 || delta > 4) return set_err(c, "IBM options"), LBM_EINVAL;
  if (moving && method == LBM_IBM && n_iter == 0)
    return set_err(c, "a moving IBM solid needs forcing iterations"), LBM_EINVAL;
  c->solids.assign(s, s + n);
  c->dsolids = ds;
  c->nsolid = n;
  c->method = method;
  c->any_moving = moving && method != LBM_IBM;
  c->any_free = any_free && method != LBM_IBM;
  c->ibm_moving = moving && method == LBM_IBM;
  c->ibm_free = any_free && method == LBM_IBM;
  c->solids_t = c->t;
  c->max_box_chunks = mbc;
  // the link masks of the count pass live in the staging region (4 N doubles) while links are built
  c->mask_cells = mask_total * 4 <= (uint64_t)4 * c->N * 8 ? mask_total : 0;
  c->n_iter = n_iter;
  c->delta = delta;
  c->retraction = retraction;
  c->nlinks = 0;
  c->k5_chunks = 0;
  c->link_lists = false;
  c->link_stride = 0;
  c->nlag = 0;
  c->nshell = 0;
  c->ibm_poly = false;
  c->lag_user = false;
  HIPCALL(hipMemcpyAsync(c->ws + c->L.solids, ds.data(), sizeof(DevSolid) * ds.size(), hipMemcpyHostToDevice,
                         c->stream));
  // the refill count and overflow flag (misc[3], misc[4]) and the free-solid flag (misc[6])
  HIPCALL(hipMemsetAsync(c->ws + c->L.misc + 3 * sizeof(uint32_t), 0, 4 * sizeof(uint32_t), c->stream));
  // no covering / uncovering momentum carried over from the previous solids
  HIPCALL(hipMemsetAsync(c->ws + c->L.cu, 0, (size_t)c->L.max_solids * 6 * 8, c->stream));
  // the whole-cell shifts of a moving IBM shell (both slots: no shift yet)
  HIPCALL(hipMemsetAsync(c->ws + c->L.misc + 64 + 16 * (size_t)c->L.max_solids, 0, 8 * sizeof(int32_t), c->stream));
  HIPCALL(hipMemsetAsync(c->ws + c->L.flags, 0, (size_t)c->N, c->stream));
  if (n == 0) {
    HIPCALL(hipStreamSynchronize(c->stream));
    return LBM_OK;
  }
  launch_classify(c, c->t, true);
  if (method != LBM_IBM) {
    launch_link_count(c, c->t);
    launch_link_scan(c);
    launch_link_emit(c, c->t);
    std::vector<SolidLinks> sl((size_t)n);
    uint32_t misc[2];
    HIPCALL(hipMemcpyAsync(sl.data(), c->ws + c->L.solid_links, sizeof(SolidLinks) * n, hipMemcpyDeviceToHost,
                           c->stream));
    HIPCALL(hipMemcpyAsync(misc, c->ws + c->L.misc, sizeof(misc), hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipStreamSynchronize(c->stream));
    if (misc[1]) {
      set_err(c, "more boundary links than max_links");
      return clear_solids(c, LBM_ENOMEM);
    }
    c->nlinks = misc[0];
    int32_t mx = 0;
    for (auto &q : sl) mx = std::max<int32_t>(mx, (int32_t)q.nchunks);
    // translating solids gain and lose links: leave headroom, checked after each lbm_step
    c->k5_chunks = moving ? 2 * mx + 2 : mx;
    HIPCALL(build_link_lists(c));
    return LBM_OK;
  }
  const lbm_status st = build_ibm(c);
  HIPCALL(hipStreamSynchronize(c->stream));
  return st == LBM_OK ? st : clear_solids(c, st);
}

// After a failure past the point where lbm_set_solids starts writing the
// context: no solid is left, so lbm_step is a plain periodic sweep (the node
// flags were cleared before the geometry was built and are cleared again).
static lbm_status clear_solids(lbm_ctx *c, lbm_status st) {
  c->solids.clear();
  c->nsolid = 0;
  c->nlinks = 0;
  c->k5_chunks = 0;
  c->link_lists = false;
  c->nlag = 0;
  c->nshell = 0;
  c->any_moving = c->any_free = c->ibm_moving = c->ibm_free = false;
  c->ibm_poly = false;
  c->lag_user = false;
  if (hipMemsetAsync(c->ws + c->L.flags, 0, (size_t)c->N, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return LBM_EDEVICE;
  return st;
}

// Lagrangian points of every solid (generated unless given by the caller),
// their stencils, the shell of stencil cells and its transpose.
static lbm_status build_ibm(lbm_ctx *c) {
  if (!c->lag_user) {
    c->lag_X.clear();
    c->lag_dV.clear();
    c->lag_start.assign(c->nsolid, 0);
    c->lag_count.assign(c->nsolid, 0);
    std::vector<double> X;
    for (int k = 0; k < c->nsolid; k++) {
      const lbm_solid &q = c->solids[k];
      const double R = q.inverted ? q.radius + c->retraction : q.radius - c->retraction;
      if (!(R > 0.0)) return set_err(c, "retraction larger than the radius"), LBM_EINVAL;
      X.clear();
      double dV = 0.0;
      if (c->D == 2) circle(q.centre, R, 0.0, X, dV);
      else if (q.kind == LBM_CYLINDER)
        for (int z = 0; z < c->p.nz; z++) circle(q.centre, R, (double)z, X, dV);
      else icosphere(q.centre, R, X, dV);
      c->lag_start[k] = (int64_t)(c->lag_X.size() / 3);
      c->lag_count[k] = (int64_t)(X.size() / 3);
      c->lag_X.insert(c->lag_X.end(), X.begin(), X.end());
      c->lag_dV.insert(c->lag_dV.end(), X.size() / 3, dV);
    }
  }
  const int64_t nl = (int64_t)(c->lag_X.size() / 3);
  if (nl > c->L.max_lag) return set_err(c, "more Lagrangian points than max_lagrangian"), LBM_ENOMEM;
  // a moving solid keeps a 5-node box per axis per point (125 slots in a
  // 128-entry row), twice the fixed stencil's room: half the point capacity
  const bool mv = c->ibm_moving;
  if (mv && 2 * nl > c->L.max_lag)
    return set_err(c, "a moving IBM solid holds at most max_lagrangian / 2 points"), LBM_ENOMEM;
  const int bw = mv ? 5 : 4, row = mv ? 128 : 64, sbits = mv ? 7 : 6;
  std::vector<int32_t> sid((size_t)std::max<int64_t>(nl, 1)), base((size_t)std::max<int64_t>(3 * nl, 3));
  for (int k = 0; k < c->nsolid; k++)
    for (int64_t l = c->lag_start[k]; l < c->lag_start[k] + c->lag_count[k]; l++) sid[l] = k;
  const int nzs = c->D == 2 ? 1 : bw;
  std::vector<uint32_t> cellof((size_t)std::max<int64_t>(nl * row, 1), 0);
  std::vector<uint32_t> all;
  all.reserve((size_t)nl * row);
  for (int64_t l = 0; l < nl; l++) {
    int b[3];
    for (int a = 0; a < 3; a++) b[a] = (a < c->D) ? (int)std::floor(c->lag_X[3 * l + a]) - 1 : 0;
    for (int a = 0; a < 3; a++) base[3 * l + a] = b[a];
    for (int kz = 0; kz < nzs; kz++)
      for (int ky = 0; ky < bw; ky++)
        for (int kx = 0; kx < bw; kx++) {
          auto w = [](int v, int L) { return ((v % L) + L) % L; };
          const uint32_t cell = (uint32_t)w(b[0] + kx, c->p.nx) +
                                (uint32_t)c->p.nx * ((uint32_t)w(b[1] + ky, c->p.ny) +
                                                     (uint32_t)c->p.ny * (uint32_t)w(b[2] + kz, c->p.nz));
          cellof[(size_t)l * row + (kz * bw + ky) * bw + kx] = cell;
          all.push_back(cell);
        }
  }
  std::sort(all.begin(), all.end());
  all.erase(std::unique(all.begin(), all.end()), all.end());
  const int64_t ns = (int64_t)all.size();
  if (ns > c->L.max_shell) return set_err(c, "IBM shell larger than its capacity"), LBM_ENOMEM;
  const int nslot = bw * bw * nzs;
  std::vector<uint32_t> idx((size_t)std::max<int64_t>(nl * row, 1), 0), rowcnt((size_t)ns + 1, 0);
  for (int64_t l = 0; l < nl; l++)
    for (int slot = 0; slot < nslot; slot++) {
      const uint32_t cell = cellof[(size_t)l * row + slot];
      const uint32_t si = (uint32_t)(std::lower_bound(all.begin(), all.end(), cell) - all.begin());
      idx[(size_t)l * row + slot] = si;
      rowcnt[si + 1]++;
    }
  std::vector<uint32_t> rowptr((size_t)ns + 1, 0);
  for (int64_t s = 0; s < ns; s++) rowptr[s + 1] = rowptr[s] + rowcnt[s + 1];
  std::vector<uint32_t> ent((size_t)std::max<uint32_t>(rowptr[ns], 1)), fill(rowptr.begin(), rowptr.end() - 1);
  for (int64_t l = 0; l < nl; l++)  // points in order, so each row is sorted by point
    for (int slot = 0; slot < nslot; slot++) {
      const uint32_t si = idx[(size_t)l * row + slot];
      ent[fill[si]++] = (uint32_t)(l << sbits) | (uint32_t)slot;
    }
  // fixed solids: the point coupling of the forcing iterations (Eq. 5 after
  // Eq. 8-9), A_lm = dV_m sum_x delta(x - X_l) delta(x - X_m): nonzero where
  // the stencils of l and m share a cell; each row lists those m in order,
  // padded to a fixed width (the values are formed on the device from the
  // delta weights); the stencil slots hold cells, not shell indices
  std::vector<uint32_t> rlen;
  std::vector<unsigned char> rows;
  int nw = 64;
  if (!mv) {
    rlen.assign((size_t)std::max<int64_t>(nl, 1), 0);
    std::vector<std::vector<uint32_t>> lists((size_t)nl);
    std::vector<int64_t> seen((size_t)std::max<int64_t>(nl, 1), -1);
    for (int64_t l = 0; l < nl; l++) {
      std::vector<uint32_t> &rowl = lists[(size_t)l];
      for (int slot = 0; slot < nslot; slot++) {
        const uint32_t si = idx[(size_t)l * row + slot];
        for (uint32_t e = rowptr[si]; e < rowptr[si + 1]; e++) {
          const uint32_t m = ent[e] >> sbits;
          if (seen[m] != l) {
            seen[m] = l;
            rowl.push_back(m);
          }
        }
      }
      std::sort(rowl.begin(), rowl.end());
      rlen[(size_t)l] = (uint32_t)rowl.size();
      if (rowl.size() > (size_t)kIbmNbr)
        return set_err(c, "a Lagrangian point couples to more than 128 others (points too close together)"),
               LBM_ENOMEM;
      if (rowl.size() > 64) nw = 128;
    }
    const size_t es = csize_of(c->p.storage) == 8 ? 16 : 8;
    rows.assign((size_t)std::max<int64_t>(nl, 1) * nw * es, 0);
    for (int64_t l = 0; l < nl; l++)
      for (int j = 0; j < nw; j++) {  // padding: column l, value 0
        const uint32_t m = j < (int)rlen[(size_t)l] ? lists[(size_t)l][(size_t)j] : (uint32_t)l;
        std::memcpy(rows.data() + ((size_t)l * nw + j) * es, &m, 4);
      }
    for (int64_t l = 0; l < nl; l++)
      for (int slot = 0; slot < nslot; slot++) idx[(size_t)l * row + slot] = cellof[(size_t)l * row + slot];
  }
  c->ibm_nw = nw;
  c->nlag = nl;
  c->nshell = ns;
  auto up = [&](size_t off, const void *src, size_t bytes) {
    return bytes ? hipMemcpyAsync(c->ws + off, src, bytes, hipMemcpyHostToDevice, c->stream) : hipSuccess;
  };
  HIPCALL(up(c->L.lag_X, c->lag_X.data(), sizeof(double) * 3 * nl));
  HIPCALL(up(c->L.lag_dV, c->lag_dV.data(), sizeof(double) * nl));
  HIPCALL(up(c->L.lag_sid, sid.data(), sizeof(int32_t) * nl));
  HIPCALL(up(c->L.lag_base, base.data(), sizeof(int32_t) * 3 * nl));
  HIPCALL(up(c->L.lag_idx, idx.data(), sizeof(uint32_t) * row * nl));
  HIPCALL(up(c->L.shell_cell, all.data(), sizeof(uint32_t) * ns));
  HIPCALL(up(c->L.shell_rowptr, rowptr.data(), sizeof(uint32_t) * (ns + 1)));
  HIPCALL(up(c->L.shell_ent, ent.data(), sizeof(uint32_t) * rowptr[ns]));
  if (!mv) {
    HIPCALL(up(c->L.lag_nptr, rlen.data(), sizeof(uint32_t) * nl));
    HIPCALL(up(c->L.lag_nrow, rows.data(), (size_t)nl * nw * (csize_of(c->p.storage) == 8 ? 16 : 8)));
  }
  HIPCALL(up(c->L.misc + 64, c->lag_start.data(), sizeof(int64_t) * c->nsolid));
  HIPCALL(up(c->L.misc + 64 + 8 * (size_t)c->L.max_solids, c->lag_count.data(), sizeof(int64_t) * c->nsolid));
  HIPCALL(hipMemsetAsync(c->ws + c->L.fibm, 0, (size_t)3 * c->L.stride * csize_of(c->p.storage), c->stream));
  launch_ibm_setup(c);
  // the host vectors must outlive the copies
  HIPCALL(hipStreamSynchronize(c->stream));
  c->ibm_poly = false;
  if (!mv && c->n_iter > 1) return ibm_polynomial(c, rlen);
  return LBM_OK;
}

// Fixed points: replace the rows of A (formed on the device
// from the delta weights) with those of P = sum_{k < n_iter} B^k, B = I - A,
// built in FP64 (row by row, each product B^k = B^(k-1) B through a dense
// accumulator), so that one product P F^0 gives the summed force of all
// iterations.  Kept as A (the iterations run one by one) when P's widest row
// does not fit the row capacity.
static lbm_status ibm_polynomial(lbm_ctx *c, const std::vector<uint32_t> &rlen) {
  const int64_t nl = c->nlag;
  const bool f64 = csize_of(c->p.storage) == 8;
  const size_t es = f64 ? 16 : 8;
  const int nw = c->ibm_nw;
  std::vector<unsigned char> raw((size_t)nl * nw * es);
  HIPCALL(hipMemcpyAsync(raw.data(), c->ws + c->L.lag_nrow, raw.size(), hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  // A in CSR (entry: column at byte 0, value at byte 8 (FP64) or 4 (FP32))
  std::vector<int64_t> ap((size_t)nl + 1, 0);
  for (int64_t l = 0; l < nl; l++) ap[(size_t)l + 1] = ap[(size_t)l] + rlen[(size_t)l];
  std::vector<uint32_t> acol((size_t)ap[(size_t)nl]);
  std::vector<double> aval((size_t)ap[(size_t)nl]);
  for (int64_t l = 0; l < nl; l++)
    for (uint32_t j = 0; j < rlen[(size_t)l]; j++) {
      const unsigned char *e = raw.data() + ((size_t)l * nw + j) * es;
      uint32_t col;
      std::memcpy(&col, e, 4);
      double v;
      if (f64) std::memcpy(&v, e + 8, 8);
      else {
        float f;
        std::memcpy(&f, e + 4, 4);
        v = (double)f;
      }
      acol[(size_t)(ap[(size_t)l] + j)] = col;
      aval[(size_t)(ap[(size_t)l] + j)] = v;
    }
  // row l of P: t = e_l; p = e_l; n_iter - 1 times t = t B, p += t
  std::vector<std::vector<std::pair<uint32_t, double>>> prow((size_t)nl);
  std::vector<double> t((size_t)nl, 0.0), tn((size_t)nl, 0.0), pacc((size_t)nl, 0.0);
  std::vector<char> in_t((size_t)nl, 0), in_tn((size_t)nl, 0), in_p((size_t)nl, 0);
  std::vector<uint32_t> lt, ltn, lp;
  size_t widest = 0;
  for (int64_t l = 0; l < nl; l++) {
    lt.assign(1, (uint32_t)l);
    lp.assign(1, (uint32_t)l);
    t[(size_t)l] = 1.0;
    in_t[(size_t)l] = 1;
    pacc[(size_t)l] = 1.0;
    in_p[(size_t)l] = 1;
    for (int k = 1; k < c->n_iter; k++) {
      ltn.clear();
      for (uint32_t m : lt) {
        const double tm = t[m];
        // (t B)_j = t_j - sum_m t_m A_mj
        if (!in_tn[m]) {
          in_tn[m] = 1;
          ltn.push_back(m);
        }
        tn[m] += tm;
        for (int64_t q = ap[m]; q < ap[(size_t)m + 1]; q++) {
          const uint32_t j = acol[(size_t)q];
          if (!in_tn[j]) {
            in_tn[j] = 1;
            ltn.push_back(j);
          }
          tn[j] -= tm * aval[(size_t)q];
        }
      }
      for (uint32_t m : lt) {
        t[m] = 0.0;
        in_t[m] = 0;
      }
      lt.swap(ltn);
      for (uint32_t j : lt) {
        t[j] = tn[j];
        tn[j] = 0.0;
        in_tn[j] = 0;
        in_t[j] = 1;
        if (!in_p[j]) {
          in_p[j] = 1;
          lp.push_back(j);
        }
        pacc[j] += t[j];
      }
    }
    std::sort(lp.begin(), lp.end());
    auto &row = prow[(size_t)l];
    row.reserve(lp.size());
    for (uint32_t j : lp) {
      row.emplace_back(j, pacc[j]);
      pacc[j] = 0.0;
      in_p[j] = 0;
    }
    for (uint32_t m : lt) {
      t[m] = 0.0;
      in_t[m] = 0;
    }
    widest = std::max(widest, row.size());
  }
  const int64_t pw = (int64_t)((widest + 63) / 64 * 64);
  if (nl * pw > c->L.max_lag * (int64_t)kIbmNbr) return LBM_OK;  // the iterations stay
  std::vector<unsigned char> out((size_t)nl * pw * es, 0);
  std::vector<uint32_t> plen((size_t)nl);
  for (int64_t l = 0; l < nl; l++) {
    const auto &row = prow[(size_t)l];
    plen[(size_t)l] = (uint32_t)row.size();
    for (size_t j = 0; j < row.size(); j++) {
      unsigned char *e = out.data() + ((size_t)l * pw + j) * es;
      std::memcpy(e, &row[j].first, 4);
      if (f64) std::memcpy(e + 8, &row[j].second, 8);
      else {
        const float f = (float)row[j].second;
        std::memcpy(e + 4, &f, 4);
      }
    }
  }
  HIPCALL(hipMemcpyAsync(c->ws + c->L.lag_nrow, out.data(), out.size(), hipMemcpyHostToDevice, c->stream));
  HIPCALL(hipMemcpyAsync(c->ws + c->L.lag_nptr, plen.data(), plen.size() * 4, hipMemcpyHostToDevice, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));  // the host vectors end here
  c->ibm_nw = (int)pw;
  c->ibm_poly = true;
  return LBM_OK;
}

lbm_status lbm_set_lagrangian(lbm_ctx *c, int32_t solid, const double *X, int64_t n, double dV) {
  if (c) c->version++;
  if (!c) return LBM_EINVAL;
  if (c->method != LBM_IBM || solid < 0 || solid >= c->nsolid || n < 0 || (n > 0 && !X) || !(dV >= 0.0))
    return set_err(c, "lbm_set_lagrangian needs an IBM solid"), LBM_EINVAL;
  if (c->ibm_moving && c->t != c->solids_t)
    return set_err(c, "the points of a moving IBM solid are set before it moves"), LBM_EINVAL;
  // rebuild the per-solid point lists with this solid replaced
  std::vector<double> NX, NdV;
  std::vector<int64_t> st(c->nsolid), ct(c->nsolid);
  for (int k = 0; k < c->nsolid; k++) {
    st[k] = (int64_t)(NX.size() / 3);
    if (k == solid) {
      for (int64_t l = 0; l < n; l++) {
        for (int a = 0; a < 3; a++) NX.push_back(a < c->D ? X[3 * l + a] : 0.0);
        NdV.push_back(dV);
      }
      ct[k] = n;
    } else {
      for (int64_t l = c->lag_start[k]; l < c->lag_start[k] + c->lag_count[k]; l++) {
        for (int a = 0; a < 3; a++) NX.push_back(c->lag_X[3 * l + a]);
        NdV.push_back(c->lag_dV[l]);
      }
      ct[k] = c->lag_count[k];
    }
  }
  for (double v : NX)
    if (!std::isfinite(v)) return set_err(c, "non-finite Lagrangian point"), LBM_EINVAL;
  if (bounded(c)) {
    // the delta kernel's support (two nodes either side) stays off the bounded faces
    const int nn[3] = {c->p.nx, c->p.ny, c->p.nz};
    for (int64_t l = 0; l < n; l++)
      for (int a = 0; a < c->D; a++)
        if (c->p.boundary[a] != BND_PERIODIC && !(X[3 * l + a] >= 3.0 && X[3 * l + a] <= nn[a] - 4.0))
          return set_err(c, "a Lagrangian point must stay 3 nodes clear of the bounded faces"), LBM_EINVAL;
  }
  c->lag_X = NX;
  c->lag_dV = NdV;
  c->lag_start = st;
  c->lag_count = ct;
  c->lag_user = true;
  HIPCALL(hipMemsetAsync(c->ws + c->L.flags, 0, (size_t)c->N, c->stream));
  launch_classify(c, c->t, true);
  return build_ibm(c);
}

// ----------------------------------------------------------------------------
// Sweep autotuner.  The sweep's only free choice is how its stores treat the
// caches: plain stores keep the freshly written tile in L2 / Infinity Cache
// (wins when the two population arrays nearly fit the 256 MB cache),
// non-temporal stores stream past them (wins beyond it).  The first 2R real
// sweeps of a context run R with each policy, timed by events attached to
// the dispatches; the faster policy is used from the end of that lbm_step
// call on and remembered per (lattice, collision, storage, flags, size) for
// later contexts of this process.  Both policies compute identical values.
// ----------------------------------------------------------------------------
static std::map<uint64_t, std::array<double, 5>> g_tune_cache;  // policy, time of each policy (us)
static std::mutex g_tune_mutex;
static constexpr int kTuneReps = 12;

static uint64_t tune_key(const lbm_ctx *c) {
  uint64_t k = (uint64_t)c->N;
  k = k * 31 + (uint64_t)c->Q;
  k = k * 31 + (uint64_t)c->p.collision * 7 + (c->default_rates ? 1 : 0);
  k = k * 31 + (uint64_t)c->p.storage;
  k = k * 31 + (c->nsolid > 0 ? 1 : 0);
  k = k * 31 + (uint64_t)(c->nsolid > 0 ? c->method : 0) * 2 + (c->link_lists ? 1 : 0);
  return k;
}

// Sweep policy tuning.  Stores are non-temporal (policy bit 0): tuning runs
// did not rank plain against non-temporal stores the way long runs do (plain
// stores won short runs at 128^3 FP32 and lost the long ones), so only the
// tile order is tuned.  The first kTuneSkip sweeps of a context use the
// default policy (the first ones after set-up run faster than the steady
// state).  Then the two candidates run kTuneReps consecutive sweeps each, in
// the order A B B A, so that a drift of the sweep time over the tuning
// cancels in each candidate's mean; one pair of events spans sweeps 2 ..
// kTuneReps of a run, so that the first sweep (whose time depends on how the
// sweep before it left its output) is not counted and the others run back to
// back, as they do in steady state.
static constexpr int kPolicies = 4;
static constexpr int kTuneSkip = 8;
static constexpr int kCands[2] = {1, 3};  // non-temporal stores, linear / XCD-contiguous tile order
static constexpr int kTuneRuns = 4;
static int tune_run_policy(int r) { return kCands[(r == 0 || r == 3) ? 0 : 1]; }

struct TuneStep {
  int policy;
  bool start, end;  // record the span's first / last event around this launch
};

static TuneStep tune_step(lbm_ctx *c) {
  const uint64_t key = tune_key(c);
  if (c->tuned_key != key) {
    for (auto &t : c->tune_events) {
      (void)hipEventDestroy(t.e0);
      (void)hipEventDestroy(t.e1);
    }
    c->tune_events.clear();
    c->sweep_policy = -1;
    c->tune_skipped = 0;
    c->tune_k = 0;
    c->tuned_key = key;
    std::lock_guard<std::mutex> g(g_tune_mutex);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      c->sweep_policy = (int)it->second[0];
      for (int p = 0; p < kPolicies; p++) c->tune_us[p] = it->second[1 + p];
    }
  }
  if (c->sweep_policy >= 0) return {c->sweep_policy, false, false};
  if (c->tune_skipped < kTuneSkip) {
    c->tune_skipped++;
    return {1, false, false};
  }
  const int j = c->tune_k;
  if (j >= kTuneRuns * kTuneReps) return {1, false, false};  // decided at the end of this call
  c->tune_k++;
  const int r = j % kTuneReps;
  return {tune_run_policy(j / kTuneReps), r == 1, r == kTuneReps - 1};
}

static lbm_status tune_finish(lbm_ctx *c) {
  if (c->sweep_policy >= 0 || c->tune_k < kTuneRuns * kTuneReps) return LBM_OK;
  HIPCALL(hipStreamSynchronize(c->stream));
  for (int p = 0; p < kPolicies; p++) c->tune_us[p] = 0.0;
  for (auto &t : c->tune_events) {  // two runs per candidate
    float ms = 0.0f;
    HIPCALL(hipEventElapsedTime(&ms, t.e0, t.e1));
    c->tune_us[t.policy] += 1e3 * (double)ms / (2 * (kTuneReps - 1));
    (void)hipEventDestroy(t.e0);
    (void)hipEventDestroy(t.e1);
  }
  c->tune_events.clear();
  // the linear order is kept unless the XCD-contiguous one is faster by 1 %
  const int best = c->tune_us[kCands[1]] < 0.99 * c->tune_us[kCands[0]] ? kCands[1] : kCands[0];
  c->sweep_policy = best;
  std::lock_guard<std::mutex> g(g_tune_mutex);
  g_tune_cache[c->tuned_key] = {(double)best, c->tune_us[0], c->tune_us[1], c->tune_us[2], c->tune_us[3]};
  return LBM_OK;
}

lbm_status lbm_step(lbm_ctx *c, int64_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  c->version++;

  const bool ibb = c->method != LBM_IBM && c->nsolid > 0;
  const bool inl = ibb && !c->any_moving && c->link_lists;
  // Zhao-Yong (x_f only) is evaluated by the sweep of its own step, every step of
  // the call; the other schemes by the sweep of the next step, steps 2..n
  const bool zy = inl && c->method == LBM_IBB_ZHAO_YONG;
  // convective outflow (Sec. 3.4) after each sweep
  const bool open_x = c->p.boundary[0] == BND_OPEN;
  if (inl && (nsteps > 1 || (zy && nsteps > 0))) launch_link_table(c);
  bool span = false;  // a profiling span over the sweeps of this call is open
  for (int64_t k = 0; k < nsteps; k++) {
    void *A = c->state(), *B = c->other();
    // IBM: forcing iterations now; the solid force of this step is summed in the sweep launch
    const bool ibm = c->method == LBM_IBM && c->nsolid > 0 && c->nlag > 0 && c->n_iter > 0;
    if (ibm) launch_ibm_step(c, A, c->t, false);
    else if (c->ibm_free) launch_ibm_ft_free(c, c->t);  // no points: no fluid force, the motion by Eq. 23 still
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const TuneStep ts = tune_step(c);
    const int policy = ts.policy;
    if (ts.start) {
      hipEvent_t t0, t1;
      HIPCALL(hipEventCreate(&t0));
      HIPCALL(hipEventCreate(&t1));
      HIPCALL(hipEventRecord(t0, c->stream));
      c->tune_events.push_back({policy, t0, t1});
    }
    // profiling (once tuned): the sweeps of steps 1 .. n-1 of a call with fixed
    // solids run back to back and are timed as one span; elsewhere every
    // prof_every-th sweep launch carries its own events
    const bool tuned = c->sweep_policy >= 0;
    if (inl && k == 1 && tuned && c->prof_every > 0) {
      hipEvent_t s0, s1;
      HIPCALL(take_prof_events(c, &s0, &s1));
      HIPCALL(hipEventRecord(s0, c->stream));
      c->prof_events.push_back({s0, s1, nsteps - 1});
      span = true;
    }
    if (!span && tuned && c->prof_every > 0 && c->prof_count++ % c->prof_every == 0) {
      HIPCALL(take_prof_events(c, &e0, &e1));
      c->prof_events.push_back({e0, e1, 1});
    }
    if (zy) {
      // the sweep evaluates this step's links after relaxing; its leading blocks
      // form the chunk partials of step t - 1 and the sums of step t - 2
      launch_sweep(c, A, B, policy, e0, e1, k >= 2 ? c->t - 2 : -1, -1, c->t, k >= 1 ? c->t - 1 : -1);
      if (open_x) launch_outflow(c, A, B);
      if (ts.end) HIPCALL(hipEventRecord(c->tune_events.back().e1, c->stream));
      if (span && k == nsteps - 1) HIPCALL(hipEventRecord(c->prof_events.back().e1, c->stream));
      c->cur ^= 1;
      c->t++;
      c->fresh = false;
      continue;
    }
    if (inl) {
      // fixed solids: from the second step of the call on, the sweep applies the
      // bounce-back of the previous step itself; the force terms of step t - 2
      // become chunk partials and those of step t - 3 are summed, in its
      // leading blocks (the last steps are finished after the loop)
      launch_sweep(c, A, B, policy, e0, e1, k >= 3 ? c->t - 3 : -1, -1, k >= 1 ? c->t - 1 : -1,
                   k >= 2 ? c->t - 2 : -1, k == nsteps - 1);
      if (open_x) launch_outflow(c, A, B);
      if (ts.end) HIPCALL(hipEventRecord(c->tune_events.back().e1, c->stream));
      if (span && k == nsteps - 1) HIPCALL(hipEventRecord(c->prof_events.back().e1, c->stream));
      c->cur ^= 1;
      c->t++;
      c->fresh = false;
      continue;
    }
    // the forces of the previous step of this call are reduced inside this sweep
    // launch (translating solids rebuild the link table first, so they reduce at once)
    const bool fused_reduce = ibb && k > 0 && !c->any_moving;
    launch_sweep(c, A, B, policy, e0, e1, fused_reduce ? c->t - 1 : -1, ibm && !c->ibm_free ? c->t : -1);
    if (open_x) launch_outflow(c, A, B);
    if (ts.end) HIPCALL(hipEventRecord(c->tune_events.back().e1, c->stream));
    if (ibb) {
      launch_ibb(c, B, A, c->t);
      if (c->any_free) launch_ft_reduce_free(c, c->t);  // force of step t, then the motion to t+1
      else if (k == nsteps - 1 || c->any_moving) launch_ft_reduce(c, c->t);
      if (c->any_moving) {
        launch_classify(c, c->t + 1, false);
        launch_refill_count(c, c->t + 1, B);
        if (c->nsolid != 1) launch_link_scan(c);
        launch_link_emit(c, c->t + 1);
      }
    }
    c->cur ^= 1;
    c->t++;
    c->fresh = false;
  }
  if (zy && nsteps > 0) {
    // the ghost slots are filled; the forces of the last two steps are summed
    const int64_t T = c->t - 1;
    if (nsteps >= 2) launch_ft_reduce(c, T - 1);
    launch_chunk_sum(c, T);
    launch_ft_reduce(c, T);
  } else if (inl && nsteps > 0) {
    // the last step's bounce-back fills the ghost slots of the state the call
    // leaves behind; every step of the call has its force summed on return
    const int64_t T = c->t - 1;
    if (nsteps >= 3) launch_ft_reduce(c, T - 2);
    if (nsteps >= 2) {
      launch_chunk_sum(c, T - 1);
      launch_ft_reduce(c, T - 1);
    }
    launch_ibb(c, c->state(), c->other(), T);
    launch_ft_reduce(c, T);
  }
  HIPCALL(hipGetLastError());
  {
    const lbm_status st = tune_finish(c);
    if (st != LBM_OK) return st;
  }
  if (c->ibm_free && nsteps > 0) {
    uint32_t flag = 0;
    HIPCALL(hipMemcpyAsync(&flag, c->ws + c->L.misc + 6 * sizeof(uint32_t), sizeof(flag), hipMemcpyDeviceToHost,
                           c->stream));
    HIPCALL(hipStreamSynchronize(c->stream));
    if (flag) return set_err(c, "a free solid reached half a cell per step"), LBM_EDIVERGED;
  }
  if (ibb && c->any_moving && nsteps > 0) {
    uint32_t misc[7];
    std::vector<SolidLinks> sl((size_t)c->nsolid);
    HIPCALL(hipMemcpyAsync(misc, c->ws + c->L.misc, sizeof(misc), hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipMemcpyAsync(sl.data(), c->ws + c->L.solid_links, sizeof(SolidLinks) * c->nsolid,
                           hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipStreamSynchronize(c->stream));
    c->nlinks = misc[0];
    if (misc[1]) return set_err(c, "more boundary links than max_links"), LBM_ENOMEM;
    if (misc[4]) return set_err(c, "more uncovered nodes in one step than the refill list holds"), LBM_ENOMEM;
    if (misc[6]) return set_err(c, "a free solid reached half a cell per step"), LBM_EDIVERGED;
    for (auto &q : sl)
      if ((int32_t)q.nchunks > c->k5_chunks)
        return set_err(c, "a translating solid outgrew its link headroom"), LBM_ENOMEM;
  }
  return LBM_OK;
}

lbm_status lbm_force_history(lbm_ctx *c, int64_t first, int64_t count, double *ft) {
  if (!c || count < 0 || (count > 0 && !ft)) return LBM_EINVAL;
  if (first < 0 || first + count > c->t || first < c->t - kHistCap)
    return set_err(c, "requested steps are not in the history"), LBM_EINVAL;
  const size_t per = (size_t)c->L.max_solids * 6;
  std::vector<double> buf(per);
  for (int64_t k = 0; k < count; k++) {
    const int64_t slot = (first + k) % kHistCap;
    HIPCALL(hipMemcpyAsync(buf.data(), c->ws + c->L.hist + (size_t)slot * per * 8, per * 8, hipMemcpyDeviceToHost,
                           c->stream));
    HIPCALL(hipStreamSynchronize(c->stream));
    std::memcpy(ft + (size_t)k * c->nsolid * 6, buf.data(), sizeof(double) * 6 * c->nsolid);
  }
  return LBM_OK;
}

lbm_status lbm_force_torque(lbm_ctx *c, double *force, double *torque) {
  if (!c) return LBM_EINVAL;
  if (c->t == 0) return set_err(c, "no step taken yet"), LBM_ESTATE;
  std::vector<double> ft((size_t)std::max(c->nsolid, 1) * 6);
  const lbm_status st = lbm_force_history(c, c->t - 1, 1, ft.data());
  if (st != LBM_OK) return st;
  for (int k = 0; k < c->nsolid; k++)
    for (int a = 0; a < 3; a++) {
      if (force) force[3 * k + a] = ft[6 * k + a];
      if (torque) torque[3 * k + a] = ft[6 * k + 3 + a];
    }
  return LBM_OK;
}

static lbm_status node_types_at(lbm_ctx *c, uint8_t *node_type, bool last_collision);

lbm_status lbm_macros(lbm_ctx *c, double *rho, double *u, uint8_t *node_type) {
  if (!c) return LBM_EINVAL;
  double *stg = c->at<double>(c->L.staging);
  // after a step the other array still holds the input of the last collision
  launch_macros(c, c->fresh ? c->state() : c->other(), stg, c->fresh ? 0 : 1);
  HIPCALL(hipGetLastError());
  const size_t N = (size_t)c->N;
  if (rho) HIPCALL(hipMemcpyAsync(rho, stg, N * 8, hipMemcpyDeviceToHost, c->stream));
  if (u) HIPCALL(hipMemcpyAsync(u, stg + N, 3 * N * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  if (node_type) return node_types_at(c, node_type, !c->fresh && c->any_moving);
  return LBM_OK;
}

lbm_status lbm_solid_state(lbm_ctx *c, double *state) {
  if (!c || (!state && c->nsolid > 0)) return LBM_EINVAL;
  if (c->nsolid <= 0) return LBM_OK;
  std::vector<DevSolid> ds((size_t)c->nsolid);
  HIPCALL(hipMemcpyAsync(ds.data(), c->ws + c->L.solids, sizeof(DevSolid) * ds.size(), hipMemcpyDeviceToHost,
                         c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  for (int k = 0; k < c->nsolid; k++) {
    const DevSolid &d = ds[(size_t)k];
    for (int a = 0; a < 3; a++) {
      // the device's centre_at, on the host
      double y = d.c0[a];
      if (d.moving && a < c->D) {
        const double L = (double)dim_of(c, a);
        y = d.c0[a] + (double)(c->t - d.tref) * d.U[a];
        if (!(y >= 0.0 && y < L)) {
          y = std::fmod(y, L);
          if (y < 0.0) y = y + L;
        }
      }
      state[9 * k + a] = y;
      state[9 * k + 3 + a] = d.U[a];
      state[9 * k + 6 + a] = d.W[a];
    }
  }
  return LBM_OK;
}

lbm_status lbm_strain(lbm_ctx *c, double *S, double *eps) {
  if (!c || (!S && !eps)) return LBM_EINVAL;
  if (c->fresh) return set_err(c, "lbm_strain needs a step since the populations were set"), LBM_ESTATE;
  double *stg = c->at<double>(c->L.staging);
  const size_t N = (size_t)c->N;
  // the other array still holds the input of the last collision; two passes of
  // 4 and 3 fields fit the staging region (4 N doubles)
  launch_strain(c, c->other(), stg, 0);
  HIPCALL(hipGetLastError());
  if (S) HIPCALL(hipMemcpyAsync(S, stg, 3 * N * 8, hipMemcpyDeviceToHost, c->stream));
  if (eps) HIPCALL(hipMemcpyAsync(eps, stg + 3 * N, N * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  if (S) {
    launch_strain(c, c->other(), stg, 1);
    HIPCALL(hipGetLastError());
    HIPCALL(hipMemcpyAsync(S + 3 * N, stg, 3 * N * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}

// Node types of the current geometry, or of the geometry of the last
// collision (translating solids move after the collision of each step).
static lbm_status node_types_at(lbm_ctx *c, uint8_t *node_type, bool last_collision) {
  const size_t N = (size_t)c->N;
  std::vector<uint8_t> fl(N);
  std::vector<uint16_t> own(N);
  HIPCALL(hipMemcpyAsync(fl.data(), c->ws + c->L.flags, N, hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipMemcpyAsync(own.data(), c->ws + (last_collision ? c->L.owner1 : c->L.owner0), N * 2,
                         hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  const uint8_t bit = last_collision ? F_WAS_SOLID : F_SOLID;
  for (size_t n = 0; n < N; n++) node_type[n] = (fl[n] & bit) ? 1 : (own[n] != 0xFFFF ? 2 : 0);
  return LBM_OK;
}

lbm_status lbm_node_types(lbm_ctx *c, uint8_t *node_type) {
  if (!c || !node_type) return LBM_EINVAL;
  return node_types_at(c, node_type, false);
}

lbm_status lbm_get_f(lbm_ctx *c, double *f) {
  if (!c || !f) return LBM_EINVAL;
  double *stg = c->at<double>(c->L.staging);
  for (int i = 0; i < c->Q; i++) {
    launch_decode_gather(c, i, c->state(), stg, false);
    HIPCALL(hipMemcpyAsync(f + (size_t)i * c->N, stg, (size_t)c->N * 8, hipMemcpyDeviceToHost, c->stream));
  }
  HIPCALL(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_f(lbm_ctx *c, const double *f) {
  if (!c || !f) return LBM_EINVAL;
  double *stg = c->at<double>(c->L.staging);
  for (int i = 0; i < c->Q; i++) {
    HIPCALL(hipMemcpyAsync(stg, f + (size_t)i * c->N, (size_t)c->N * 8, hipMemcpyHostToDevice, c->stream));
    launch_encode_shift(c, i, stg, c->state(), false);
  }
  HIPCALL(hipStreamSynchronize(c->stream));
  c->fresh = true;
  c->version++;
  return LBM_OK;
}

// Direction i of the velocity set (ABI order) and its weight.
static void lattice_dir(int Q, int i, int e[3], double *w) {
  if (Q == 9) {
    e[0] = Lat<9>::ex(i), e[1] = Lat<9>::ey(i), e[2] = 0;
    *w = wgt<9>(i);
  } else {
    e[0] = Lat<19>::ex(i), e[1] = Lat<19>::ey(i), e[2] = Lat<19>::ez(i);
    *w = wgt<19>(i);
  }
}

lbm_status lbm_set_equilibrium(lbm_ctx *c, double rho, const double *u) {
  if (!c || !u || !(rho > 0.0) || !std::isfinite(rho)) return LBM_EINVAL;
  double uu = 0.0;
  for (int a = 0; a < c->D; a++) {
    if (!std::isfinite(u[a])) return LBM_EINVAL;
    uu += u[a] * u[a];
  }
  // f_eq_i - w_i = w_i [(rho - 1) + rho (3 e.u + 4.5 (e.u)^2 - 1.5 u.u)], rest state rho = 1, u = 0
  double h[kMaxQ];
  for (int i = 0; i < c->Q; i++) {
    int e[3];
    double w;
    lattice_dir(c->Q, i, e, &w);
    double eu = 0.0;
    for (int a = 0; a < c->D; a++) eu += e[a] * u[a];
    h[i] = w * ((rho - 1.0) + rho * (3.0 * eu + 4.5 * eu * eu - 1.5 * uu));
  }
  launch_fill_uniform(c, c->state(), h);
  if (bounded(c)) launch_bnd_uniform(c, c->state(), h);
  HIPCALL(hipGetLastError());
  HIPCALL(hipStreamSynchronize(c->stream));
  c->fresh = true;
  c->version++;
  return LBM_OK;
}

lbm_status lbm_get_state(lbm_ctx *c, void *host) {
  if (!c || !host) return LBM_EINVAL;
  double *stg = c->at<double>(c->L.staging);
  const size_t bytes = (size_t)c->N * c->store_bytes;
  for (int i = 0; i < c->Q; i++) {
    launch_decode_gather(c, i, c->state(), stg, true);
    HIPCALL(hipMemcpyAsync(static_cast<char *>(host) + (size_t)i * bytes, stg, bytes, hipMemcpyDeviceToHost,
                           c->stream));
  }
  HIPCALL(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

lbm_status lbm_set_state(lbm_ctx *c, const void *host) {
  if (!c || !host) return LBM_EINVAL;
  double *stg = c->at<double>(c->L.staging);
  const size_t bytes = (size_t)c->N * c->store_bytes;
  for (int i = 0; i < c->Q; i++) {
    HIPCALL(hipMemcpyAsync(stg, static_cast<const char *>(host) + (size_t)i * bytes, bytes, hipMemcpyHostToDevice,
                           c->stream));
    launch_encode_shift(c, i, stg, c->state(), true);
  }
  HIPCALL(hipStreamSynchronize(c->stream));
  c->fresh = true;
  c->version++;
  return LBM_OK;
}

lbm_status lbm_link_list(lbm_ctx *c, int64_t *count, uint32_t *cell, uint8_t *dir, int32_t *solid, double *q) {
  if (!c || !count) return LBM_EINVAL;
  const int64_t nl = c->nlinks;
  if (!cell && !dir && !solid && !q) {
    *count = nl;
    return LBM_OK;
  }
  if (*count < nl) {
    *count = nl;
    return set_err(c, "output arrays too short"), LBM_EINVAL;
  }
  std::vector<uint32_t> lc((size_t)std::max<int64_t>(nl, 1)), lm((size_t)std::max<int64_t>(nl, 1));
  std::vector<double> lq((size_t)std::max<int64_t>(nl, 1));
  std::vector<SolidLinks> sl((size_t)std::max(c->nsolid, 1));
  if (nl > 0) {
    HIPCALL(hipMemcpyAsync(lc.data(), c->ws + c->L.link_cell, nl * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipMemcpyAsync(lm.data(), c->ws + c->L.link_meta, nl * 4, hipMemcpyDeviceToHost, c->stream));
    HIPCALL(hipMemcpyAsync(lq.data(), c->ws + c->L.link_q, nl * 8, hipMemcpyDeviceToHost, c->stream));
  }
  if (c->nsolid > 0)
    HIPCALL(hipMemcpyAsync(sl.data(), c->ws + c->L.solid_links, sizeof(SolidLinks) * c->nsolid,
                           hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  std::vector<int32_t> ls((size_t)std::max<int64_t>(nl, 1));
  for (int k = 0; k < c->nsolid; k++)
    for (uint32_t l = sl[k].start; l < sl[k].start + sl[k].count && l < (uint32_t)nl; l++) ls[l] = k;
  std::vector<int64_t> ord((size_t)nl);
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    if (lc[a] != lc[b]) return lc[a] < lc[b];
    return (lm[a] & 31u) < (lm[b] & 31u);
  });
  for (int64_t k = 0; k < nl; k++) {
    const int64_t l = ord[k];
    if (cell) cell[k] = lc[l];
    if (dir) dir[k] = (uint8_t)(lm[l] & 31u);
    if (solid) solid[k] = ls[l];
    if (q) q[k] = lq[l];
  }
  *count = nl;
  return LBM_OK;
}

lbm_status lbm_check(lbm_ctx *c) {
  if (!c) return LBM_EINVAL;
  uint32_t *flag = c->at<uint32_t>(c->L.misc + 8);
  launch_check_finite(c, c->state(), flag);
  uint32_t h = 0;
  HIPCALL(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, c->stream));
  HIPCALL(hipStreamSynchronize(c->stream));
  if (h) return set_err(c, "non-finite value in the populations"), LBM_EDIVERGED;
  return LBM_OK;
}

lbm_status lbm_autotune_info(lbm_ctx *c, int32_t *nontemporal, double *us_plain, double *us_nontemporal) {
  if (!c) return LBM_EINVAL;
  const int p = c->sweep_policy;
  if (nontemporal) *nontemporal = p < 0 ? -1 : (p & 1);
  const int order = p < 0 ? 0 : (p & 2);
  if (us_plain) *us_plain = c->tune_us[order];
  if (us_nontemporal) *us_nontemporal = c->tune_us[order | 1];
  return LBM_OK;
}

lbm_status lbm_autotune_policy(lbm_ctx *c, int32_t *policy, double *us) {
  if (!c) return LBM_EINVAL;
  if (policy) *policy = c->sweep_policy;
  if (us)
    for (int p = 0; p < 4; p++) us[p] = c->tune_us[p];
  return LBM_OK;
}

lbm_status lbm_copy_probe(const void *src, void *dst, size_t bytes, void *hip_stream) {
  if (!src || !dst || (bytes & 15) || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return LBM_EINVAL;
  launch_copy_probe(src, dst, bytes, static_cast<hipStream_t>(hip_stream));
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EDEVICE;
}

}  // extern "C"
