// lbm_device.hpp -- device-side lattice description and helpers (gfx950).
//
// Velocity sets D2Q9 / D3Q19 with c_s^2 = 1/3 in the ABI order (rest, then
// +/- pairs, axis pairs first).  The MRT transform M of Eq. 3 is not printed
// in the paper; here its rows are the integer polynomials of e_i obtained by
// orthogonalising the monomials 1, |e|^2, |e|^4, e_x, e_x|e|^2, ... in that
// order (row scaling is free: M^-1 S M does not depend on it).  Everything is
// constexpr so that the compiler folds the zero and unit entries away.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// ----------------------------------------------------------------------------
// velocity sets
// ----------------------------------------------------------------------------
template <int Q>
struct Lat;

template <>
struct Lat<9> {
  static constexpr int D = 2;
  __host__ __device__ static constexpr int ex(int i) {
    constexpr int v[9] = {0, 1, -1, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int ey(int i) {
    constexpr int v[9] = {0, 0, 0, 1, -1, 1, -1, -1, 1};
    return v[i];
  }
  __host__ __device__ static constexpr int ez(int) { return 0; }
};

template <>
struct Lat<19> {
  static constexpr int D = 3;
  __host__ __device__ static constexpr int ex(int i) {
    constexpr int v[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    return v[i];
  }
  __host__ __device__ static constexpr int ey(int i) {
    constexpr int v[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    return v[i];
  }
  __host__ __device__ static constexpr int ez(int i) {
    constexpr int v[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    return v[i];
  }
};

template <int Q>
__host__ __device__ constexpr int esq(int i) {
  return Lat<Q>::ex(i) * Lat<Q>::ex(i) + Lat<Q>::ey(i) * Lat<Q>::ey(i) + Lat<Q>::ez(i) * Lat<Q>::ez(i);
}
// opposite direction: pairs are (1,2), (3,4), ...
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

// Weights: rest 4/9 (D2Q9) or 1/3 (D3Q19); |e| = 1: 1/9 or 1/18; |e| = sqrt 2: 1/36.
template <int Q>
__host__ __device__ constexpr double wgt(int i) {
  return Q == 9 ? (esq<Q>(i) == 0 ? 4.0 / 9.0 : (esq<Q>(i) == 1 ? 1.0 / 9.0 : 1.0 / 36.0))
                : (esq<Q>(i) == 0 ? 1.0 / 3.0 : (esq<Q>(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0));
}

// ----------------------------------------------------------------------------
// MRT rows (integer polynomials of e), in the ABI moment order.
// ----------------------------------------------------------------------------
template <int Q>
__host__ __device__ constexpr int mrow(int k, int i) {
  const int x = Lat<Q>::ex(i), y = Lat<Q>::ey(i), z = Lat<Q>::ez(i);
  const int s = x * x + y * y + z * z;
  if (Q == 9) {
    switch (k) {
      case 0: return 1;
      case 1: return 3 * s - 4;
      case 2: return (9 * s * s - 21 * s + 8) / 2;
      case 3: return x;
      case 4: return (3 * s - 5) * x;
      case 5: return y;
      case 6: return (3 * s - 5) * y;
      case 7: return x * x - y * y;
      default: return x * y;
    }
  }
  switch (k) {
    case 0: return 1;
    case 1: return 19 * s - 30;
    case 2: return (21 * s * s - 53 * s + 24) / 2;
    case 3: return x;
    case 4: return (5 * s - 9) * x;
    case 5: return y;
    case 6: return (5 * s - 9) * y;
    case 7: return z;
    case 8: return (5 * s - 9) * z;
    case 9: return 3 * x * x - s;
    case 10: return (3 * s - 5) * (3 * x * x - s);
    case 11: return y * y - z * z;
    case 12: return (3 * s - 5) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}
template <int Q>
__host__ __device__ constexpr int mnorm(int k) {
  int s = 0;
  for (int i = 0; i < Q; i++) s += mrow<Q>(k, i) * mrow<Q>(k, i);
  return s;
}
// conserved moments: density and momentum rows
template <int Q>
__host__ __device__ constexpr bool conserved(int k) {
  return Q == 9 ? (k == 0 || k == 3 || k == 5) : (k == 0 || k == 3 || k == 5 || k == 7);
}
// odd rows: antisymmetric under e -> -e
template <int Q>
__host__ __device__ constexpr bool odd_row(int k) {
  for (int i = 1; i < Q; i++)
    if (mrow<Q>(k, i) != -mrow<Q>(k, opp(i))) return false;
  return true;
}

// ----------------------------------------------------------------------------
// population layout: tiles of kTile consecutive cells; inside a tile the Q
// directions are stored one after the other (kTile values each).  A sweep
// then streams two contiguous Q*kTile blocks per tile instead of 2Q arrays
// that are far apart, which keeps the HBM access pattern dense.
// ----------------------------------------------------------------------------
constexpr uint32_t kTile = 256;

// Tiles swept per block (one cell of each per thread): two for half-precision
// storage, whose loads carry half the bytes, one otherwise.
template <typename S>
__host__ __device__ constexpr int sweep_cpt_of() {
  return sizeof(S) == 2 ? 2 : 1;
}
__host__ __device__ constexpr uint32_t sweep_cpt_storage(int storage_bytes) { return storage_bytes == 2 ? 2u : 1u; }
template <int Q>
__host__ __device__ inline uint64_t pidx(int i, uint32_t n) {
  return (uint64_t)(n / kTile) * (Q * kTile) + (uint64_t)i * kTile + (n % kTile);
}
// The same offset in 32 bits, for arrays of fewer than 2^32 values: one
// 24-bit multiply-add instead of a 64-bit one.
template <int Q>
__device__ inline uint32_t pidx32(int i, uint32_t n) {
  return __umul24(n >> 8, (uint32_t)(Q * kTile)) + (uint32_t)i * kTile + (n & (kTile - 1));
}
__host__ __device__ inline uint64_t pidx_rt(int Q, int i, uint32_t n) {
  return (uint64_t)(n / kTile) * ((uint64_t)Q * kTile) + (uint64_t)i * kTile + (n % kTile);
}

// ----------------------------------------------------------------------------
// domain boundaries (Sec. 3.4)
// ----------------------------------------------------------------------------
// Per axis: periodic; stress-free planes halfway outside the first and last
// node layers (specular reflection: the normal component of a population
// that would cross one is reversed and it stays in its layer); or, on x only,
// a velocity inlet halfway before x = 0 (bounce-back with the inflow velocity
// as wall velocity, the form of Eq. 10) and a convective outflow at the last
// layer.
enum : int32_t { BND_PERIODIC = 0, BND_SLIP = 1, BND_OPEN = 2 };

// Direction i with its components on the axes of mask m (bit a: axis a) reversed.
template <int Q>
__host__ __device__ constexpr int dir_flip(int i, int m) {
  const int ex = (m & 1) ? -Lat<Q>::ex(i) : Lat<Q>::ex(i);
  const int ey = (m & 2) ? -Lat<Q>::ey(i) : Lat<Q>::ey(i);
  const int ez = (m & 4) ? -Lat<Q>::ez(i) : Lat<Q>::ez(i);
  for (int k = 0; k < Q; k++)
    if (Lat<Q>::ex(k) == ex && Lat<Q>::ey(k) == ey && Lat<Q>::ez(k) == ez) return k;
  return i;
}

// Where the population of direction e = (ex, ey, ez) that arrives at node
// (x, y, z) is kept in the pull form (the stored array holds each node's
// post-collision values in its own slots).  Inside the domain, and across a
// periodic axis: node x - e, same direction.  Across a stress-free plane:
// the node's own layer on that axis, the direction mirrored on it (flip).
// Before the inlet or past the outlet (open): the node's own slot of the
// reverse direction -- at the inlet the reflected post-collision value, to
// which the inlet term 6 w_i e_ix U_in is added; at the outlet the value the
// convective outflow condition set there after the previous sweep (the
// reverse direction leaves the domain, so no node pulls that slot).
struct BndSrc {
  uint32_t cell;
  int flip;
  bool open, inlet;
};
__device__ __forceinline__ BndSrc bnd_src(int ex, int ey, int ez, int x, int y, int z, int nx, int ny, int nz,
                                          const int32_t *bc) {
  const bool ox = ex != 0 && bc[0] != BND_PERIODIC && (ex > 0 ? x == 0 : x == nx - 1);
  const bool oy = ey != 0 && bc[1] != BND_PERIODIC && (ey > 0 ? y == 0 : y == ny - 1);
  const bool oz = ez != 0 && bc[2] != BND_PERIODIC && (ez > 0 ? z == 0 : z == nz - 1);
  BndSrc s;
  s.open = ox && bc[0] == BND_OPEN;
  s.inlet = s.open && ex > 0;
  if (s.open) {
    s.cell = (uint32_t)x + (uint32_t)nx * ((uint32_t)y + (uint32_t)ny * (uint32_t)z);
    s.flip = 0;
    return s;
  }
  int sx = ox ? x : x - ex, sy = oy ? y : y - ey, sz = oz ? z : z - ez;
  sx = sx < 0 ? sx + nx : (sx >= nx ? sx - nx : sx);
  sy = sy < 0 ? sy + ny : (sy >= ny ? sy - ny : sy);
  sz = sz < 0 ? sz + nz : (sz >= nz ? sz - nz : sz);
  s.cell = (uint32_t)sx + (uint32_t)nx * ((uint32_t)sy + (uint32_t)ny * (uint32_t)sz);
  s.flip = (ox ? 1 : 0) | (oy ? 2 : 0) | (oz ? 4 : 0);
  return s;
}
// Slot direction of bnd_src for direction i of a compile-time lattice (i a
// constant after unrolling: every candidate folds to a constant).
template <int Q>
__device__ __forceinline__ int bnd_dir(int i, const BndSrc &s) {
  if (s.open) return opp(i);
  const int f = s.flip;
  return f == 0 ? i
       : f == 1 ? dir_flip<Q>(i, 1)
       : f == 2 ? dir_flip<Q>(i, 2)
       : f == 3 ? dir_flip<Q>(i, 3)
       : f == 4 ? dir_flip<Q>(i, 4)
       : f == 5 ? dir_flip<Q>(i, 5)
       : f == 6 ? dir_flip<Q>(i, 6)
                : dir_flip<Q>(i, 7);
}

// ----------------------------------------------------------------------------
// node flags
// ----------------------------------------------------------------------------
enum : uint8_t {
  F_SOLID = 1,     // IBB solid node: no collision, no streaming out
  F_NOBODY = 2,    // no body force (inside a solid's volume, fluid-only forcing)
  F_IBM = 4,       // cell of an IBM stencil: read the spread boundary force
  F_WAS_SOLID = 8, // solid in the geometry of the previous step (moving solids)
  F_LINK = 16,     // fluid node with boundary links (fixed solids)
};

// ----------------------------------------------------------------------------
// storage formats: the stored value is the deviation f - w
// ----------------------------------------------------------------------------
template <typename S>
struct Store;
template <>
struct Store<double> {
  using C = double;
  __device__ static inline C ld(const double *p) { return *p; }
  __device__ static inline void st(double *p, C v) { *p = v; }
  __device__ static inline void st_nt(double *p, C v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<float> {
  using C = float;
  __device__ static inline C ld(const float *p) { return *p; }
  __device__ static inline void st(float *p, C v) { *p = v; }
  __device__ static inline void st_nt(float *p, C v) { __builtin_nontemporal_store(v, p); }
};
template <>
struct Store<_Float16> {
  using C = float;
  __device__ static inline C ld(const _Float16 *p) { return (float)*p; }
  __device__ static inline void st(_Float16 *p, C v) { *p = (_Float16)v; }
  __device__ static inline void st_nt(_Float16 *p, C v) { __builtin_nontemporal_store((_Float16)v, p); }
};

// ----------------------------------------------------------------------------
// FP16 storage with stochastic rounding (LBM_F16_SR)
// ----------------------------------------------------------------------------
// Round-to-nearest loses every change smaller than half a unit in the last
// place of the stored value: in a slowly developing flow the per-step
// increments of the populations fall below it and the flow lags.  Stochastic
// rounding rounds up with probability equal to the dropped fraction, so the
// stored value is unbiased.  The dither is a deterministic hash of the slot
// and the time step, so runs repeat bit for bit.
//
// Integer hash: two multiply-xorshift rounds (Wellons's "lowbias32").
__host__ __device__ inline uint32_t hash32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}
// Per-step seed of the dither.
__host__ __device__ inline uint32_t sr_seed(int64_t t) { return hash32((uint32_t)t * 0x9e3779b9U + 0x632be5abU); }
// 13 dither bits of direction i from a cell's hash h: the top bits of the low
// word of (h >> 8) times an odd 24-bit constant of that direction in
// [2^23, 2^24).  The product spans about 2^47, so its low word wraps some 2^15
// times and its top 13 bits are uniform to about 2^-15 when h is.  Both
// factors are below 2^24, so the compiler takes the full-rate 24-bit multiply
// (v_mul_u32_u24), where a 32-bit one takes four times as long.
__device__ inline uint32_t sr_bits(uint32_t h, int i) {
  const uint32_t k = ((0x9e3779U * (2U * (uint32_t)i + 1U)) & 0x7fffffU) | 0x800001U;
  return ((h >> 8) * k) >> 19;
}
// v rounded to FP16 stochastically with dither r (13 bits, the bits FP16
// drops from an FP32 mantissa), in FP16's normal range; nearest elsewhere.
__device__ inline _Float16 f16_round_sr(float v, uint32_t r) {
  const uint32_t b = __float_as_uint(v), mag = b & 0x7fffffffU;
  if (mag < 0x38800000U || mag >= 0x477fe000U) return (_Float16)v;
  return (_Float16)__uint_as_float((b + r) & 0xffffe000U);  // exact in FP16
}
// Storage value of a computed population: stochastic for FP16 when sr is
// set (dither r), the plain conversion otherwise.
template <typename S, typename C>
__device__ inline S store_value(C v, bool sr, uint32_t r) {
  if constexpr (sizeof(S) == 2) {
    if (sr) return f16_round_sr((float)v, r);
  }
  (void)sr;
  (void)r;
  return (S)v;
}

// ----------------------------------------------------------------------------
// integer helpers
// ----------------------------------------------------------------------------
// Division by a runtime constant d for n < 2^31: q = (umulhi(n, m) + n) >> s.
struct FastDiv {
  uint32_t d, m, s;
};
__device__ inline uint32_t fdiv(uint32_t n, FastDiv f) { return (__umulhi(n, f.m) + n) >> f.s; }

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical blocks so neighbouring tiles share its L2.
__device__ inline uint32_t xcd_remap(uint32_t b, uint32_t G) {
  const uint32_t G8 = G >> 3;
  if (b >= (G8 << 3)) return b;
  return (b & 7u) * G8 + (b >> 3);
}

// Periodic wrap of a coordinate into [0, n).  Neighbour and box offsets stay
// within one period, where one compare-and-add suffices; the remainder is
// taken only outside [-n, 2n).
__device__ inline int wrapi(int a, int n) {
  if (a < 0) a += n;
  else if (a >= n) a -= n;
  if ((unsigned)a >= (unsigned)n) {
    a %= n;
    if (a < 0) a += n;
  }
  return a;
}

// Block-wide sum of a double (blockDim.x a multiple of 64, <= 1024); fixed order.
__device__ inline double block_sum(double v, double *lds) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < (int)(blockDim.x >> 6); k++) r += lds[k];
  return r;  // valid in thread 0
}

}  // namespace lbm
