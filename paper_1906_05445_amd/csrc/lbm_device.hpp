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
