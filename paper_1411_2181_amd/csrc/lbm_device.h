// Device-side definitions shared by the lbmve kernels: the D3Q19 tables as
// compile-time constants, the per-run parameter record, the tile record and
// the storage conversions of the three precisions.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include <type_traits>

namespace lbm {

// ---- D3Q19 (direction order documented in include/lbmve.h) -------------
constexpr int Q = 19;
constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPPI[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
// weight classes: 0 rest (1/3), 1 axis (1/18), 2 diagonal (1/36)
constexpr int WCLASS[Q] = {0, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2, 2};

template <typename T>
__host__ __device__ constexpr T wgt(int i) {
  return WCLASS[i] == 0 ? T(1) / T(3) : (WCLASS[i] == 1 ? T(1) / T(18) : T(1) / T(36));
}

// c.v for a lattice vector c (components -1, 0, 1) over its nonzero
// components only: with c known at compile time this is at most one add or
// subtract (a sum started from 0 would keep a 0 + x, which is not x for -0).
template <typename T>
__device__ __forceinline__ T cdot(int cx, int cy, int cz, T x, T y, T z) {
  T r = T(0);
  bool any = false;
  if (cx != 0) { r = cx > 0 ? x : -x; any = true; }
  if (cy != 0) { r = any ? (cy > 0 ? r + y : r - y) : (cy > 0 ? y : -y); any = true; }
  if (cz != 0) r = any ? (cz > 0 ? r + z : r - z) : (cz > 0 ? z : -z);
  return r;
}

// ---- records -------------------------------------------------------------
template <typename T>
struct alignas(4 * sizeof(T)) V4 {
  T x, y, z, w;
};
template <typename T>
struct alignas(2 * sizeof(T)) V2 {
  T x, y;
};

// Per-run parameters in device memory (read through the scalar cache).
struct RunDev {
  int32_t nx, ny, nz, visc;   // visc: -1 Newtonian, 0 polymer in A, 1 in B
  int64_t n;                  // nodes of this run
  int64_t ld;                 // stride between the component arrays of a field
                              // (n padded so arrays do not alias in HBM channels)
  int64_t off;                // offset of this run inside the pools, in strides
  int32_t target;             // steps to take in the current step call
  int32_t base;               // the run's step count at call start (mod 2^31)
  int32_t min_cc;             // smallest droplet piece counted (nodes)
  int32_t pad0;
  double u_wall, G;
  double tau[2], inv_tau[2];          // even (viscous) rate: BGK tau, or TRT tau^+
  double inv_tauP, etaP_over_tauP, L2;
  double chi_lo, inv_chi_range;
  double tau_m[2], inv_tau_m[2];      // odd (momentum) rate: tau^- (= tau under BGK)
};

// One tile of the step launch: a bx*by column block at (x0, y0) covering
// planes z0 .. z1-1 of run `run` (run < 0: padding entry, skipped).
struct Tile {
  int32_t run, x0, y0, z0, z1;
};

// ---- storage conversions -------------------------------------------------
// Populations are stored shifted by the first two moments of the node that
// holds them: g_i = f_i - w_i (rho_s(x) + 3 c_i.j_s(x)), with rho_s(x) and
// j_s(x) the density and momentum arrays of the same parity.  The shift is
// the equilibrium up to first order in the velocity, so g_i holds only the
// second-order and non-equilibrium parts: small values, whose rounding (FP16
// keeps 11 significant bits) is small against the flow.  The moments
// themselves are carried by the rho / j arrays in the compute type.  Stored
// as S in units of 1/kScale (FP16 keeps g * 2^12, which moves the small
// values of the minority phase out of the subnormal range; |g| < 1 stays far
// below the FP16 maximum), arithmetic in T.  The time step rounds FP16 values
// stochastically (put); set-up and import round to nearest even (store).
template <typename T, typename S>
struct Store;

// Population stores stream past the caches (each value is read back only by
// the next step, long after the line would have been evicted).
#ifndef LBM_NT_STORES
#define LBM_NT_STORES 1
#endif

// SplitMix64's output function (G. Steele, D. Lea, C. Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014): the word of counter k of
// seed s is splitmix64_mix(s + (k + 1) * 0x9e3779b97f4a7c15).
__host__ __device__ inline uint64_t splitmix64_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

// MurmurHash3's 32-bit finaliser (A. Appleby, public domain): a bijective
// mixer, used as a counter-based generator.
__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85ebca6bu;
  h ^= h >> 13;
  h *= 0xc2b2ae35u;
  h ^= h >> 16;
  return h;
}
template <typename T>
struct Store<T, T> {
  static constexpr bool kRandom = false;
  static constexpr double kScale = 1.0;
  static __device__ __forceinline__ T load(const T* p, int64_t k) { return p[k]; }
  // the stored form of v (r: random word, unused here), and its store
  using Raw = T;
  static __device__ __forceinline__ Raw encode(T v, uint32_t /*r*/) { return v; }
  static __device__ __forceinline__ void write(T* p, int64_t k, Raw v) {
#if LBM_NT_STORES
    __builtin_nontemporal_store(v, p + k);
#else
    p[k] = v;
#endif
  }
  static __device__ __forceinline__ void put(T* p, int64_t k, T v, uint32_t r) {
    write(p, k, encode(v, r));
  }
  static __device__ __forceinline__ void store(T* p, int64_t k, T v) { put(p, k, v, 0u); }
};

#ifndef LBM_FP16_RN
#define LBM_FP16_RN 0   // 1: round to nearest even instead of stochastically
#endif

typedef _Float16 half2v __attribute__((ext_vector_type(2)));

template <>
struct Store<float, __half> {
  static constexpr bool kRandom = !LBM_FP16_RN;
  static constexpr double kScale = 4096.0;
  static __device__ __forceinline__ float load(const __half* p, int64_t k) {
    return __half2float(p[k]);
  }
  static __device__ __forceinline__ void raw_store(__half* p, int64_t k, unsigned short h) {
#if LBM_NT_STORES
    __builtin_nontemporal_store(h, reinterpret_cast<unsigned short*>(p) + k);
#else
    reinterpret_cast<unsigned short*>(p)[k] = h;
#endif
  }
  // Stochastic rounding to FP16 with the random word r: gfx950's conversion
  // adds the top 13 bits of r to the 13 mantissa bits of |v| that FP16 drops
  // and truncates them, so |v| rounds up with probability
  // (|v| - lower)/spacing and the rounding error has zero mean.
  // Deterministic rounding leaves the same error at every node of a uniform
  // region, step after step, and that coherent bias accumulates in the flow.
  // the FP16 bits (in the low half of a 32-bit register) and their store
  using Raw = uint32_t;
  static __device__ __forceinline__ Raw encode(float v, uint32_t r) {
#if LBM_FP16_RN
    (void)r;
    return __builtin_bit_cast(unsigned short, __float2half_rn(v));
#else
    // the conversion writes the low half of a register; the high half keeps
    // the bits of v (not stored), which spares clearing a register first
    const half2v h = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(half2v, v), v, r, false);
    return __builtin_bit_cast(uint32_t, h);
#endif
  }
  static __device__ __forceinline__ void write(__half* p, int64_t k, Raw v) {
    raw_store(p, k, (unsigned short)v);
  }
  static __device__ __forceinline__ void put(__half* p, int64_t k, float v, uint32_t r) {
    write(p, k, encode(v, r));
  }
  static __device__ __forceinline__ void store(__half* p, int64_t k, float v) {
    raw_store(p, k, __builtin_bit_cast(unsigned short, __float2half_rn(v)));
  }
};

// ---- pools: all runs' fields, concatenated per field -----------------------
template <typename T, typename S>
struct Pools {
  S* f[2];            // [38][n] per run (component-major, then direction)
  T* rho[2];          // [2][n] per run: rho_A, rho_B
  T* j[2];            // [6][n] per run: j_A xyz, j_B xyz
  T* C[2];            // [6][n] per run: xx yy zz xy xz yz
  T* u;               // [3][n] per run: physical velocity (observe / export)
  uint32_t* status;   // per run: bit 0 non-finite, bit 1 tr C >= L^2
};

constexpr uint32_t ST_NAN = 1u;
constexpr uint32_t ST_FENE = 2u;
constexpr uint32_t ST_CC = 4u;   // component labelling hit its iteration cap

// Element of a uniform array base at a 32-bit byte offset: global accesses
// then take the scalar base + 32-bit vector offset form (the library keeps
// every per-run array below 4 GiB).
template <typename P>
__device__ __forceinline__ P* boff(P* base, uint32_t off) {
  using B = typename std::conditional<std::is_const<P>::value, const char, char>::type;
  return reinterpret_cast<P*>(reinterpret_cast<B*>(base) + off);
}

// Reciprocal in the compute type: FP64 divides exactly; FP32 uses the
// hardware reciprocal (1 ulp), whose error is far below the FP32 path's
// bars against FP64.
__device__ __forceinline__ double rcpT(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcpT(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int wrapm(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }
__device__ __forceinline__ int clampz(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

}  // namespace lbm
