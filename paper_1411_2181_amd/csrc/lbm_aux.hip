// Per-node auxiliary kernels: initial state, observable reductions and
// connected-component labelling of the droplet.
//
// All kernels use a (AUX_BLOCKS, nruns) grid: block b of run r owns the
// contiguous node range [b*chunk, (b+1)*chunk) of that run.  Reductions are
// two-stage with a fixed combination order, so every observable is
// bit-reproducible.
#include "lbm_internal.h"

namespace lbm {

__device__ __forceinline__ void node_range(int64_t N, int64_t& beg, int64_t& end) {
  const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
  beg = (int64_t)blockIdx.x * chunk;
  end = beg + chunk < N ? beg + chunk : N;
}

// ---- initial state ----------------------------------------------------------
// Sphere |x - c|^2 < R^2 (strict) holds rho_A = rho_major, rho_B = rho_minor,
// the rest the reverse (Section 3: a spherical droplet at mid-gap, shear
// started from rest); f = w_i rho_s, i.e. zero momentum and the shifted
// value g_i = 0 against the node's moments; C = I.  Written at parity 0.
template <typename T, typename S>
__global__ void k_init(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  const int64_t N = R.ld;   // stride between the component arrays of a field
  int64_t beg, end;
  node_range(R.n, beg, end);
  const double rad = a.radius_centre[4 * r], cx = a.radius_centre[4 * r + 1];
  const double cy = a.radius_centre[4 * r + 2], cz = a.radius_centre[4 * r + 3];
  const double rmaj = a.rho_init[4 * r], rmin = a.rho_init[4 * r + 1];
  const double noise = a.rho_init[4 * r + 2];
  const uint64_t seed = __builtin_bit_cast(uint64_t, a.rho_init[4 * r + 3]);
  using St = Store<T, S>;
  S* f = a.P.f[0] + 38 * R.off;
  T* rho = a.P.rho[0] + 2 * R.off;
  T* J = a.P.j[0] + 6 * R.off;
  T* C = a.P.C[0] + 6 * R.off;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    const int x = (int)(n % R.nx);
    const int y = (int)((n / R.nx) % R.ny);
    const int z = (int)(n / ((int64_t)R.nx * R.ny));
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    const bool inside = dx * dx + dy * dy + dz * dz < rad * rad;
    double rho_s[2] = {inside ? rmaj : rmin, inside ? rmin : rmaj};
    if (noise > 0.0) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        // u in [-1, 1) from the SplitMix64 word of counter 2n + s
        const uint64_t w = splitmix64_mix(seed + (uint64_t)(2 * n + s + 1) * 0x9e3779b97f4a7c15ull);
        const double u = (double)(w >> 11) * 0x1p-52 - 1.0;
        const double t = noise * u;   // separate statements: no fused multiply-add
        rho_s[s] = rho_s[s] * (1.0 + t);
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      rho[s * N + n] = T(rho_s[s]);
#pragma unroll
      for (int c = 0; c < 3; ++c) J[(3 * s + c) * N + n] = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) St::store(f + ((int64_t)s * Q + i) * N, n, T(0));
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) C[k * N + n] = k < 3 ? T(1) : T(0);
  }
}

// ---- observables ---------------------------------------------------------------
__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

__host__ __device__ constexpr int obs_kind(int k) {  // 0 sum, 1 max, 2 min
  return (k == OB_U2MAX || k == OB_TRCMAX || k == OB_XMAX) ? 1 : (k == OB_XMIN ? 2 : 0);
}

// Phase field phi = (rho_A - rho_B)/(rho_A + rho_B), droplet weight
// w = max(phi, 0); moments of w about the box centre; x-extent of phi > 0;
// max |u|^2 and max tr C; count of non-finite nodes.  FP64 throughout.
template <typename T, typename S>
__global__ void __launch_bounds__(AUX_THREADS) k_obs_partial(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  const int par = a.use_parity ? (R.base & 1) : 0;
  const int64_t N = R.ld;   // stride between the component arrays of a field
  int64_t beg, end;
  node_range(R.n, beg, end);
  const T* rho = a.P.rho[par] + 2 * R.off;
  // a Newtonian run never updates C, which stays at parity 0
  const T* C = a.P.C[R.visc >= 0 ? par : 0] + 6 * R.off;
  const T* U = a.P.u + 3 * R.off;
  const double hx = 0.5 * (R.nx - 1), hy = 0.5 * (R.ny - 1), hz = 0.5 * (R.nz - 1);
  double acc[NOBS];
#pragma unroll
  for (int k = 0; k < NOBS; ++k) acc[k] = 0.0;
  acc[OB_XMIN] = 1e300;
  acc[OB_XMAX] = -1e300;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    const int x = (int)(n % R.nx);
    const int y = (int)((n / R.nx) % R.ny);
    const int z = (int)(n / ((int64_t)R.nx * R.ny));
    const double rA = (double)rho[n], rB = (double)rho[N + n];
    const double phi = (rA - rB) / (rA + rB);
    const double w = phi > 0.0 ? phi : 0.0;
    const double xr = x - hx, yr = y - hy, zr = z - hz;
    acc[OB_MA] += rA;
    acc[OB_MB] += rB;
    acc[OB_W] += w;
    acc[OB_WX] += w * xr;
    acc[OB_WY] += w * yr;
    acc[OB_WZ] += w * zr;
    acc[OB_WXX] += w * xr * xr;
    acc[OB_WXZ] += w * xr * zr;
    acc[OB_WZZ] += w * zr * zr;
    if (phi > 0.0) {
      acc[OB_XMIN] = fmin(acc[OB_XMIN], (double)x);
      acc[OB_XMAX] = fmax(acc[OB_XMAX], (double)x);
    }
    const double u0 = U[n], u1 = U[N + n], u2 = U[2 * N + n];
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    const double tr = (double)C[n] + (double)C[N + n] + (double)C[2 * N + n];
    if (!(isfinite(rA + rB) && isfinite(uu) && isfinite(tr))) acc[OB_NONFINITE] += 1.0;
    acc[OB_U2MAX] = fmax(acc[OB_U2MAX], uu);
    acc[OB_TRCMAX] = fmax(acc[OB_TRCMAX], tr);
  }
  __shared__ double sh[NOBS][AUX_THREADS / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NOBS; ++k) {
    const int kind = obs_kind(k);
    const double v = kind == 0 ? wsum(acc[k]) : (kind == 1 ? wmax(acc[k]) : wmin(acc[k]));
    if (lane == 0) sh[k][wave] = v;
  }
  __syncthreads();
  if (threadIdx.x < NOBS) {
    const int k = threadIdx.x;
    const int kind = obs_kind(k);
    double v = sh[k][0];
    for (int wv = 1; wv < AUX_THREADS / 64; ++wv)
      v = kind == 0 ? v + sh[k][wv] : (kind == 1 ? fmax(v, sh[k][wv]) : fmin(v, sh[k][wv]));
    a.partials[((int64_t)r * gridDim.x + blockIdx.x) * NOBS + k] = v;
  }
}

template <typename T, typename S>
__global__ void k_obs_final(AuxArgs<T, S> a, int nblocks) {
  const int r = blockIdx.x;
  const int k = threadIdx.x;
  if (k >= NOBS) return;
  const int kind = obs_kind(k);
  const double* p = a.partials + (int64_t)r * nblocks * NOBS;
  double v = p[k];
  for (int b = 1; b < nblocks; ++b) {
    const double q = p[b * NOBS + k];
    v = kind == 0 ? v + q : (kind == 1 ? fmax(v, q) : fmin(v, q));
  }
  a.obs[r * NOBS + k] = v;
}

// ---- connected components of {phi > 0} -----------------------------------------
// Lock-free union-find on node indices: each set's root is its smallest
// index; unions link the larger root under the smaller with atomicMin, so
// parent pointers only decrease.  Root searches halve the path as they walk
// (each visited node is pointed at its grandparent, with atomicMin: the
// grandparent is in the same set and no larger than the parent), which keeps
// the trees shallow even for a long, thread-shaped droplet whose unions would
// otherwise build chains as long as the thread.  A generous iteration cap
// turns any unforeseen livelock into a status flag instead of a hang.
constexpr int CC_CAP = 1 << 22;

__device__ __forceinline__ int32_t ld_agent(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int32_t cc_find(int32_t* L, int32_t i) {
  for (int guard = 0; guard < CC_CAP; ++guard) {
    const int32_t p = ld_agent(L + i);
    if (p == i) return i;
    const int32_t gp = ld_agent(L + p);
    if (gp == p) return p;
    atomicMin(L + i, gp);   // path halving
    i = gp;
  }
  return i;
}

__device__ __forceinline__ bool cc_unite(int32_t* L, int32_t a, int32_t b) {
  for (int guard = 0; guard < CC_CAP; ++guard) {
    a = cc_find(L, a);
    b = cc_find(L, b);
    if (a == b) return true;
    if (a > b) { const int32_t t = a; a = b; b = t; }
    const int32_t old = atomicMin(L + b, a);
    if (old == b) return true;
    b = old;
  }
  return false;
}

template <typename T, typename S>
__global__ void k_cc_init(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  const int par = a.use_parity ? (R.base & 1) : 0;
  int64_t beg, end;
  node_range(R.n, beg, end);
  const T* rho = a.P.rho[par] + 2 * R.off;
  int32_t* L = a.labels + R.off;
  int32_t* cnt = a.counts + R.off;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    L[n] = rho[n] > rho[R.ld + n] ? (int32_t)n : -1;   // phi > 0  <=>  rho_A > rho_B
    cnt[n] = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.ncomp[r] = 0;
}

template <typename T, typename S>
__global__ void k_cc_merge(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  int64_t beg, end;
  node_range(R.n, beg, end);
  int32_t* L = a.labels + R.off;
  bool ok = true;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    if (ld_agent(L + n) < 0) continue;
    const int x = (int)(n % R.nx);
    const int y = (int)((n / R.nx) % R.ny);
    const int z = (int)(n / ((int64_t)R.nx * R.ny));
    const int64_t plane = (int64_t)R.nx * R.ny;
    const int64_t nbx = n - x + (x + 1 == R.nx ? 0 : x + 1);
    const int64_t nby = n + ((y + 1 == R.ny ? 0 : y + 1) - y) * (int64_t)R.nx;
    if (ld_agent(L + nbx) >= 0) ok &= cc_unite(L, (int32_t)n, (int32_t)nbx);
    if (ld_agent(L + nby) >= 0) ok &= cc_unite(L, (int32_t)n, (int32_t)nby);
    if (z + 1 < R.nz && ld_agent(L + n + plane) >= 0) ok &= cc_unite(L, (int32_t)n, (int32_t)(n + plane));
  }
  if (!ok) atomicOr(a.P.status + r, ST_CC);
}

template <typename T, typename S>
__global__ void k_cc_flatten(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  int64_t beg, end;
  node_range(R.n, beg, end);
  int32_t* L = a.labels + R.off;
  int32_t* cnt = a.counts + R.off;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    if (L[n] < 0) continue;
    const int32_t root = cc_find(L, (int32_t)n);
    atomicAdd(cnt + root, 1);
  }
}

template <typename T, typename S>
__global__ void k_cc_count(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  int64_t beg, end;
  node_range(R.n, beg, end);
  const int32_t* L = a.labels + R.off;
  const int32_t* cnt = a.counts + R.off;
  // each counted piece (a root of at least min_cc nodes) takes a slot and
  // records its size there; the host orders the sizes
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x)
    if (L[n] == (int32_t)n && cnt[n] >= R.min_cc) {
      const int slot = atomicAdd(a.ncomp + r, 1);
      if (slot < MAX_PIECES) a.pieces[r * MAX_PIECES + slot] = cnt[n];
    }
}

// ---- small helpers ----------------------------------------------------------------
__global__ void k_set_step(int32_t* g, int32_t v) { if (threadIdx.x == 0 && blockIdx.x == 0) *g = v; }
__global__ void k_inc_step(int32_t* g) { if (threadIdx.x == 0 && blockIdx.x == 0) *g = *g + 1; }
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_set_step(int32_t* g, int32_t v, hipStream_t s) { k_set_step<<<1, 64, 0, s>>>(g, v); }
void launch_inc_step(int32_t* g, hipStream_t s) { k_inc_step<<<1, 64, 0, s>>>(g); }
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  const int64_t blocks = (n + 255) / 256;
  k_fill_u32<<<(unsigned)(blocks < 1024 ? blocks : 1024), 256, 0, s>>>(p, v, n);
}

template <typename T, typename S>
void launch_init(const AuxArgs<T, S>& a, hipStream_t s) {
  k_init<T, S><<<dim3(AUX_BLOCKS, a.nruns), AUX_THREADS, 0, s>>>(a);
}
template <typename T, typename S>
void launch_observe(const AuxArgs<T, S>& a, hipStream_t s) {
  k_obs_partial<T, S><<<dim3(AUX_BLOCKS, a.nruns), AUX_THREADS, 0, s>>>(a);
  k_obs_final<T, S><<<a.nruns, 64, 0, s>>>(a, AUX_BLOCKS);
}
template <typename T, typename S>
void launch_components(const AuxArgs<T, S>& a, hipStream_t s) {
  const dim3 grid(AUX_BLOCKS, a.nruns), block(AUX_THREADS);
  k_cc_init<T, S><<<grid, block, 0, s>>>(a);
  k_cc_merge<T, S><<<grid, block, 0, s>>>(a);
  k_cc_flatten<T, S><<<grid, block, 0, s>>>(a);
  k_cc_count<T, S><<<grid, block, 0, s>>>(a);
}

#define LBM_INST(T, S)                                                   \
  template void launch_init<T, S>(const AuxArgs<T, S>&, hipStream_t);     \
  template void launch_observe<T, S>(const AuxArgs<T, S>&, hipStream_t);  \
  template void launch_components<T, S>(const AuxArgs<T, S>&, hipStream_t);
LBM_INST(double, double)
LBM_INST(float, float)
LBM_INST(float, __half)
#undef LBM_INST

}  // namespace lbm
