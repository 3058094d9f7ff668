// Step kernel of the hybrid LB / FENE-P solver (gfx950): one launch per step.
//
// Dependencies of one step n -> n+1 at a node x:
//   * the lattice-Boltzmann part pulls the 19 populations that arrive at x,
//     each collided at its source node s = x - c_i with the equilibrium of s;
//     that equilibrium needs the force at s: the Shan-Chen force from the
//     densities of s's neighbours and the polymer force, the centred
//     divergence of the stress T = chi (eta_P/tau_P)(f C - I) over s's face
//     neighbours (Section 2, Eqs. (1) and (3));
//   * the FENE-P update at x (Eqs. (2) and (4)) needs the physical velocity,
//     hence the force, at x's face neighbours.
// So a tile of nodes needs the state within two nodes of it: densities and C
// at radius 2, momenta and populations at radius 1.  The kernel reads exactly
// that (state n, parity p) and writes state n+1 (parity p^1): populations,
// densities, momenta and C.  No intermediate field goes through HBM.
//
// Work split.  One workgroup of 2 * bx * by threads per tile.  For the forces
// every thread owns one position of the tile + 1-node frame (and of the
// 2-node frame); for the collision and the FENE-P update the threads with
// threadIdx.z = s handle component s of the bx * by columns (s = 0 updates
// C_xx, C_yy, C_zz, s = 1 updates C_xy, C_xz, C_yz).
//
// z-march.  The workgroup advances its column block plane by plane, with two
// barriers per plane.  In the iteration of plane r:
//   phase X: stage plane r of both densities (LDS ring) and of the stress T
//            (computed once per node, Peterlin factor in FP64; transient);
//            collide, stream and update C at plane r-3 (records, moments,
//            velocities and C of planes r-4 .. r-2 from LDS rings);
//   phase Y: stage C of plane r (ring); add plane r's terms of the stress
//            divergence at planes r-1, r, r+1 (per thread, in registers);
//            finalise plane r-1 on the 1-node frame: Shan-Chen force from the
//            density ring, polymer force, velocity shift, the records the
//            collision reads, the node moments and the physical velocity.
// The loads of the next plane's densities and C, of the populations of the
// next plane to collide and of the momenta of plane r are in flight while
// the rest of the iteration computes; the population loads and the moment
// and C stores are spread over both phases (FP32, FP64).  The registers of
// the iteration's global stores are held to its end, so that no store's
// data is overwritten while it may still be read (a wait on the store).
//
// Storage and collision.  Populations are held as
// g_i = f_i - w_i (rho + 3 c_i.j) against the moments of the node that holds
// them (see Store).  With w = 1/tau and the record of the source node s,
// a = rho (1 - 1.5 w |u^eq|^2), P = w rho u^eq + (1 - w) j (the post-collision
// momentum), b = 4.5 w rho, the BGK collision f* = (1 - w) f + w f^eq reads
//   f*_i(s) = (1 - w) g_i(s) + w_i [a + 3 c_i.P + b (c_i.u^eq)^2];
// the arriving value is re-referenced to the moments of x, the new moments
// of x are the old ones plus the sums of the re-referenced values, and the
// value stored is the difference to the new moments.  With two relaxation
// times (TRT: the parts of f even and odd under c -> -c relax at w+ = 1/tau
// and w- = 1/tau^-), a and b take w+, P takes w-, and the pulled term is
// alpha g_i(s) + beta g_opp(i)(s), alpha = 1 - (w+ + w-)/2, beta =
// (w- - w+)/2: the instance with TRT loads the opposite population of each
// source as well.  The records are read
// from LDS one whole 16-byte vector at a time: lanes 16 bytes apart reading
// fewer values would share LDS banks.
//
// The set-up (walls at -+U_w half a link outside z = 0 and z = nz-1, periodic
// x and y) is Section 3.  A node's arithmetic does not depend on the tile
// shape or on the other runs of a batch, so every launch shape and batch
// composition is bit-identical.
#include "lbm_internal.h"

#include <type_traits>

namespace lbm {

__device__ __forceinline__ int wrapp(int v, int n) { return ((v % n) + n) % n; }

// Frame geometry of a BX x BY tile: the 1-node frame (tile + 1 on each side)
// and the 2-node frame, both in row-major order.
template <int BX, int BY>
struct Frame {
  static constexpr int NT = BX * BY, NW = 2 * NT;        // columns, threads
  static constexpr int HX1 = BX + 2, HY1 = BY + 2, N1 = HX1 * HY1;
  static constexpr int HX2 = BX + 4, HY2 = BY + 4, N2 = HX2 * HY2;
  static constexpr int K2 = (N2 + NW - 1) / NW;          // 2-frame positions per thread
  static_assert(N1 <= NW, "one 1-frame position per thread");
};

template <typename T, int BX, int BY>
struct StepLds {
  using F = Frame<BX, BY>;
  T rho[3][2][F::N2];         // planes mod 3: rho_A, rho_B on the 2-frame
  T stress[6][F::N2];         // plane r: T on the 2-frame
  T C[4][6][F::N1];           // planes mod 4: C on the 1-frame
  V4<T> rec[3][2][2][F::N1];  // planes mod 3, component: (a, P), (u^eq, b)
  T u[3][3][F::N1];           // planes mod 3: physical velocity on the 1-frame
  T M[2][2][4][F::NT];        // planes mod 2, component: rho, j of the tile columns
};

// A whole record from LDS in one access: the lanes of a wave read records
// 16 B (FP32) apart, and only full-width reads keep them on distinct banks
// (a read of one or two of the four values would put 2-4 lanes on a bank).
template <typename T>
__device__ __forceinline__ V4<T> lds_v4(const V4<T>* p) {
  typedef T vec4 __attribute__((ext_vector_type(4)));
  typedef const volatile __attribute__((address_space(3))) vec4* lds_vec4;
  const vec4 v = *(lds_vec4)p;
  return V4<T>{v.x, v.y, v.z, v.w};
}

template <int BX, int BY, typename T>
constexpr bool step_fits() { return sizeof(StepLds<T, BX, BY>) <= 160 * 1024; }

// Shapes with a compiled instance (those whose rings fit the 160 KiB of LDS
// in the compute type).
#define LBM_FOR_SHAPES(M) M(32, 8) M(16, 16) M(16, 8) M(8, 16)


template <typename T, typename S, int BX, int BY, int DG, bool TRT>
__global__ void __launch_bounds__(2 * BX * BY) k_step(StepArgs<T, S> a) {
  using F = Frame<BX, BY>;
  constexpr int NT = F::NT, NW = F::NW, HX1 = F::HX1, N1 = F::N1, HX2 = F::HX2, N2 = F::N2;
  constexpr int K2 = F::K2;
  static_assert(step_fits<BX, BY, T>(), "LDS rings exceed 160 KiB");
  __shared__ StepLds<T, BX, BY> L;
  using St = Store<T, S>;
  const T kS = T(St::kScale), ikS = T(1.0 / St::kScale);
  constexpr bool kHalf = std::is_same<S, __half>::value;
  constexpr int kPopsEarly = kHalf ? Q : 8;     // population loads before barrier (2)
  constexpr bool kMomentsLate = !kHalf;         // moment and C stores after it
  const int g = *a.gstep;
  // every wave lies in one threadIdx.z half (bx * by is a multiple of 64),
  // so the component index is wave-uniform: read it as a scalar, which keeps
  // the per-component array bases in scalar registers
  static_assert((BX * BY) % 64 == 0, "a wave must not straddle the two components");
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y;
  const int s = __builtin_amdgcn_readfirstlane((int)threadIdx.z);
  const int tid = (s * BY + ty) * BX + tx;

  // this thread's 1-frame position (threads past N1 repeat the last one and
  // store nothing) and 2-frame positions
  const bool has1 = tid < N1;
  const int e1 = has1 ? tid : N1 - 1;
  const int h1x = e1 % HX1, h1y = e1 / HX1;
  const int c2of1 = (h1y + 1) * HX2 + h1x + 1;              // its 2-frame index
  const bool inner = h1x >= 1 && h1x <= BX && h1y >= 1 && h1y <= BY;
  const int mcol = (h1y - 1) * BX + (h1x - 1);               // its tile column if inner
  int e2[K2], q1[K2];
  bool has2[K2];
#pragma unroll
  for (int k = 0; k < K2; ++k) {
    has2[k] = tid + k * NW < N2;
    e2[k] = has2[k] ? tid + k * NW : N2 - 1;
    const int hx = e2[k] % HX2, hy = e2[k] / HX2;
    const bool in1 = hx >= 1 && hx <= BX + 2 && hy >= 1 && hy <= BY + 2;
    q1[k] = has2[k] && in1 ? (hy - 1) * HX1 + (hx - 1) : -1;
  }
  const int lc = (ty + 1) * HX1 + (tx + 1);   // own column in the 1-frame
  const int oc = ty * BX + tx;                // own column in the tile

  for (int t = (int)blockIdx.x; t < a.ntiles; t += (int)gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz, nxy = nx * ny;
    const bool visc = R.visc >= 0;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool active = x < nx && y < ny;
    // run parameters in registers: a load of them inside the z-march would
    // wait for every load in flight as well
    const T G = T(R.G);
    const T itA = T(R.inv_tau[0]), itB = T(R.inv_tau[1]);     // w+ (BGK: w)
    // tau^- and w-: in the BGK instance every run has tau^- = tau
    const T tmA = T(TRT ? R.tau_m[0] : R.tau[0]), tmB = T(TRT ? R.tau_m[1] : R.tau[1]);
    const T itmA = TRT ? T(R.inv_tau_m[0]) : itA, itmB = TRT ? T(R.inv_tau_m[1]) : itB;
    const T om = s ? itB : itA;   // w+ of this thread's component
    const T omm = s ? itmB : itmA;
    // weights of g_i(s) and g_opp(i)(s) in the collision (BGK: 1 - w, 0)
    const T om1 = TRT ? T(1) - T(0.5) * (om + omm) : T(1) - om;
    const T omb = T(0.5) * (omm - om);
    const T uw = T(R.u_wall);
    const int vph = R.visc;
    const T chi_lo = T(R.chi_lo), ichr = T(R.inv_chi_range), eP = T(R.etaP_over_tauP);
    const T itP = T(R.inv_tauP);
    const double L2 = R.L2;
    const T L2m3 = T(R.L2 - 3.0);
    const uint32_t hstep = ((uint32_t)(R.base + g) * 2u + (uint32_t)s) * 0x85ebca77u;

    const T* __restrict__ rho_in = a.P.rho[par] + 2 * R.off;
    const T* __restrict__ J_in = a.P.j[par] + 6 * R.off;
    const T* __restrict__ C_in = a.P.C[par] + 6 * R.off;
    const S* __restrict__ fs = a.P.f[par] + (38 * R.off + (int64_t)s * Q * N);
    S* __restrict__ fo = a.P.f[par ^ 1] + (38 * R.off + (int64_t)s * Q * N);
    T* __restrict__ rho_out = a.P.rho[par ^ 1] + 2 * R.off + s * N;
    T* __restrict__ j_out = a.P.j[par ^ 1] + 6 * R.off + 3 * s * N;
    T* __restrict__ C_out = a.P.C[par ^ 1] + 6 * R.off;

    // plane offsets of the frame positions (periodic in x and y)
    const int col1 = wrapp(tl.y0 + h1y - 1, ny) * nx + wrapp(tl.x0 + h1x - 1, nx);
    int col2[K2];
#pragma unroll
    for (int k = 0; k < K2; ++k)
      col2[k] = wrapp(tl.y0 + e2[k] / HX2 - 2, ny) * nx + wrapp(tl.x0 + e2[k] % HX2 - 2, nx);

    // Pulls: byte offsets inside one direction array (a run's array is
    // < 4 GiB, which the library checks).  Inactive threads of a ragged tile
    // address the edge node (loads in bounds, values unused).
    const int xq = x < nx ? x : nx - 1, yq = y < ny ? y : ny - 1;
    const int xm = xq == 0 ? nx - 1 : xq - 1, xp = xq >= nx - 1 ? 0 : xq + 1;
    const int ym = yq == 0 ? ny - 1 : yq - 1, yp = yq >= ny - 1 ? 0 : yq + 1;
    constexpr uint32_t SZ = sizeof(S);
    const uint32_t pb = (uint32_t)nxy * SZ;
    const uint32_t rowb[3] = {(uint32_t)(ym * nx) * SZ, (uint32_t)(yq * nx) * SZ,
                              (uint32_t)(yp * nx) * SZ};
    const uint32_t colb[3] = {(uint32_t)xm * SZ, (uint32_t)xq * SZ, (uint32_t)xp * SZ};
    // direction i's array: the base of its group of DG arrays (uniform,
    // 64-bit) plus a 32-bit byte offset (i % DG) * db + position
    const uint32_t db = (uint32_t)N * SZ;
    auto grp = [&](auto* base, int i) { return base + (int64_t)(i / DG * DG) * N; };
    const int own = yq * nx + xq;

    T raw[K2][8];    // densities and C of the 2-frame positions (next plane)
    T cst[K2][6];    // C of the plane being staged, kept for the C ring
    T jv[6];         // momenta of the 1-frame position (plane to finalise)
    T pops[Q];       // populations arriving at the own column (plane to collide)
    T popo[TRT ? Q : 1];   // with TRT: the opposite population of each source
    // values of the iteration's global stores: their registers are held to
    // the end of the iteration, so that none is overwritten while its store
    // may still be reading it (which would wait for the store to finish)
    T held[Q + 7];
    typename St::Raw held_s[Q];
    T acc[3][3];     // stress divergence of the 1-frame position: planes r-1, r, r+1
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[p][c] = T(0);
    uint32_t st = 0;

    // ---- loads ---------------------------------------------------------------
    constexpr uint32_t TB = sizeof(T);
    auto load_raw = [&](int r) {
      const uint32_t zo = (uint32_t)(clampz(r, nz) * nxy) * TB;
#pragma unroll
      for (int k = 0; k < K2; ++k) {
        const uint32_t mo = zo + (uint32_t)col2[k] * TB;
        raw[k][0] = *boff(rho_in, mo);
        raw[k][1] = *boff(rho_in + N, mo);
        if (visc) {
#pragma unroll
          for (int c = 0; c < 6; ++c) raw[k][2 + c] = *boff(C_in + c * N, mo);
        }
      }
    };
    auto load_j = [&](int r) {
      const uint32_t mo = (uint32_t)(clampz(r, nz) * nxy + col1) * TB;
#pragma unroll
      for (int c = 0; c < 6; ++c) jv[c] = *boff(J_in + c * N, mo);
    };
    // populations arriving at the own column in plane zz: pulled from
    // x - c_i, or the node's own opposite
    // population where the link crosses the wall
    auto load_pops = [&](int zz, auto lo_c, auto hi_c) {
      constexpr int lo = decltype(lo_c)::value, hi = decltype(hi_c)::value;
      const uint32_t ownb = (uint32_t)zz * pb + rowb[1] + colb[1];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (i < lo || i >= hi) continue;
        const int zs = zz - CZ[i];
        const S* src = grp(fs, i);
        uint32_t off = (uint32_t)(i % DG) * db + ((uint32_t)zs * pb + rowb[1 - CY[i]] + colb[1 - CX[i]]);
        if (CZ[i] != 0) {
          const bool in = zs >= 0 && zs < nz;
          src = in ? src : grp(fs, OPPI[i]);
          off = in ? off : (uint32_t)(OPPI[i] % DG) * db + ownb;
        }
        pops[i] = St::load(boff(src, off), 0);
        if constexpr (TRT) {
          // g_opp(i) at the source, or g_i of x itself across a wall
          const S* srco = grp(fs, OPPI[i]);
          uint32_t offo = (uint32_t)(OPPI[i] % DG) * db +
                          ((uint32_t)zs * pb + rowb[1 - CY[i]] + colb[1 - CX[i]]);
          if (CZ[i] != 0) {
            const bool in = zs >= 0 && zs < nz;
            srco = in ? srco : grp(fs, i);
            offo = in ? offo : (uint32_t)(i % DG) * db + ownb;
          }
          popo[i] = St::load(boff(srco, offo), 0);
        }
      }
    };

    // ---- phase X: stage plane r ------------------------------------------------
    auto ingest = [&](int r) {
      const int sl3 = (r + 3) % 3;
#pragma unroll
      for (int k = 0; k < K2; ++k) {
        const T rA = raw[k][0], rB = raw[k][1];
        if (has2[k]) {
          L.rho[sl3][0][e2[k]] = rA;
          L.rho[sl3][1][e2[k]] = rB;
        }
        if (visc) {
          // T = chi (eta_P/tau_P)(f C - I): chi the clamped rescaled mass
          // fraction of the polymer phase's component, f in FP64
          const T rp = vph == 0 ? rA : rB;
          T chi = (rp * rcpT(rA + rB) - chi_lo) * ichr;
          chi = chi < T(0) ? T(0) : (chi > T(1) ? T(1) : chi);
          // L^2 - tr C in FP64 (the cancellation as tr C -> L^2)
          const double tr = (double)raw[k][2] + (double)raw[k][3] + (double)raw[k][4];
          const T fP = L2m3 * rcpT(T(L2 - tr));
          const T coef = chi * eP;
          if (has2[k]) {
#pragma unroll
            for (int c = 0; c < 6; ++c)
              L.stress[c][e2[k]] = coef * (fP * raw[k][2 + c] - (c < 3 ? T(1) : T(0)));
          }
#pragma unroll
          for (int c = 0; c < 6; ++c) cst[k][c] = raw[k][2 + c];
        }
      }
    };

    // the new moments (and with withC the new C) of plane q, from the
    // registers that hold them since the collision and FENE-P update
    auto store_moments = [&](int q, bool withC) {
      const uint32_t no = (uint32_t)(q * nxy + own) * TB;
      *boff(rho_out, no) = held[Q];
      *boff(j_out, no) = held[Q + 1];
      *boff(j_out + N, no) = held[Q + 2];
      *boff(j_out + 2 * N, no) = held[Q + 3];
      if (!isfinite(held[Q] + held[Q + 1] + held[Q + 2] + held[Q + 3])) st |= ST_NAN;
      if (withC && visc) {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) *boff(C_out + (3 * s + kk) * N, no) = held[Q + 4 + kk];
        if (!isfinite(held[Q + 4] + held[Q + 5] + held[Q + 6])) st |= ST_NAN;
      }
    };

    // ---- phase X: collide and stream component s into plane q of the own
    // column.  The arithmetic runs in every iteration (on clamped or stale
    // values outside the tile's planes, and for the columns of a ragged tile
    // past the lattice), so that the populations loaded for it are consumed
    // on every path; only ok (a plane of the tile, an active column) stores.
    auto collide = [&](int q, bool ok) {
      const int n = q * nxy + own;
      const uint32_t nb = (uint32_t)n * SZ;
      const int slq = (q + 3) % 3, slm = (q + 2) % 3, slp = (q + 4) % 3;
      const int sm2 = q & 1;
      const T rx = L.M[sm2][s][0][oc];
      const T jx0 = L.M[sm2][s][1][oc], jx1 = L.M[sm2][s][2][oc], jx2 = L.M[sm2][s][3][oc];
      // the destination's part of the re-reference, k_i = 3 c_i.j(x), once
      // per pair of opposite directions (odd i; its opposite is i + 1)
      const T j30 = T(3) * jx0, j31 = T(3) * jx1, j32 = T(3) * jx2;
      T k3[Q];
      T drho = T(0), dj0 = T(0), dj1 = T(0), dj2 = T(0);
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        k3[i] = (i & 1) ? cdot(CX[i], CY[i], CZ[i], j30, j31, j32) : (i ? -k3[i - 1] : T(0));
        int sl = CZ[i] == 0 ? slq : (CZ[i] > 0 ? slm : slp);
        int src = lc - CY[i] * HX1 - CX[i];
        T sg = T(1), wall = T(0);
        if (CZ[i] != 0) {
          // the pulled value, or (where the link crosses a wall) the
          // half-way bounce-back of x's own population in o = opp(i), with
          // c_o = -c_i and the moving-wall term -6 w_o rho c_o.u_wall
          const int zs = q - CZ[i];
          const bool in = zs >= 0 && zs < nz;
          const int o = OPPI[i];
          sl = in ? sl : slq;
          src = in ? src : lc;
          sg = in ? T(1) : T(-1);
          const T uwall = CZ[o] > 0 ? uw : -uw;
          wall = in ? T(0) : ((T(6) * kS * wgt<T>(o)) * rx) * (T(CX[o]) * uwall);
        }
        const V4<T> r0 = lds_v4(&L.rec[sl][s][0][src]), r1 = lds_v4(&L.rec[sl][s][1][src]);
        // e = (f*_i(source) in units of w_i, less the destination's shift)
        //   = (a - rho(x)) + 3 c.P - k_i + b (c.u^eq)^2
        T e = r0.x - rx;
        if (i != 0) {
          T cP = cdot(CX[i], CY[i], CZ[i], r0.y, r0.z, r0.w);
          T cu = cdot(CX[i], CY[i], CZ[i], r1.x, r1.y, r1.z);
          if (CZ[i] != 0) { cP = sg * cP; cu = sg * cu; }
          e = e + (T(3) * cP - k3[i]) + r1.w * cu * cu;
        }
        T h = om1 * pops[i] + (wgt<T>(i) * kS) * e;
        if constexpr (TRT) h = h + omb * popo[i];
        if (CZ[i] != 0) h = h - wall;
        pops[i] = h;
        drho = i == 0 ? h : drho + h;
        if (CX[i] != 0) dj0 = i == 1 ? h : dj0 + T(CX[i]) * h;
        if (CY[i] != 0) dj1 = i == 3 ? h : dj1 + T(CY[i]) * h;
        if (CZ[i] != 0) dj2 = i == 5 ? h : dj2 + T(CZ[i]) * h;
      }
      // new moments; stored values against them.  FP16 rounding takes a
      // random word per value: a hash of (node, component, step) starts a
      // Weyl sequence over the directions (independent of the tile shape and
      // batch layout, and reproducible).
      T& rnew = held[Q];
      T& jn0 = held[Q + 1];
      T& jn1 = held[Q + 2];
      T& jn2 = held[Q + 3];
      rnew = rx + drho * ikS;
      jn0 = jx0 + dj0 * ikS;
      jn1 = jx1 + dj1 * ikS;
      jn2 = jx2 + dj2 * ikS;
      uint32_t hb = 0;
      if (St::kRandom) hb = fmix32((uint32_t)n * 0x9e3779b1u ^ hstep);
      T cd = T(0);   // c_i.dj, shared by the two directions of a pair
      T* out = held;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        if (i & 1) cd = cdot(CX[i], CY[i], CZ[i], dj0, dj1, dj2);
        out[i] = i == 0 ? pops[i] - wgt<T>(i) * drho
                        : pops[i] - wgt<T>(i) * (drho + T(3) * ((i & 1) ? cd : -cd));
      }
      // encoded on every path (a value kept only where stored would be a
      // loop-carried merge: register copies in every iteration)
#pragma unroll
      for (int i = 0; i < Q; ++i) held_s[i] = St::encode(out[i], hb + (uint32_t)i * 0x9e3779b9u);
      if (ok) {
#pragma unroll
        for (int i = 0; i < Q; ++i)
          St::write(boff(grp(fo, i), (uint32_t)(i % DG) * db + nb), 0, held_s[i]);
        if (!kMomentsLate) store_moments(q, false);
      }
    };

    // ---- phase X: FENE-P for this thread's C components at plane q of the own
    // column: C^{n+1} = C - A + S - (f C - I)/tau_P with centred grad u,
    // first-order upwind A and S_kl = sum_m C_km G_ml + G_mk C_ml.  Ghost
    // planes: C zero-gradient (the clamped planes of the ring), u extrapolated
    // through the wall velocity, u(-1) = 2 u_bot - u(0), u(nz) = 2 u_top - u(nz-1).
    auto fene = [&](int q, auto half, bool ok) {
      constexpr int base = decltype(half)::value * 3;
      const int su = (q + 3) % 3, sum_ = (q + 2) % 3, sup = (q + 4) % 3;
      const int sc = q & 3, scm = (q + 3) & 3, scp = (q + 1) & 3;
      const T u0 = L.u[su][0][lc], u1 = L.u[su][1][lc], u2 = L.u[su][2][lc];
      T um[3], up[3];
      if (q == 0) { um[0] = T(2) * (-uw) - u0; um[1] = -u1; um[2] = -u2; }
      else { um[0] = L.u[sum_][0][lc]; um[1] = L.u[sum_][1][lc]; um[2] = L.u[sum_][2][lc]; }
      if (q == nz - 1) { up[0] = T(2) * uw - u0; up[1] = -u1; up[2] = -u2; }
      else { up[0] = L.u[sup][0][lc]; up[1] = L.u[sup][1][lc]; up[2] = L.u[sup][2][lc]; }
      T Gm[3][3];
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        Gm[0][bb] = T(0.5) * (L.u[su][bb][lc + 1] - L.u[su][bb][lc - 1]);
        Gm[1][bb] = T(0.5) * (L.u[su][bb][lc + HX1] - L.u[su][bb][lc - HX1]);
        Gm[2][bb] = T(0.5) * (up[bb] - um[bb]);
      }
      T c[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) c[i] = L.C[sc][i][lc];
      const double tr = (double)c[0] + (double)c[1] + (double)c[2];
      if (ok && base == 0 && tr >= L2) st |= ST_FENE;
      const T fP = L2m3 * rcpT(T(L2 - tr));
      const T ua0 = u0 > T(0) ? u0 : T(0), ub0 = u0 < T(0) ? u0 : T(0);
      const T ua1 = u1 > T(0) ? u1 : T(0), ub1 = u1 < T(0) ? u1 : T(0);
      const T ua2 = u2 > T(0) ? u2 : T(0), ub2 = u2 < T(0) ? u2 : T(0);
      constexpr int KK[6] = {0, 1, 2, 0, 0, 1};
      constexpr int LL[6] = {0, 1, 2, 1, 2, 2};
      constexpr int SYM[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
      T* cn = held + Q + 4;
#pragma unroll
      for (int kk = 0; kk < 3; ++kk) {
        const int k = base + kk;
        const T ck = c[k];
        T adv = ua0 * (ck - L.C[sc][k][lc - 1]) + ub0 * (L.C[sc][k][lc + 1] - ck);
        adv += ua1 * (ck - L.C[sc][k][lc - HX1]) + ub1 * (L.C[sc][k][lc + HX1] - ck);
        adv += ua2 * (ck - L.C[scm][k][lc]) + ub2 * (L.C[scp][k][lc] - ck);
        T Sk = c[SYM[KK[k]][0]] * Gm[0][LL[k]] + Gm[0][KK[k]] * c[SYM[0][LL[k]]];
#pragma unroll
        for (int mm = 1; mm < 3; ++mm)
          Sk += c[SYM[KK[k]][mm]] * Gm[mm][LL[k]] + Gm[mm][KK[k]] * c[SYM[mm][LL[k]]];
        const T delta = k < 3 ? T(1) : T(0);
        cn[kk] = ck + (-adv + Sk - (fP * ck - delta) * itP);
      }
      if (!kMomentsLate && ok) {
        const uint32_t no = (uint32_t)(q * nxy + own) * TB;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) *boff(C_out + (base + kk) * N, no) = cn[kk];
        if (!isfinite(cn[0] + cn[1] + cn[2])) st |= ST_NAN;
      }
    };

    // ---- phase Y: stage C of plane r; stress-divergence terms of plane r ------
    auto stage_c_and_divergence = [&](int r) {
      if (!visc) return;
      const int sl4 = r & 3;
#pragma unroll
      for (int k = 0; k < K2; ++k) {
        if (q1[k] >= 0) {
#pragma unroll
          for (int c = 0; c < 6; ++c) L.C[sl4][c][q1[k]] = cst[k][c];
        }
      }
      // F^P_a = sum_b [T_ab(x+e_b) - T_ab(x-e_b)]/2: the x and y terms from
      // plane r; T_az(r) enters the node above with + and the node below
      // with -
      const int c2 = c2of1;
      const T dx0 = T(0.5) * (L.stress[0][c2 + 1] - L.stress[0][c2 - 1]);
      const T dx1 = T(0.5) * (L.stress[3][c2 + 1] - L.stress[3][c2 - 1]);
      const T dx2 = T(0.5) * (L.stress[4][c2 + 1] - L.stress[4][c2 - 1]);
      const T dy0 = T(0.5) * (L.stress[3][c2 + HX2] - L.stress[3][c2 - HX2]);
      const T dy1 = T(0.5) * (L.stress[1][c2 + HX2] - L.stress[1][c2 - HX2]);
      const T dy2 = T(0.5) * (L.stress[5][c2 + HX2] - L.stress[5][c2 - HX2]);
      acc[1][0] += dx0 + dy0;
      acc[1][1] += dx1 + dy1;
      acc[1][2] += dx2 + dy2;
      const T z0h = T(0.5) * L.stress[4][c2], z1h = T(0.5) * L.stress[5][c2];
      const T z2h = T(0.5) * L.stress[2][c2];
      acc[0][0] += z0h; acc[0][1] += z1h; acc[0][2] += z2h;
      acc[2][0] -= z0h; acc[2][1] -= z1h; acc[2][2] -= z2h;
    };

    // ---- phase Y: plane m = r-1 of the 1-frame: forces, velocity shift,
    // records, moments, u
    auto finalise = [&](int m) {
      const int sm = (m + 3) % 3, smm = (m + 2) % 3, smp = (m + 4) % 3;
      const int c2 = c2of1;
      const T rA = L.rho[sm][0][c2], rB = L.rho[sm][1][c2];
      // Shan-Chen: F_A = -G rho_A sum_i 3 w_i rho_B(x+c_i) c_i (and A<->B)
      T sA[3] = {T(0), T(0), T(0)}, sB[3] = {T(0), T(0), T(0)};
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int sl = CZ[i] == 0 ? sm : (CZ[i] > 0 ? smp : smm);
        const int nb = c2 + CY[i] * HX2 + CX[i];
        const T nA = L.rho[sl][0][nb], nB = L.rho[sl][1][nb];
        const T wt = T(3) * wgt<T>(i);
        if (CX[i] != 0) { sA[0] += (wt * T(CX[i])) * nB; sB[0] += (wt * T(CX[i])) * nA; }
        if (CY[i] != 0) { sA[1] += (wt * T(CY[i])) * nB; sB[1] += (wt * T(CY[i])) * nA; }
        if (CZ[i] != 0) { sA[2] += (wt * T(CZ[i])) * nB; sB[2] += (wt * T(CZ[i])) * nA; }
      }
      T FA[3], FB[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        FA[c] = -G * rA * sA[c];
        FB[c] = -G * rB * sB[c];
      }
      const T irt = rcpT(rA + rB);
      if (visc) {
        // polymer force split over the components by mass fraction
        const T fa = rA * irt, fb = rB * irt;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          FA[c] = FA[c] + fa * acc[0][c];
          FB[c] = FB[c] + fb * acc[0][c];
        }
      }
      // velocity shift u' = sum(j_s/tau_s)/sum(rho_s/tau_s),
      // u^eq_s = u' + tau_s F_s/rho_s, with the momentum's rate tau^-
      const T iden = rcpT(rA * itmA + rB * itmB);
      const T qA = tmA * rcpT(rA), qB = tmB * rcpT(rB);
      T ueA[3], ueB[3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T up = (jv[c] * itmA + jv[3 + c] * itmB) * iden;
        ueA[c] = up + qA * FA[c];
        ueB[c] = up + qB * FB[c];
      }
      if (has1) {
#pragma unroll
        for (int cp = 0; cp < 2; ++cp) {
          const T rs = cp ? rB : rA;
          const T* ue = cp ? ueB : ueA;
          const T w = cp ? itB : itA, wm = cp ? itmB : itmA;
          const T wr = w * rs, wmr = wm * rs, wm1 = T(1) - wm;
          const T usq = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
          V4<T> r0, r1;
          r0.x = rs - T(1.5) * wr * usq;
          r0.y = wmr * ue[0] + wm1 * jv[3 * cp];
          r0.z = wmr * ue[1] + wm1 * jv[3 * cp + 1];
          r0.w = wmr * ue[2] + wm1 * jv[3 * cp + 2];
          r1.x = ue[0]; r1.y = ue[1]; r1.z = ue[2];
          r1.w = T(4.5) * wr;
          L.rec[sm][cp][0][e1] = r0;
          L.rec[sm][cp][1][e1] = r1;
        }
        if (inner) {
          const int s2 = m & 1;
          L.M[s2][0][0][mcol] = rA;
          L.M[s2][1][0][mcol] = rB;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            L.M[s2][0][1 + c][mcol] = jv[c];
            L.M[s2][1][1 + c][mcol] = jv[3 + c];
          }
        }
        if (visc) {
          // physical velocity u = (j_A + j_B + (F_A + F_B)/2)/rho
#pragma unroll
          for (int c = 0; c < 3; ++c)
            L.u[sm][c][e1] = (jv[c] + jv[3 + c] + T(0.5) * (FA[c] + FB[c])) * irt;
        }
      }
    };
    auto shift_acc = [&]() {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        acc[0][c] = acc[1][c];
        acc[1][c] = acc[2][c];
        acc[2][c] = T(0);
      }
    };

    const int z0 = tl.z0, zend = tl.z1;
    load_raw(z0 - 2);
    load_j(z0 - 3);
    load_pops(clampz(z0 - 4, nz), std::integral_constant<int, 0>{}, std::integral_constant<int, Q>{});
    for (int r = z0 - 2; r <= zend + 2; ++r) {
      __syncthreads();   // (1) readers of the previous iteration are done
      ingest(r);
      // loads for the next iterations; past the lattice or the tile they
      // re-read clamped planes (in bounds, unused), so every load issues
      // unconditionally
      load_raw(r + 1);
      const int q = r - 3;
      const bool ok = q >= z0 && q < zend && active;
      collide(q, ok);
      if (visc) {
        if (s) fene(q, std::integral_constant<int, 1>{}, ok);
        else fene(q, std::integral_constant<int, 0>{}, ok);
      }
      // the next plane's populations load in two parts, one on each side of
      // the barrier, and the moments and C are stored after it: the memory
      // requests spread over the iteration (measured faster in FP32 and
      // FP64; with FP16 storage the loads stay in phase X and the moments
      // and C are stored where they are computed)
      load_pops(clampz(r - 2, nz), std::integral_constant<int, 0>{},
                std::integral_constant<int, kPopsEarly>{});
      __syncthreads();   // (2) plane r staged, plane r-3 collided
      if (kMomentsLate && ok) store_moments(q, true);
      load_pops(clampz(r - 2, nz), std::integral_constant<int, kPopsEarly>{},
                std::integral_constant<int, Q>{});
      stage_c_and_divergence(r);
      const int m = r - 1;
      if (m >= z0 - 1 && m <= zend && m >= 0 && m < nz) finalise(m);
      shift_acc();
      load_j(r);
#pragma unroll
      for (int i = 0; i < Q; ++i) asm volatile("" ::"v"(held_s[i]));
#pragma unroll
      for (int i = Q; i < Q + 4; ++i) asm volatile("" ::"v"(held[i]));
      if (visc) {
#pragma unroll
        for (int i = Q + 4; i < Q + 7; ++i) asm volatile("" ::"v"(held[i]));
      }
    }
    if (st) atomicOr(a.P.status + tl.run, st);
  }
}

// ---- physical velocity (observe, export) ------------------------------------------
// u = (j_A + j_B + (F_A + F_B)/2)/rho at every node of every run, with the
// forces of the step: Shan-Chen from the 18 neighbours' densities (mirror
// ghost in z) and the polymer force as the centred divergence of T over the
// six face neighbours (zero-gradient ghost in z).  One thread per node,
// plain global loads: this runs only when the velocity is observed.
template <typename T>
__device__ __forceinline__ void stress_at(const T* rho, const T* C, int64_t N, int64_t m,
                                          const RunDev& R, T (&out)[6]) {
  const T rA = rho[m], rB = rho[N + m];
  const T rp = R.visc == 0 ? rA : rB;
  T chi = (rp / (rA + rB) - T(R.chi_lo)) * T(R.inv_chi_range);
  chi = chi < T(0) ? T(0) : (chi > T(1) ? T(1) : chi);
  const double tr = (double)C[m] + (double)C[N + m] + (double)C[2 * N + m];
  const T fP = (T)((R.L2 - 3.0) / (R.L2 - tr));
  const T coef = chi * T(R.etaP_over_tauP);
#pragma unroll
  for (int c = 0; c < 6; ++c) out[c] = coef * (fP * C[c * N + m] - (c < 3 ? T(1) : T(0)));
}

template <typename T, typename S>
__global__ void __launch_bounds__(AUX_THREADS) k_flow(AuxArgs<T, S> a) {
  const int r = blockIdx.y;
  const RunDev& R = a.runs[r];
  const int par = a.use_parity ? (R.base & 1) : 0;
  const int64_t N = R.ld;
  const int64_t chunk = (R.n + gridDim.x - 1) / gridDim.x;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < R.n ? beg + chunk : R.n;
  const T* rho = a.P.rho[par] + 2 * R.off;
  const T* J = a.P.j[par] + 6 * R.off;
  const T* C = a.P.C[R.visc >= 0 ? par : 0] + 6 * R.off;
  T* U = a.P.u + 3 * R.off;
  const int nx = R.nx, ny = R.ny, nz = R.nz;
  const T G = T(R.G), itA = T(R.inv_tau[0]), itB = T(R.inv_tau[1]);
  (void)itA; (void)itB;
  for (int64_t n = beg + threadIdx.x; n < end; n += blockDim.x) {
    const int x = (int)(n % nx), y = (int)((n / nx) % ny), z = (int)(n / ((int64_t)nx * ny));
    auto node = [&](int dx, int dy, int dz) -> int64_t {
      return ((int64_t)clampz(z + dz, nz) * ny + wrapm(y + dy, ny)) * nx + wrapm(x + dx, nx);
    };
    const T rA = rho[n], rB = rho[N + n];
    T sA[3] = {0, 0, 0}, sB[3] = {0, 0, 0};
#pragma unroll
    for (int i = 1; i < Q; ++i) {
      const int64_t m = node(CX[i], CY[i], CZ[i]);
      const T nA = rho[m], nB = rho[N + m];
      const T wt = T(3) * wgt<T>(i);
      if (CX[i] != 0) { sA[0] += (wt * T(CX[i])) * nB; sB[0] += (wt * T(CX[i])) * nA; }
      if (CY[i] != 0) { sA[1] += (wt * T(CY[i])) * nB; sB[1] += (wt * T(CY[i])) * nA; }
      if (CZ[i] != 0) { sA[2] += (wt * T(CZ[i])) * nB; sB[2] += (wt * T(CZ[i])) * nA; }
    }
    T F[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) F[c] = -G * rA * sA[c] - G * rB * sB[c];
    if (R.visc >= 0) {
      // F^P_a = sum_b [T_ab(x+e_b) - T_ab(x-e_b)]/2 (total over components)
      constexpr int SYM[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
      T P[3] = {0, 0, 0};
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        T tp[6], tm[6];
        stress_at(rho, C, N, node(bb == 0, bb == 1, bb == 2), R, tp);
        stress_at(rho, C, N, node(-(bb == 0), -(bb == 1), -(bb == 2)), R, tm);
#pragma unroll
        for (int c = 0; c < 3; ++c) P[c] += T(0.5) * (tp[SYM[c][bb]] - tm[SYM[c][bb]]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) F[c] += P[c];
    }
    const T irt = T(1) / (rA + rB);
#pragma unroll
    for (int c = 0; c < 3; ++c) U[c * N + n] = (J[c * N + n] + J[(3 + c) * N + n] + T(0.5) * F[c]) * irt;
  }
}

// ---- host launchers ------------------------------------------------------------------
bool step_shape_ok(int bx, int by, bool fp64) {
#define SHAPE_OK(BX, BY) \
  if (bx == BX && by == BY) return fp64 ? step_fits<BX, BY, double>() : step_fits<BX, BY, float>();
  LBM_FOR_SHAPES(SHAPE_OK)
#undef SHAPE_OK
  return false;
}

template <typename T, typename S, int BX, int BY>
void launch_step_shape(const StepArgs<T, S>& a, dim3 grid, hipStream_t st) {
  if constexpr (step_fits<BX, BY, T>()) {
    const dim3 blk(BX, BY, 2);
    if (a.trt) {
      if (a.wide) k_step<T, S, BX, BY, DG_WIDE, true><<<grid, blk, 0, st>>>(a);
      else k_step<T, S, BX, BY, Q, true><<<grid, blk, 0, st>>>(a);
    } else {
      if (a.wide) k_step<T, S, BX, BY, DG_WIDE, false><<<grid, blk, 0, st>>>(a);
      else k_step<T, S, BX, BY, Q, false><<<grid, blk, 0, st>>>(a);
    }
  }
}

template <typename T, typename S>
void launch_step(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
#define STEP_CASE(BX, BY) \
  else if (block.x == BX && block.y == BY) launch_step_shape<T, S, BX, BY>(a, grid, s);
  if (false) {}
  LBM_FOR_SHAPES(STEP_CASE)
#undef STEP_CASE
}

// Workgroups of the step kernel that one CU holds at once (LDS, registers).
template <typename T, typename S>
int step_blocks_per_cu(int bx, int by, bool wide, bool trt) {
  int n = 0;
  auto occ = [&](auto kern, int threads) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kern, threads, 0) != hipSuccess) n = 0;
  };
#define STEP_OCC(BX, BY)                                                            \
  if (bx == BX && by == BY) {                                                       \
    if constexpr (step_fits<BX, BY, T>()) {                                         \
      if (trt) {                                                                    \
        if (wide) occ(k_step<T, S, BX, BY, DG_WIDE, true>, 2 * BX * BY);            \
        else occ(k_step<T, S, BX, BY, Q, true>, 2 * BX * BY);                       \
      } else {                                                                      \
        if (wide) occ(k_step<T, S, BX, BY, DG_WIDE, false>, 2 * BX * BY);           \
        else occ(k_step<T, S, BX, BY, Q, false>, 2 * BX * BY);                      \
      }                                                                             \
    }                                                                               \
  }
  LBM_FOR_SHAPES(STEP_OCC)
#undef STEP_OCC
  return n;
}

template <typename T, typename S>
void launch_flow(const AuxArgs<T, S>& a, hipStream_t s) {
  k_flow<T, S><<<dim3(AUX_BLOCKS, a.nruns), AUX_THREADS, 0, s>>>(a);
}

#define LBM_INST(T, S)                                                                  \
  template void launch_step<T, S>(const StepArgs<T, S>&, dim3, dim3, hipStream_t);     \
  template int step_blocks_per_cu<T, S>(int, int, bool, bool);                          \
  template void launch_flow<T, S>(const AuxArgs<T, S>&, hipStream_t);
LBM_INST(double, double)
LBM_INST(float, float)
LBM_INST(float, __half)
#undef LBM_INST

}  // namespace lbm
