// Step kernels of the hybrid LB / FENE-P solver (gfx950).
//
// One time step n -> n+1 is three launches over the tile table:
//
//   force pass    (per node): Shan-Chen force from the densities of the 18
//                 neighbours (mirror ghost in z), polymer force as the centred
//                 divergence of T = chi (eta_P/tau_P)(f C - I) over the six
//                 face neighbours, then the Shan-Chen velocity shift
//                 u' = sum(j_s/tau_s)/sum(rho_s/tau_s), u^eq_s = u' + tau_s F_s/rho_s
//                 and the physical velocity u = (j_A + j_B + (F_A+F_B)/2)/rho.
//                 Writes (rho_s, u^eq_s) per component and u.
//   collide pass  (per node and component): pull streaming -- each population
//                 arriving at x is the BGK post-collision value
//                 f_i - (f_i - f^eq_i)/tau_s of the source node x - c_i,
//                 computed on the fly from that node's (rho_s, u^eq_s); links
//                 that cross a wall are replaced by the half-way bounce-back
//                 of the node's own outgoing population with the moving-wall
//                 term -6 w_i rho_s c_i.u_wall.  The new density and momentum
//                 of the component at x are summed from the values written.
//                 Populations are held as g_i = f_i - w_i rho_s(node) (see
//                 Store), and the collision is done in that variable.
//   FENE-P pass   (per node, viscoelastic runs only): explicit Euler step of
//                 C with u^n and C^n of the six face neighbours (first-order
//                 upwind advection, centred grad u, Peterlin factor in FP64).
//
// The model is Section 2 of the paper (Eqs. (1)-(4), Peterlin factor below
// Eq. (2)); the set-up (walls at +-U_w, periodic x and y) is Section 3.
// Every pass reads the state at parity (base + step) & 1; the collide and
// FENE-P passes write the other parity, so no node reads a value written in
// the same pass.  A node's arithmetic does not depend on the tile shape or on
// the other runs of a batch, so every launch shape and batch composition is
// bit-identical.
#include "lbm_internal.h"

namespace lbm {

// Equilibrium minus its rest part, f^eq_i - w_i rho (the shifted
// equilibrium), times a power-of-two storage scale folded into the weight.
template <typename T>
__device__ __forceinline__ T geq(int i, T rho, T ux, T uy, T uz, T scale) {
  const T cu = T(CX[i]) * ux + T(CY[i]) * uy + T(CZ[i]) * uz;
  const T usq = ux * ux + uy * uy + uz * uz;
  return (wgt<T>(i) * scale) * rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
}

__device__ __forceinline__ int64_t nid(int x, int y, int z, int nx, int ny) {
  return ((int64_t)z * ny + y) * nx + x;
}

// Optional occupancy target of the collide pass (waves per SIMD), a build
// option: the register budget then shrinks to 512 / waves.
#ifdef LBM_COLLIDE_WAVES
#define LBM_COLLIDE_OCC __attribute__((amdgpu_waves_per_eu(LBM_COLLIDE_WAVES)))
#else
#define LBM_COLLIDE_OCC
#endif

// Planes held in the LDS rings of the force and FENE-P passes.  Three (the
// minimum for a radius-1 stencil in z) take a second barrier per plane before
// a slot is overwritten; four need one barrier but 4/3 the LDS, which limits
// the workgroups per CU.
#ifndef LBM_RING_SLOTS
#define LBM_RING_SLOTS 3
#endif
constexpr int RS = LBM_RING_SLOTS;
static_assert(RS == 3 || RS == 4, "ring of 3 or 4 planes");
// ring slot of plane zp >= -1
__device__ __forceinline__ int rslot(int zp) { return RS == 4 ? (zp & 3) : (zp + 3) % 3; }

// Shapes of the tile (bx, by) with a compiled instance of every pass.
#define LBM_FOR_SHAPES(M) M(64, 4) M(32, 8) M(128, 2) M(64, 2) M(32, 4)

// ---- force pass ----------------------------------------------------------------
// One workgroup marches up the z range of a bx*by tile.  The densities (and,
// for a viscoelastic run, the polymer stress T computed once per node) of
// planes z-1, z, z+1 of the tile plus a one-node halo live in an LDS ring;
// the raw values of plane z+2 are loaded into registers while plane z is
// computed.  Ghost planes beyond the walls repeat the boundary plane (mirror
// density, zero-gradient C, hence the same T).
template <typename T, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX * BY) k_force(StepArgs<T, S> a) {
  constexpr int HX = BX + 2, HY = BY + 2, HN = HX * HY, NT = BX * BY;
  constexpr int KP = (HN + NT - 1) / NT;
  __shared__ T srho[RS][2][HN];
  __shared__ T sT[RS][6][HN];
  const int g = *a.gstep;
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y, tid = ty * BX + tx;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool active = x < nx && y < ny;
    const bool visc = R.visc >= 0;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const T* __restrict__ rho = a.P.rho[par] + 2 * R.off;
    const T* __restrict__ J = a.P.j[par] + 6 * R.off;
    const T* __restrict__ C = a.P.C[par] + 6 * R.off;
    V4<T>* __restrict__ recA = a.P.recA + R.off;
    V4<T>* __restrict__ recB = a.P.recB + R.off;
    T* __restrict__ U = a.P.u + 3 * R.off;
    // run parameters in registers: a load of them inside the z-march would
    // wait for every load in flight (the prefetched planes) as well
    const T G = T(R.G);
    const T tA = T(R.tau[0]), tB = T(R.tau[1]);
    const T itA = T(R.inv_tau[0]), itB = T(R.inv_tau[1]);
    const int vph = R.visc;
    const T chi_lo = T(R.chi_lo), ichr = T(R.inv_chi_range), eP = T(R.etaP_over_tauP);
    const double L2 = R.L2;
    T raw[KP][8];
    auto load_raw = [&](int zp) {
      const int zc = zp < 0 ? 0 : (zp >= nz ? nz - 1 : zp);
#pragma unroll
      for (int kk = 0; kk < KP; ++kk) {
        const int k = tid + kk * NT;
        if (k < HN) {
          int gx = (tl.x0 + k % HX - 1) % nx;
          int gy = (tl.y0 + k / HX - 1) % ny;
          gx += gx < 0 ? nx : 0;
          gy += gy < 0 ? ny : 0;
          const int64_t m = nid(gx, gy, zc, nx, ny);
          raw[kk][0] = rho[m];
          raw[kk][1] = rho[N + m];
          if (visc) {
#pragma unroll
            for (int c = 0; c < 6; ++c) raw[kk][2 + c] = C[c * N + m];
          }
        }
      }
    };
    // T = chi (eta_P/tau_P)(f C - I): chi the clamped rescaled mass fraction
    // of the polymer phase's component, f the Peterlin factor in FP64
    auto store_raw = [&](int zp) {
      const int sl = rslot(zp);
#pragma unroll
      for (int kk = 0; kk < KP; ++kk) {
        const int k = tid + kk * NT;
        if (k < HN) {
          const T rA = raw[kk][0], rB = raw[kk][1];
          srho[sl][0][k] = rA;
          srho[sl][1][k] = rB;
          if (visc) {
            const T rp = vph == 0 ? rA : rB;
            T chi = (rp / (rA + rB) - chi_lo) * ichr;
            chi = chi < T(0) ? T(0) : (chi > T(1) ? T(1) : chi);
            const double tr = (double)raw[kk][2] + (double)raw[kk][3] + (double)raw[kk][4];
            const T fP = (T)((L2 - 3.0) / (L2 - tr));
            const T coef = chi * eP;
#pragma unroll
            for (int c = 0; c < 6; ++c)
              sT[sl][c][k] = coef * (fP * raw[kk][2 + c] - (c < 3 ? T(1) : T(0)));
          }
        }
      }
    };
    __syncthreads();   // the previous tile's readers are done with the ring
    const int zend = min(tl.z0 + a.bz, nz);
    load_raw(tl.z0 - 1);
    store_raw(tl.z0 - 1);
    load_raw(tl.z0);
    store_raw(tl.z0);
    load_raw(tl.z0 + 1);
    const int lc = (ty + 1) * HX + (tx + 1);
    // momenta of the thread's node, one plane ahead (inactive threads of a
    // ragged tile read a valid node and discard it); the two register sets
    // alternate roles (the march is unrolled by two planes), so no copy
    // waits for loads in flight
    auto load_j = [&](int zz, T (&v)[6]) {
      const int64_t m = nid(active ? x : 0, active ? y : 0, zz, nx, ny);
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] = J[c * N + m];
    };
    auto plane = [&](int z, const T (&jc)[6], T (&jn)[6]) {
      if (RS == 3) __syncthreads();   // plane z-2's slot is free (plane z-1 done)
      store_raw(z + 1);
      // the loads of plane z+2 and of the momenta of plane z+1 stay in
      // flight while plane z is computed; past the tile's end they re-read
      // its last planes (in bounds, unused)
      load_raw(min(z + 2, zend));
      load_j(min(z + 1, zend - 1), jn);
      const int64_t n = nid(active ? x : 0, active ? y : 0, z, nx, ny);
      __syncthreads();
      if (!active) return;
      const T jA0 = jc[0], jA1 = jc[1], jA2 = jc[2], jB0 = jc[3], jB1 = jc[4], jB2 = jc[5];
      // Shan-Chen: F_A = -G rho_A sum_i 3 w_i rho_B(x+c_i) c_i (and A<->B)
      T sA0 = 0, sA1 = 0, sA2 = 0, sB0 = 0, sB1 = 0, sB2 = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int sl = rslot(z + CZ[i]);
        const int k = lc + CY[i] * HX + CX[i];
        const T nA = srho[sl][0][k], nB = srho[sl][1][k];
        const T wt = T(3) * wgt<T>(i);
        if (CX[i] != 0) { sA0 += (wt * T(CX[i])) * nB; sB0 += (wt * T(CX[i])) * nA; }
        if (CY[i] != 0) { sA1 += (wt * T(CY[i])) * nB; sB1 += (wt * T(CY[i])) * nA; }
        if (CZ[i] != 0) { sA2 += (wt * T(CZ[i])) * nB; sB2 += (wt * T(CZ[i])) * nA; }
      }
      const int s0 = rslot(z), sp = rslot(z + 1), sm = rslot(z - 1);
      const T rA = srho[s0][0][lc], rB = srho[s0][1][lc];
      const T irt = T(1) / (rA + rB);
      T FA0 = -G * rA * sA0, FA1 = -G * rA * sA1, FA2 = -G * rA * sA2;
      T FB0 = -G * rB * sB0, FB1 = -G * rB * sB1, FB2 = -G * rB * sB2;
      if (visc) {
        // F^P_a = sum_b [T_ab(x+e_b) - T_ab(x-e_b)]/2
        const T dx0 = T(0.5) * (sT[s0][0][lc + 1] - sT[s0][0][lc - 1]);
        const T dx1 = T(0.5) * (sT[s0][3][lc + 1] - sT[s0][3][lc - 1]);
        const T dx2 = T(0.5) * (sT[s0][4][lc + 1] - sT[s0][4][lc - 1]);
        const T dy0 = T(0.5) * (sT[s0][3][lc + HX] - sT[s0][3][lc - HX]);
        const T dy1 = T(0.5) * (sT[s0][1][lc + HX] - sT[s0][1][lc - HX]);
        const T dy2 = T(0.5) * (sT[s0][5][lc + HX] - sT[s0][5][lc - HX]);
        const T dz0 = T(0.5) * (sT[sp][4][lc] - sT[sm][4][lc]);
        const T dz1 = T(0.5) * (sT[sp][5][lc] - sT[sm][5][lc]);
        const T dz2 = T(0.5) * (sT[sp][2][lc] - sT[sm][2][lc]);
        T P0 = 0, P1 = 0, P2 = 0;
        P0 = ((P0 + dx0) + dy0) + dz0;
        P1 = ((P1 + dx1) + dy1) + dz1;
        P2 = ((P2 + dx2) + dy2) + dz2;
        const T fa = rA * irt, fb = rB * irt;
        FA0 = FA0 + fa * P0; FA1 = FA1 + fa * P1; FA2 = FA2 + fa * P2;
        FB0 = FB0 + fb * P0; FB1 = FB1 + fb * P1; FB2 = FB2 + fb * P2;
      }
      // one reciprocal per denominator
      const T iden = T(1) / (rA * itA + rB * itB);
      const T up0 = (jA0 * itA + jB0 * itB) * iden;
      const T up1 = (jA1 * itA + jB1 * itB) * iden;
      const T up2 = (jA2 * itA + jB2 * itB) * iden;
      const T sA = tA / rA, sB = tB / rB;
      V4<T> ra, rb;
      ra.x = rA; ra.y = up0 + sA * FA0; ra.z = up1 + sA * FA1; ra.w = up2 + sA * FA2;
      rb.x = rB; rb.y = up0 + sB * FB0; rb.z = up1 + sB * FB1; rb.w = up2 + sB * FB2;
      recA[n] = ra;
      recB[n] = rb;
      U[n] = (jA0 + jB0 + T(0.5) * (FA0 + FB0)) * irt;
      U[N + n] = (jA1 + jB1 + T(0.5) * (FA1 + FB1)) * irt;
      U[2 * N + n] = (jA2 + jB2 + T(0.5) * (FA2 + FB2)) * irt;
    };
    T ja[6], jb[6];
    load_j(tl.z0, ja);
    for (int z = tl.z0; z < zend; z += 2) {
      plane(z, ja, jb);
      if (z + 1 < zend) plane(z + 1, jb, ja);
    }
  }
}

// ---- collide + stream pass ------------------------------------------------------
// One workgroup advances one component (blockIdx.y) of a bx*by tile while it
// marches up the tile's z range.  The (rho_s, u^eq_s) records of planes z-1,
// z, z+1 of the tile plus a one-node halo are staged in LDS (a four-slot
// ring, one barrier per plane): each record is read from HBM about once
// instead of once by each of its 19 pulling neighbours.
template <typename T, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX * BY) LBM_COLLIDE_OCC k_collide(StepArgs<T, S> a) {
  constexpr int HX = BX + 2, HY = BY + 2, HN = HX * HY, NT = BX * BY;
  constexpr int KR = (HN + NT - 1) / NT;   // records staged per thread and plane
  __shared__ V4<T> ring[4][HN];
  const int g = *a.gstep;
  const int s = (int)blockIdx.y;
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y, tid = ty * BX + tx;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool active = x < nx && y < ny;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const S* __restrict__ fs = a.P.f[par] + (38 * R.off + (int64_t)s * Q * N);
    S* __restrict__ fo = a.P.f[par ^ 1] + (38 * R.off + (int64_t)s * Q * N);
    T* __restrict__ rho_out = a.P.rho[par ^ 1] + 2 * R.off + s * N;
    T* __restrict__ j_out = a.P.j[par ^ 1] + 6 * R.off + 3 * s * N;
    const V4<T>* __restrict__ rec = (s == 0 ? a.P.recA : a.P.recB) + R.off;
    // inactive threads of a ragged tile address the edge node (their loads
    // are in bounds and their values unused)
    const int xq = x < nx ? x : nx - 1, yq = y < ny ? y : ny - 1;
    const int xm = xq == 0 ? nx - 1 : xq - 1, xp = xq >= nx - 1 ? 0 : xq + 1;
    const int ym = yq == 0 ? ny - 1 : yq - 1, yp = yq >= ny - 1 ? 0 : yq + 1;
    // run parameters in registers: a load of them inside the z-march would
    // wait for the populations in flight as well
    const T uw = T(R.u_wall);
    const T it = T(R.inv_tau[s]);
    const uint32_t hstep = ((uint32_t)(R.base + g) * 2u + (uint32_t)s) * 0x85ebca77u;
    using St = Store<T, S>;
    const T kS = T(St::kScale), ikS = T(1.0 / St::kScale);
    // records of plane zp of the tile + halo (periodic in x and y), the
    // kk-th of each thread: loaded into registers ahead of the populations,
    // so that writing them to the ring waits for these loads only.  Threads
    // past the halo's end load and rewrite its last record (no branch, so
    // the loads stay where they are issued).
    static_assert(KR <= 3, "at most three records per thread and plane");
    auto rec_at = [&](int zp, int kk) -> V4<T> {
      const int k = min(tid + kk * NT, HN - 1);
      int gx = (tl.x0 + k % HX - 1) % nx;
      int gy = (tl.y0 + k / HX - 1) % ny;
      gx += gx < 0 ? nx : 0;
      gy += gy < 0 ? ny : 0;
      return rec[nid(gx, gy, zp, nx, ny)];
    };
    auto rec_put = [&](int zp, int kk, const V4<T>& v) {
      ring[zp & 3][min(tid + kk * NT, HN - 1)] = v;
    };
    // Byte offsets inside one direction array (a run's array is < 4 GiB, which
    // the library checks): the plane term is uniform, rows and columns
    // (periodic) are per thread, and the array base is uniform, so every
    // population access is a uniform base plus one 32-bit offset.
    constexpr uint32_t SB = sizeof(S);
    const uint32_t pb = (uint32_t)nx * (uint32_t)ny * SB;
    const uint32_t rowb[3] = {(uint32_t)(ym * nx) * SB, (uint32_t)(yq * nx) * SB,
                              (uint32_t)(yp * nx) * SB};
    const uint32_t colb[3] = {(uint32_t)xm * SB, (uint32_t)xq * SB, (uint32_t)xp * SB};
    auto arr = [&](const S* base, int i, uint32_t off) {
      return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base + (int64_t)i * N) + off);
    };
    // the populations that arrive at (x, y, zz): pulled from x - c_i, or the
    // node's own opposite population where the link crosses a wall
    auto load_plane = [&](int zz, T (&v)[Q]) {
      const uint32_t own = (uint32_t)zz * pb + rowb[1] + colb[1];
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        const int zs = zz - CZ[i];
        const uint32_t off = (uint32_t)zs * pb + rowb[1 - CY[i]] + colb[1 - CX[i]];
        if (CZ[i] == 0) {
          v[i] = St::load(arr(fs, i, off), 0);
        } else {
          // uniform choice between the pulled value and the wall's reflection
          // of the node's own opposite population, made by selects so that
          // the plane's loads issue back to back
          const bool in = zs >= 0 && zs < nz;
          v[i] = St::load(arr(fs, in ? i : OPPI[i], in ? off : own), 0);
        }
      }
    };
    __syncthreads();   // the previous tile's readers are done with the ring
    const int zend = min(tl.z0 + a.bz, nz);
    for (int zp = max(tl.z0 - 1, 0); zp <= tl.z0; ++zp)
      for (int kk = 0; kk < KR; ++kk) rec_put(zp, kk, rec_at(zp, kk));
    // software pipeline: the populations of plane z+1 are in flight while
    // plane z is collided; the two register sets alternate roles (the march
    // is unrolled by two planes), so no copy is made between planes.  The
    // loads are unconditional (past the tile's end they re-read its last
    // plane, past the lattice's end its top plane): a load skipped on some
    // path would make the compiler wait for all of them before plane z.
    auto plane = [&](int z, T (&cur)[Q], T (&nxt)[Q]) {
      {
        const int zr = min(z + 1, nz - 1);
        const V4<T> r0 = rec_at(zr, 0);
        const V4<T> r1 = KR > 1 ? rec_at(zr, 1) : r0;
        const V4<T> r2 = KR > 2 ? rec_at(zr, 2) : r0;
        __builtin_amdgcn_sched_barrier(0);   // the record loads issue first
        load_plane(min(z + 1, zend - 1), nxt);
        if (z + 1 < nz) {
          rec_put(z + 1, 0, r0);
          if (KR > 1) rec_put(z + 1, 1, r1);
          if (KR > 2) rec_put(z + 1, 2, r2);
        }
      }
      __syncthreads();
      if (active) {
        const int64_t n = nid(x, y, z, nx, ny);
        const uint32_t nb = (uint32_t)z * pb + rowb[1] + colb[1];   // n * sizeof(S)
        const int lc = (ty + 1) * HX + (tx + 1);
        // BGK collision of each arriving population in the shifted variable
        // of the node that holds it (the record's node in both branches),
        // g* = g - (g - g^eq)/tau, then re-referenced to the density rho_x of
        // x: h_i = g*_i + w_i (rho_src,i - rho_x) = f*_i - w_i rho_x.  The new
        // density is rho_x + sum_i h_i (sum_i w_i = 1): rho_x enters with
        // weight exactly 1 and the rounded weights (FP32 sum 1 + 1.5e-8) only
        // multiply small differences, so they do not leak into the mass.
        // Shifted values are in storage units (times kScale, a power of 2).
        const T rx = ring[z & 3][lc].x;
        T drho = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const int zs = z - CZ[i];
          if (CZ[i] == 0) {
            const V4<T> r = ring[z & 3][lc - CY[i] * HX - CX[i]];
            cur[i] = cur[i] - (cur[i] - geq<T>(i, r.x, r.y, r.z, r.w, kS)) * it;
            if (i != 0) cur[i] += (wgt<T>(i) * kS) * (r.x - rx);
          } else {
            // Links through z: the pulled value, or (where the link crosses a
            // wall) the half-way bounce-back of x's own population in
            // o = opp(i), whose equilibrium has c_o = -c_i and which gains
            // the moving-wall term -6 w rho c_o.u_wall.  The choice is uniform
            // and made by selects; the re-reference term vanishes for the
            // bounce-back (its record is x's own).
            const bool in = zs >= 0 && zs < nz;
            const int o = OPPI[i];
            const V4<T> r = ring[in ? (zs & 3) : (z & 3)][in ? lc - CY[i] * HX - CX[i] : lc];
            const T sg = in ? T(1) : T(-1);
            const T cu = sg * (T(CX[i]) * r.y + T(CY[i]) * r.z + T(CZ[i]) * r.w);
            const T usq = r.y * r.y + r.z * r.z + r.w * r.w;
            const T ge = (wgt<T>(i) * kS) * r.x * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
            const T uwall = CZ[o] > 0 ? uw : -uw;
            const T wall = in ? T(0) : ((T(6) * kS * wgt<T>(o)) * r.x) * (T(CX[o]) * uwall);
            cur[i] = cur[i] - (cur[i] - ge) * it - wall;
            cur[i] += (wgt<T>(i) * kS) * (r.x - rx);
          }
          drho += cur[i];
        }
        const T rsum = rx + drho * ikS;
        // stored: f*_i - w_i rho_x_new = h_i - w_i drho; the momentum is
        // summed from the values as stored (the rest parts cancel pairwise
        // in sum_i c_i w_i).  FP16 rounding takes 13 random bits per value:
        // a hash of (node, component, step) starts a Weyl sequence over the
        // directions (uniform for every direction, independent of the tile
        // shape and batch layout, and reproducible).
        uint32_t hb = 0;
        if (St::kRandom) hb = fmix32((uint32_t)n * 0x9e3779b1u ^ hstep);
        T jx = 0, jy = 0, jz = 0;
#pragma unroll
        for (int i = 0; i < Q; ++i) {
          const uint32_t rb = (hb + (uint32_t)i * 0x9e3779b9u) >> 19;
          const T v = cur[i] - wgt<T>(i) * drho;
          S* dst = reinterpret_cast<S*>(reinterpret_cast<char*>(fo + (int64_t)i * N) + nb);
          const T fq = St::put(dst, 0, v, rb);
          if (CX[i] != 0) jx += T(CX[i]) * fq;
          if (CY[i] != 0) jy += T(CY[i]) * fq;
          if (CZ[i] != 0) jz += T(CZ[i]) * fq;
        }
        jx *= ikS;
        jy *= ikS;
        jz *= ikS;
        rho_out[n] = rsum;
        j_out[n] = jx;
        j_out[N + n] = jy;
        j_out[2 * N + n] = jz;
        if (!isfinite(rsum + jx + jy + jz)) atomicOr(a.P.status + tl.run, ST_NAN);
      }
    };
    T va[Q], vb[Q];
    load_plane(tl.z0, va);
    for (int z = tl.z0; z < zend; z += 2) {
      plane(z, va, vb);
      if (z + 1 < zend) plane(z + 1, vb, va);
    }
  }
}

// ---- FENE-P pass -------------------------------------------------------------------
// Same z-march as the force pass: C and u of planes z-1, z, z+1 (+ halo) in an
// LDS ring, plane z+2 loaded into registers while plane z is updated.  Ghost
// planes: C zero-gradient; u extrapolated through the wall velocity,
// u(-1) = 2 u_bot - u(0), u(nz) = 2 u_top - u(nz-1), u_wall = (-+U_w, 0, 0).
template <typename T, typename S, int BX, int BY>
__global__ void __launch_bounds__(BX * BY) k_fene(StepArgs<T, S> a) {
  constexpr int HX = BX + 2, HY = BY + 2, HN = HX * HY, NT = BX * BY;
  constexpr int KP = (HN + NT - 1) / NT;
  __shared__ T sC[RS][6][HN];
  __shared__ T sU[RS][3][HN];
  const int g = *a.gstep;
  const int tx = (int)threadIdx.x, ty = (int)threadIdx.y, tid = ty * BX + tx;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target || R.visc < 0) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int x = tl.x0 + tx, y = tl.y0 + ty;
    const bool active = x < nx && y < ny;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const T* __restrict__ Cin = a.P.C[par] + 6 * R.off;
    T* __restrict__ Cout = a.P.C[par ^ 1] + 6 * R.off;
    const T* __restrict__ U = a.P.u + 3 * R.off;
    const T uw = T(R.u_wall);
    const T itP = T(R.inv_tauP);
    T raw[KP][9];
    auto load_raw = [&](int zp) {
      const int zc = zp < 0 ? 0 : (zp >= nz ? nz - 1 : zp);
#pragma unroll
      for (int kk = 0; kk < KP; ++kk) {
        const int k = tid + kk * NT;
        if (k < HN) {
          int gx = (tl.x0 + k % HX - 1) % nx;
          int gy = (tl.y0 + k / HX - 1) % ny;
          gx += gx < 0 ? nx : 0;
          gy += gy < 0 ? ny : 0;
          const int64_t m = nid(gx, gy, zc, nx, ny);
#pragma unroll
          for (int c = 0; c < 6; ++c) raw[kk][c] = Cin[c * N + m];
#pragma unroll
          for (int b = 0; b < 3; ++b) raw[kk][6 + b] = U[b * N + m];
        }
      }
    };
    auto store_raw = [&](int zp) {
      const int sl = rslot(zp);
#pragma unroll
      for (int kk = 0; kk < KP; ++kk) {
        const int k = tid + kk * NT;
        if (k < HN) {
#pragma unroll
          for (int c = 0; c < 6; ++c) sC[sl][c][k] = raw[kk][c];
          if (zp < 0) {
            sU[sl][0][k] = T(2) * (-uw) - raw[kk][6];
            sU[sl][1][k] = T(2) * T(0) - raw[kk][7];
            sU[sl][2][k] = T(2) * T(0) - raw[kk][8];
          } else if (zp >= nz) {
            sU[sl][0][k] = T(2) * uw - raw[kk][6];
            sU[sl][1][k] = T(2) * T(0) - raw[kk][7];
            sU[sl][2][k] = T(2) * T(0) - raw[kk][8];
          } else {
#pragma unroll
            for (int b = 0; b < 3; ++b) sU[sl][b][k] = raw[kk][6 + b];
          }
        }
      }
    };
    __syncthreads();   // the previous tile's readers are done with the ring
    const int zend = min(tl.z0 + a.bz, nz);
    load_raw(tl.z0 - 1);
    store_raw(tl.z0 - 1);
    load_raw(tl.z0);
    store_raw(tl.z0);
    load_raw(tl.z0 + 1);
    const int lc = (ty + 1) * HX + (tx + 1);
    uint32_t st = 0;
    for (int z = tl.z0; z < zend; ++z) {
      if (RS == 3) __syncthreads();   // plane z-2's slot is free (plane z-1 done)
      store_raw(z + 1);
      if (z + 2 <= zend) load_raw(z + 2);
      __syncthreads();
      if (!active) continue;
      const int64_t n = nid(x, y, z, nx, ny);
      const int s0 = rslot(z), sp = rslot(z + 1), sm = rslot(z - 1);
      const T u0 = sU[s0][0][lc], u1 = sU[s0][1][lc], u2 = sU[s0][2][lc];
      T Gm[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Gm[0][b] = T(0.5) * (sU[s0][b][lc + 1] - sU[s0][b][lc - 1]);
        Gm[1][b] = T(0.5) * (sU[s0][b][lc + HX] - sU[s0][b][lc - HX]);
        Gm[2][b] = T(0.5) * (sU[sp][b][lc] - sU[sm][b][lc]);
      }
      T c[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) c[k] = sC[s0][k][lc];
      const double tr = (double)c[0] + (double)c[1] + (double)c[2];
      if (tr >= R.L2) st |= ST_FENE;
      const T fP = (T)((R.L2 - 3.0) / (R.L2 - tr));
      const T ua0 = u0 > T(0) ? u0 : T(0), ub0 = u0 < T(0) ? u0 : T(0);
      const T ua1 = u1 > T(0) ? u1 : T(0), ub1 = u1 < T(0) ? u1 : T(0);
      const T ua2 = u2 > T(0) ? u2 : T(0), ub2 = u2 < T(0) ? u2 : T(0);
      constexpr int KK[6] = {0, 1, 2, 0, 0, 1};
      constexpr int LL[6] = {0, 1, 2, 1, 2, 2};
      constexpr int SYM[3][3] = {{0, 3, 4}, {3, 1, 5}, {4, 5, 2}};
      T csum = 0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const T ck = c[k];
        T adv = 0;
        adv += ua0 * (ck - sC[s0][k][lc - 1]) + ub0 * (sC[s0][k][lc + 1] - ck);
        adv += ua1 * (ck - sC[s0][k][lc - HX]) + ub1 * (sC[s0][k][lc + HX] - ck);
        adv += ua2 * (ck - sC[sm][k][lc]) + ub2 * (sC[sp][k][lc] - ck);
        T Sk = 0;
#pragma unroll
        for (int m = 0; m < 3; ++m)
          Sk += c[SYM[KK[k]][m]] * Gm[m][LL[k]] + Gm[m][KK[k]] * c[SYM[m][LL[k]]];
        const T delta = k < 3 ? T(1) : T(0);
        const T cn = ck + (-adv + Sk - (fP * ck - delta) * itP);
        Cout[k * N + n] = cn;
        csum += cn;
      }
      if (!isfinite(csum)) st |= ST_NAN;
    }
    if (st) atomicOr(a.P.status + tl.run, st);
  }
}

// ---- host launchers ------------------------------------------------------------------
template <typename T, typename S>
void launch_force(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
#define FORCE_CASE(BX, BY) \
  else if (block.x == BX && block.y == BY) k_force<T, S, BX, BY><<<grid, block, 0, s>>>(a);
  if (false) {}
  LBM_FOR_SHAPES(FORCE_CASE)
#undef FORCE_CASE
}

template <typename T, typename S>
void launch_collide(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
  const dim3 g2(grid.x, 2);
#define COLLIDE_CASE(BX, BY) \
  else if (block.x == BX && block.y == BY) k_collide<T, S, BX, BY><<<g2, block, 0, s>>>(a);
  if (false) {}
  LBM_FOR_SHAPES(COLLIDE_CASE)
#undef COLLIDE_CASE
}

template <typename T, typename S>
void launch_fene(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
  if (!a.any_visc) return;
#define FENE_CASE(BX, BY) \
  else if (block.x == BX && block.y == BY) k_fene<T, S, BX, BY><<<grid, block, 0, s>>>(a);
  if (false) {}
  LBM_FOR_SHAPES(FENE_CASE)
#undef FENE_CASE
}

#define LBM_INST(T, S)                                                                        \
  template void launch_force<T, S>(const StepArgs<T, S>&, dim3, dim3, hipStream_t);          \
  template void launch_collide<T, S>(const StepArgs<T, S>&, dim3, dim3, hipStream_t);        \
  template void launch_fene<T, S>(const StepArgs<T, S>&, dim3, dim3, hipStream_t);
LBM_INST(double, double)
LBM_INST(float, float)
LBM_INST(float, __half)
#undef LBM_INST

}  // namespace lbm
