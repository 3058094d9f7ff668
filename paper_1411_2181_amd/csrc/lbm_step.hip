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

template <typename T>
__device__ __forceinline__ T feq(int i, T rho, T ux, T uy, T uz) {
  const T cu = T(CX[i]) * ux + T(CY[i]) * uy + T(CZ[i]) * uz;
  const T usq = ux * ux + uy * uy + uz * uz;
  return wgt<T>(i) * rho * (T(1) + T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq);
}

__device__ __forceinline__ int64_t nid(int x, int y, int z, int nx, int ny) {
  return ((int64_t)z * ny + y) * nx + x;
}

// Polymer stress T_k at node k (component order xx yy zz xy xz yz).
template <typename T>
__device__ __forceinline__ void stress_at(const T* __restrict__ C, const T* __restrict__ rho,
                                          int64_t N, int64_t k, const RunDev& R, T out[6]) {
  const T rA = rho[k], rB = rho[N + k];
  const T rp = R.visc == 0 ? rA : rB;
  T chi = (rp / (rA + rB) - T(R.chi_lo)) * T(R.inv_chi_range);
  chi = chi < T(0) ? T(0) : (chi > T(1) ? T(1) : chi);
  T c[6];
#pragma unroll
  for (int m = 0; m < 6; ++m) c[m] = C[m * N + k];
  const double tr = (double)c[0] + (double)c[1] + (double)c[2];
  const T fP = (T)((R.L2 - 3.0) / (R.L2 - tr));
  const T coef = chi * T(R.etaP_over_tauP);
#pragma unroll
  for (int m = 0; m < 6; ++m) out[m] = coef * (fP * c[m] - (m < 3 ? T(1) : T(0)));
}

// ---- force pass ----------------------------------------------------------------
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_force(StepArgs<T, S> a) {
  const int g = *a.gstep;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int x = tl.x0 + (int)threadIdx.x, y = tl.y0 + (int)threadIdx.y;
    if (x >= nx || y >= ny) continue;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const T* __restrict__ rho = a.P.rho[par] + 2 * R.off;
    const T* __restrict__ J = a.P.j[par] + 6 * R.off;
    const T* __restrict__ C = a.P.C[par] + 6 * R.off;
    V4<T>* __restrict__ recA = a.P.recA + R.off;
    V4<T>* __restrict__ recB = a.P.recB + R.off;
    T* __restrict__ U = a.P.u + 3 * R.off;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const T G = T(R.G);
    const T tA = T(R.tau[0]), tB = T(R.tau[1]);
    const T itA = T(R.inv_tau[0]), itB = T(R.inv_tau[1]);
    const int zend = min(tl.z0 + a.bz, nz);
    for (int z = tl.z0; z < zend; ++z) {
      const int zm = z > 0 ? z - 1 : 0, zp = z < nz - 1 ? z + 1 : nz - 1;
      const int64_t n = nid(x, y, z, nx, ny);
      // Shan-Chen: F_A = -G rho_A sum_i 3 w_i rho_B(x+c_i) c_i (and A<->B)
      T sA0 = 0, sA1 = 0, sA2 = 0, sB0 = 0, sB1 = 0, sB2 = 0;
#pragma unroll
      for (int i = 1; i < Q; ++i) {
        const int xx = CX[i] > 0 ? xp : (CX[i] < 0 ? xm : x);
        const int yy = CY[i] > 0 ? yp : (CY[i] < 0 ? ym : y);
        const int zz = CZ[i] > 0 ? zp : (CZ[i] < 0 ? zm : z);
        const int64_t k = nid(xx, yy, zz, nx, ny);
        const T nA = rho[k], nB = rho[N + k];
        const T wt = T(3) * wgt<T>(i);
        if (CX[i] != 0) { sA0 += (wt * T(CX[i])) * nB; sB0 += (wt * T(CX[i])) * nA; }
        if (CY[i] != 0) { sA1 += (wt * T(CY[i])) * nB; sB1 += (wt * T(CY[i])) * nA; }
        if (CZ[i] != 0) { sA2 += (wt * T(CZ[i])) * nB; sB2 += (wt * T(CZ[i])) * nA; }
      }
      const T rA = rho[n], rB = rho[N + n];
      T FA0 = -G * rA * sA0, FA1 = -G * rA * sA1, FA2 = -G * rA * sA2;
      T FB0 = -G * rB * sB0, FB1 = -G * rB * sB1, FB2 = -G * rB * sB2;
      if (R.visc >= 0) {
        T tp[6], tm[6];
        T P0 = 0, P1 = 0, P2 = 0;
        // b = x
        stress_at(C, rho, N, nid(xp, y, z, nx, ny), R, tp);
        stress_at(C, rho, N, nid(xm, y, z, nx, ny), R, tm);
        const T dx0 = T(0.5) * (tp[0] - tm[0]), dx1 = T(0.5) * (tp[3] - tm[3]), dx2 = T(0.5) * (tp[4] - tm[4]);
        // b = y
        stress_at(C, rho, N, nid(x, yp, z, nx, ny), R, tp);
        stress_at(C, rho, N, nid(x, ym, z, nx, ny), R, tm);
        const T dy0 = T(0.5) * (tp[3] - tm[3]), dy1 = T(0.5) * (tp[1] - tm[1]), dy2 = T(0.5) * (tp[5] - tm[5]);
        // b = z (ghost planes repeat the boundary plane)
        stress_at(C, rho, N, nid(x, y, zp, nx, ny), R, tp);
        stress_at(C, rho, N, nid(x, y, zm, nx, ny), R, tm);
        const T dz0 = T(0.5) * (tp[4] - tm[4]), dz1 = T(0.5) * (tp[5] - tm[5]), dz2 = T(0.5) * (tp[2] - tm[2]);
        P0 = ((P0 + dx0) + dy0) + dz0;
        P1 = ((P1 + dx1) + dy1) + dz1;
        P2 = ((P2 + dx2) + dy2) + dz2;
        const T rt = rA + rB;
        const T fa = rA / rt, fb = rB / rt;
        FA0 = FA0 + fa * P0; FA1 = FA1 + fa * P1; FA2 = FA2 + fa * P2;
        FB0 = FB0 + fb * P0; FB1 = FB1 + fb * P1; FB2 = FB2 + fb * P2;
      }
      const T jA0 = J[n], jA1 = J[N + n], jA2 = J[2 * N + n];
      const T jB0 = J[3 * N + n], jB1 = J[4 * N + n], jB2 = J[5 * N + n];
      const T den = rA * itA + rB * itB;
      const T up0 = (jA0 * itA + jB0 * itB) / den;
      const T up1 = (jA1 * itA + jB1 * itB) / den;
      const T up2 = (jA2 * itA + jB2 * itB) / den;
      V4<T> ra, rb;
      ra.x = rA; ra.y = up0 + tA * FA0 / rA; ra.z = up1 + tA * FA1 / rA; ra.w = up2 + tA * FA2 / rA;
      rb.x = rB; rb.y = up0 + tB * FB0 / rB; rb.z = up1 + tB * FB1 / rB; rb.w = up2 + tB * FB2 / rB;
      recA[n] = ra;
      recB[n] = rb;
      const T rt = rA + rB;
      U[n] = (jA0 + jB0 + T(0.5) * (FA0 + FB0)) / rt;
      U[N + n] = (jA1 + jB1 + T(0.5) * (FA1 + FB1)) / rt;
      U[2 * N + n] = (jA2 + jB2 + T(0.5) * (FA2 + FB2)) / rt;
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
__global__ void __launch_bounds__(BX * BY) k_collide(StepArgs<T, S> a) {
  constexpr int HX = BX + 2, HY = BY + 2, HN = HX * HY, NT = BX * BY;
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
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x >= nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y >= ny - 1 ? 0 : y + 1;
    const T uw = T(R.u_wall);
    const T it = T(R.inv_tau[s]);
    const T r0 = T(R.rho0[s]);
    // copy plane zp of the tile + halo (periodic in x and y) into its slot;
    // positions beyond a ragged edge hold valid but unused nodes
    auto stage = [&](int zp) {
      V4<T>* __restrict__ sl = ring[zp & 3];
      for (int k = tid; k < HN; k += NT) {
        int gx = (tl.x0 + k % HX - 1) % nx;
        int gy = (tl.y0 + k / HX - 1) % ny;
        gx += gx < 0 ? nx : 0;
        gy += gy < 0 ? ny : 0;
        sl[k] = rec[nid(gx, gy, zp, nx, ny)];
      }
    };
    __syncthreads();   // the previous tile's readers are done with the ring
    const int zend = min(tl.z0 + a.bz, nz);
    if (tl.z0 > 0) stage(tl.z0 - 1);
    stage(tl.z0);
    for (int z = tl.z0; z < zend; ++z) {
      if (z + 1 < nz) stage(z + 1);
      __syncthreads();
      if (!active) continue;
      const int64_t n = nid(x, y, z, nx, ny);
      const int lc = (ty + 1) * HX + (tx + 1);
      T rsum = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
      for (int i = 0; i < Q; ++i) {
        T fpost;
        const int zs = z - CZ[i];
        if (CZ[i] == 0 || (zs >= 0 && zs < nz)) {
          const int xs = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
          const int ys = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
          const T fi = Store<T, S>::load(fs + (int64_t)i * N, nid(xs, ys, zs, nx, ny), wgt<T>(i) * r0);
          const V4<T> r = ring[zs & 3][lc - CY[i] * HX - CX[i]];
          fpost = fi - (fi - feq<T>(i, r.x, r.y, r.z, r.w)) * it;
        } else {
          // half-way bounce-back: the population that left x in direction
          // opp(i) is reflected by the wall it crossed
          const int o = OPPI[i];
          const T fv = Store<T, S>::load(fs + (int64_t)o * N, n, wgt<T>(o) * r0);
          const V4<T> r = ring[z & 3][lc];
          const T uwall = CZ[o] > 0 ? uw : -uw;
          fpost = fv - (fv - feq<T>(o, r.x, r.y, r.z, r.w)) * it
                  - ((T(6) * wgt<T>(o)) * r.x) * (T(CX[o]) * uwall);
        }
        Store<T, S>::store(fo + (int64_t)i * N, n, fpost, wgt<T>(i) * r0);
        // moments of the value as stored (FP16S re-reads its rounding)
        const T fq = Store<T, S>::roundtrip(fpost, wgt<T>(i) * r0);
        rsum += fq;
        if (CX[i] != 0) jx += T(CX[i]) * fq;
        if (CY[i] != 0) jy += T(CY[i]) * fq;
        if (CZ[i] != 0) jz += T(CZ[i]) * fq;
      }
      rho_out[n] = rsum;
      j_out[n] = jx;
      j_out[N + n] = jy;
      j_out[2 * N + n] = jz;
      if (!isfinite(rsum + jx + jy + jz)) atomicOr(a.P.status + tl.run, ST_NAN);
    }
  }
}

// ---- FENE-P pass -------------------------------------------------------------------
template <typename T, typename S>
__global__ void __launch_bounds__(256) k_fene(StepArgs<T, S> a) {
  const int g = *a.gstep;
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    if (tl.run < 0) continue;
    const RunDev& R = a.runs[tl.run];
    if (g >= R.target || R.visc < 0) continue;
    const int par = (R.base + g) & 1;
    const int nx = R.nx, ny = R.ny, nz = R.nz;
    const int x = tl.x0 + (int)threadIdx.x, y = tl.y0 + (int)threadIdx.y;
    if (x >= nx || y >= ny) continue;
    const int64_t N = R.ld;   // stride between the component arrays of a field
    const T* __restrict__ Cin = a.P.C[par] + 6 * R.off;
    T* __restrict__ Cout = a.P.C[par ^ 1] + 6 * R.off;
    const T* __restrict__ U = a.P.u + 3 * R.off;
    const int xm = x == 0 ? nx - 1 : x - 1, xp = x == nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? ny - 1 : y - 1, yp = y == ny - 1 ? 0 : y + 1;
    const T uw = T(R.u_wall);
    const T itP = T(R.inv_tauP);
    const int zend = min(tl.z0 + a.bz, nz);
    uint32_t st = 0;
    for (int z = tl.z0; z < zend; ++z) {
      const int64_t n = nid(x, y, z, nx, ny);
      const int zm = z > 0 ? z - 1 : 0, zp = z < nz - 1 ? z + 1 : nz - 1;
      const int64_t nxm = nid(xm, y, z, nx, ny), nxp = nid(xp, y, z, nx, ny);
      const int64_t nym = nid(x, ym, z, nx, ny), nyp = nid(x, yp, z, nx, ny);
      const int64_t nzm = nid(x, y, zm, nx, ny), nzp = nid(x, y, zp, nx, ny);
      const T u0 = U[n], u1 = U[N + n], u2 = U[2 * N + n];
      // velocity of the face neighbours; beyond a wall the ghost value
      // extrapolates linearly through the wall velocity (+-U_w, 0, 0)
      T uzp[3], uzm[3];
      if (z < nz - 1) { uzp[0] = U[nzp]; uzp[1] = U[N + nzp]; uzp[2] = U[2 * N + nzp]; }
      else { uzp[0] = T(2) * uw - u0; uzp[1] = T(2) * T(0) - u1; uzp[2] = T(2) * T(0) - u2; }
      if (z > 0) { uzm[0] = U[nzm]; uzm[1] = U[N + nzm]; uzm[2] = U[2 * N + nzm]; }
      else { uzm[0] = T(2) * (-uw) - u0; uzm[1] = T(2) * T(0) - u1; uzm[2] = T(2) * T(0) - u2; }
      T Gm[3][3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Gm[0][b] = T(0.5) * (U[b * N + nxp] - U[b * N + nxm]);
        Gm[1][b] = T(0.5) * (U[b * N + nyp] - U[b * N + nym]);
        Gm[2][b] = T(0.5) * (uzp[b] - uzm[b]);
      }
      T c[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) c[k] = Cin[k * N + n];
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
        adv += ua0 * (ck - Cin[k * N + nxm]) + ub0 * (Cin[k * N + nxp] - ck);
        adv += ua1 * (ck - Cin[k * N + nym]) + ub1 * (Cin[k * N + nyp] - ck);
        adv += ua2 * (ck - Cin[k * N + nzm]) + ub2 * (Cin[k * N + nzp] - ck);
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
  k_force<T, S><<<grid, block, 0, s>>>(a);
}

template <typename T, typename S>
void launch_collide(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
  const dim3 g2(grid.x, 2);
  if (block.x == 64 && block.y == 4) k_collide<T, S, 64, 4><<<g2, block, 0, s>>>(a);
  else if (block.x == 32 && block.y == 8) k_collide<T, S, 32, 8><<<g2, block, 0, s>>>(a);
  else if (block.x == 128 && block.y == 2) k_collide<T, S, 128, 2><<<g2, block, 0, s>>>(a);
  else if (block.x == 64 && block.y == 2) k_collide<T, S, 64, 2><<<g2, block, 0, s>>>(a);
  else if (block.x == 32 && block.y == 4) k_collide<T, S, 32, 4><<<g2, block, 0, s>>>(a);
}

template <typename T, typename S>
void launch_fene(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s) {
  if (a.any_visc) k_fene<T, S><<<grid, block, 0, s>>>(a);
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
