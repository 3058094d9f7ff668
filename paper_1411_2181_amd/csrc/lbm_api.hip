// Host side of the lbmve C ABI: parameter validation, workspace layout,
// tile tables, HIP-graph step replays, observables, export / import.
//
// A single run is a batch of one: every entry point below drives the same
// tile-table kernels, so a run advanced alone and the same run advanced
// inside any batch produce bit-identical fields.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <new>
#include <vector>

#include "../../include/lbmve.h"
#include "lbm_internal.h"

using lbm::RunDev;
using lbm::Tile;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_TARGETS = 64;
constexpr int GRAPH_CHUNKS[4] = {64, 16, 4, 1};

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

struct Targets {
  int32_t target[MAX_TARGETS];
  int32_t base[MAX_TARGETS];
};

__global__ void k_set_targets(RunDev* runs, int32_t first, int32_t count, Targets t, int32_t* gstep) {
  const int i = threadIdx.x;
  if (i < count) {
    runs[first + i].target = t.target[i];
    runs[first + i].base = t.base[i];
  }
  if (i == 0 && first == 0) *gstep = 0;
}

// Mean-field coexistence mass fractions of the symmetric Shan-Chen mixture
// (psi = rho, unit-sum interaction weights): atanh(m) = (3/2) G rho_tot m;
// returns false when G rho_tot <= 2/3 (no demixing).
bool coexistence(double G, double rho_tot, double* lo, double* hi) {
  const double k = 1.5 * G * rho_tot;
  if (k <= 1.0) return false;
  double a = 0.0, b = 1.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (a + b);
    if (mid <= 0.0 || mid >= 1.0) break;
    if (std::atanh(mid) - k * mid > 0.0) b = mid; else a = mid;
  }
  const double m = 0.5 * (a + b);
  *lo = 0.5 * (1.0 - m);
  *hi = 0.5 * (1.0 + m);
  return true;
}

struct Layout {
  size_t f[2], rho[2], j[2], C[2], u, labels, counts, status, ncomp, pieces, gstep,
      runs, tiles, partials, obs, rc, rinit, total;
  int64_t tiles_cap;
};

// Stride between the component arrays of one run's field: the node count
// rounded up to 64 and offset by 96 more, so that arrays of a power-of-two
// lattice do not start at the same HBM channel.
int64_t ld_of(int64_t n) { return (n + 63) / 64 * 64 + 96; }

size_t elem_S(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }
size_t elem_T(int prec) { return prec == LBM_FP64 ? 8 : 4; }

int64_t max_tiles(const lbm_params* p, int32_t nruns) {
  // bound for every tile shape: bx >= 8, by >= 8, bz >= 1
  int64_t t = 0;
  for (int r = 0; r < nruns; ++r) t += (int64_t)((p[r].nx + 7) / 8) * ((p[r].ny + 7) / 8) * p[r].nz;
  // tiles have at least 128 columns (half the bound) and each round of the
  // table may add up to 7 padding entries: twice the tile count covers both
  return (t + 7) / 8 * 8 + 64;
}

Layout make_layout(const lbm_params* p, int32_t nruns) {
  Layout L{};
  int64_t nodes = 0;   // padded: sum of the runs' array strides
  for (int r = 0; r < nruns; ++r) nodes += ld_of((int64_t)p[r].nx * p[r].ny * p[r].nz);
  const int prec = p[0].precision;
  const size_t s = elem_S(prec), t = elem_T(prec);
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off = align_up(off + bytes); return o; };
  for (int b = 0; b < 2; ++b) L.f[b] = take((size_t)nodes * 38 * s);
  for (int b = 0; b < 2; ++b) L.rho[b] = take((size_t)nodes * 2 * t);
  for (int b = 0; b < 2; ++b) L.j[b] = take((size_t)nodes * 6 * t);
  for (int b = 0; b < 2; ++b) L.C[b] = take((size_t)nodes * 6 * t);
  L.u = take((size_t)nodes * 3 * t);
  L.labels = take((size_t)nodes * 4);
  L.counts = take((size_t)nodes * 4);
  L.status = take((size_t)nruns * 4);
  L.ncomp = take((size_t)nruns * 4);
  L.pieces = take((size_t)nruns * lbm::MAX_PIECES * 4);
  L.gstep = take(4);
  L.runs = take((size_t)nruns * sizeof(RunDev));
  L.tiles_cap = max_tiles(p, nruns);
  L.tiles = take((size_t)L.tiles_cap * sizeof(Tile));
  L.partials = take((size_t)nruns * lbm::AUX_BLOCKS * lbm::NOBS * 8);
  L.obs = take((size_t)nruns * lbm::NOBS * 8);
  L.rc = take((size_t)nruns * 4 * 8);
  L.rinit = take((size_t)nruns * 4 * 8);
  L.total = off;
  return L;
}

}  // namespace

struct lbm_ctx {
  int32_t nruns = 0, prec = 0;
  hipStream_t stream = nullptr;
  hipStream_t cap = nullptr;    // private stream used only to capture graphs
  std::vector<lbm_params> prm;
  std::vector<RunDev> runs;
  std::vector<int64_t> done;
  char* ws = nullptr;
  Layout L{};
  lbm_launch launch{16, 8, 16, 0, 0};
  int64_t ntiles = 0;          // entries of the (XCD-permuted) tile table
  int32_t n_cu = 256;          // compute units of the device
  std::map<int, hipGraphExec_t> graphs;
  std::map<int, hipGraph_t> graph_src;

  template <typename P>
  P* at(size_t o) const { return reinterpret_cast<P*>(ws + o); }
};

namespace {

template <typename T, typename S>
lbm::Pools<T, S> pools(const lbm_ctx* c) {
  lbm::Pools<T, S> P;
  for (int b = 0; b < 2; ++b) {
    P.f[b] = c->at<S>(c->L.f[b]);
    P.rho[b] = c->at<T>(c->L.rho[b]);
    P.j[b] = c->at<T>(c->L.j[b]);
    P.C[b] = c->at<T>(c->L.C[b]);
  }
  P.u = c->at<T>(c->L.u);
  P.status = c->at<uint32_t>(c->L.status);
  return P;
}

template <typename T, typename S>
lbm::StepArgs<T, S> step_args(const lbm_ctx* c) {
  lbm::StepArgs<T, S> a;
  a.P = pools<T, S>(c);
  a.runs = c->at<RunDev>(c->L.runs);
  a.tiles = c->at<Tile>(c->L.tiles);
  a.ntiles = (int32_t)c->ntiles;
  a.gstep = c->at<int32_t>(c->L.gstep);
  a.any_visc = 0;
  a.wide = c->launch.grouped;
  a.trt = 0;
  for (const RunDev& R : c->runs) {
    a.any_visc |= R.visc >= 0;
    a.trt |= R.tau_m[0] != R.tau[0] || R.tau_m[1] != R.tau[1];
    a.wide |= (int64_t)lbm::Q * R.ld * (int64_t)sizeof(S) >= (int64_t)1 << 32;
  }
  return a;
}

template <typename T, typename S>
lbm::AuxArgs<T, S> aux_args(const lbm_ctx* c, int use_parity) {
  lbm::AuxArgs<T, S> a;
  a.P = pools<T, S>(c);
  a.runs = c->at<RunDev>(c->L.runs);
  a.nruns = c->nruns;
  a.use_parity = use_parity;
  a.partials = c->at<double>(c->L.partials);
  a.obs = c->at<double>(c->L.obs);
  a.labels = c->at<int32_t>(c->L.labels);
  a.counts = c->at<int32_t>(c->L.counts);
  a.ncomp = c->at<int32_t>(c->L.ncomp);
  a.pieces = c->at<int32_t>(c->L.pieces);
  a.radius_centre = c->at<double>(c->L.rc);
  a.rho_init = c->at<double>(c->L.rinit);
  return a;
}

// One workgroup per tile; a persistent grid is a multiple of 8 workgroups
// (one block of tiles per XCD) that loop over the tile table.
dim3 step_grid(const lbm_ctx* c) {
  int64_t g = c->ntiles;
  if (c->launch.persistent > 0) g = std::min<int64_t>(g, std::max(8, c->launch.persistent / 8 * 8));
  return dim3((unsigned)g);
}

// Dispatch on precision: F is a generic lambda taking (T*, S*) tags.
template <typename F>
void by_precision(int prec, F&& fn) {
  if (prec == LBM_FP64) fn((double*)nullptr, (double*)nullptr);
  else if (prec == LBM_FP32) fn((float*)nullptr, (float*)nullptr);
  else fn((float*)nullptr, (__half*)nullptr);
}

int hip_ok(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EHIP; }
#define HIPCHK(x) do { if ((x) != hipSuccess) return LBM_EHIP; } while (0)

int validate(const lbm_params* p) {
  if (!p) return LBM_EINVAL;
  if (p->nx < 3 || p->ny < 3 || p->nz < 3) return LBM_EINVAL;
  const int64_t n = (int64_t)p->nx * p->ny * p->nz;
  if (n >= (int64_t)1 << 31) return LBM_EINVAL;
  if (p->precision < LBM_FP64 || p->precision > LBM_FP16S) return LBM_EINVAL;
  // every per-run array (populations, densities, momenta, C) is addressed
  // with 32-bit byte offsets
  if (n * (int64_t)elem_S(p->precision) >= (int64_t)1 << 32) return LBM_EINVAL;
  if (n * (int64_t)elem_T(p->precision) >= (int64_t)1 << 32) return LBM_EINVAL;
  // the step kernel addresses DG_WIDE direction arrays from one base
  if (lbm::DG_WIDE * ld_of(n) * (int64_t)elem_S(p->precision) >= (int64_t)1 << 32) return LBM_EINVAL;
  if (!(std::fabs(p->u_wall) < 0.2)) return LBM_EINVAL;
  if (!(p->radius >= 0.0) || !(p->radius < 0.5 * p->nz)) return LBM_EINVAL;
  if (!(p->rho_major > 0.0) || !(p->rho_minor > 0.0)) return LBM_EINVAL;
  if (!(p->G >= 0.0) || !std::isfinite(p->G)) return LBM_EINVAL;
  for (int s = 0; s < 2; ++s) {
    if (!(p->tau[s] > 0.5) || !std::isfinite(p->tau[s])) return LBM_EINVAL;
    if (p->tau_minus[s] != 0.0 && (!(p->tau_minus[s] > 0.5) || !std::isfinite(p->tau_minus[s])))
      return LBM_EINVAL;
    if (!(p->eta_P[s] >= 0.0) || !std::isfinite(p->eta_P[s])) return LBM_EINVAL;
    if (p->eta_P[s] > 0.0) {
      if (!(p->tau_P[s] > 0.0) || !std::isfinite(p->tau_P[s])) return LBM_EINVAL;
      if (!(p->L2[s] > 3.0)) return LBM_EINVAL;
    }
  }
  if (p->eta_P[0] > 0.0 && p->eta_P[1] > 0.0) return LBM_EINVAL;
  if (!(p->init_noise >= 0.0 && p->init_noise < 0.1)) return LBM_EINVAL;
  if (!(p->chi_lo == 0.0 && p->chi_hi == 0.0)) {
    if (!(p->chi_hi > p->chi_lo) || !std::isfinite(p->chi_lo) || !std::isfinite(p->chi_hi))
      return LBM_EINVAL;
  }
  if (!std::isfinite(p->cx) || !std::isfinite(p->cy) || !std::isfinite(p->cz)) return LBM_EINVAL;
  return LBM_OK;
}

int validate_all(const lbm_params* runs, int32_t nruns) {
  if (!runs || nruns < 1) return LBM_EINVAL;
  for (int r = 0; r < nruns; ++r) {
    const int e = validate(runs + r);
    if (e) return e;
    if (runs[r].precision != runs[0].precision) return LBM_EINVAL;
  }
  return LBM_OK;
}

RunDev make_run(const lbm_params& p, int64_t off) {
  RunDev R{};
  R.nx = p.nx; R.ny = p.ny; R.nz = p.nz;
  R.visc = p.eta_P[0] > 0.0 ? 0 : (p.eta_P[1] > 0.0 ? 1 : -1);
  R.n = (int64_t)p.nx * p.ny * p.nz;
  R.ld = ld_of(R.n);
  R.off = off;
  R.target = 0;
  R.base = 0;
  R.u_wall = p.u_wall;
  R.G = p.G;
  for (int s = 0; s < 2; ++s) {
    R.tau[s] = p.tau[s];
    R.inv_tau[s] = 1.0 / p.tau[s];
    R.tau_m[s] = p.tau_minus[s] != 0.0 ? p.tau_minus[s] : p.tau[s];
    R.inv_tau_m[s] = 1.0 / R.tau_m[s];
  }
  if (R.visc >= 0) {
    const int v = R.visc;
    R.inv_tauP = 1.0 / p.tau_P[v];
    R.etaP_over_tauP = p.eta_P[v] / p.tau_P[v];
    R.L2 = p.L2[v];
  } else {
    R.inv_tauP = 0.0; R.etaP_over_tauP = 0.0; R.L2 = 1e300;
  }
  double lo = p.chi_lo, hi = p.chi_hi;
  if (lo == 0.0 && hi == 0.0) {
    const double rt = p.rho_major + p.rho_minor;
    if (!coexistence(p.G, rt, &lo, &hi)) { lo = p.rho_minor / rt; hi = p.rho_major / rt; }
  }
  R.chi_lo = lo;
  R.inv_chi_range = 1.0 / (hi - lo);
  // smallest droplet piece counted: 1% of the initial droplet volume
  const double cx = p.cx < 0 ? 0.5 * (p.nx - 1) : p.cx;
  const double cy = p.cx < 0 ? 0.5 * (p.ny - 1) : p.cy;
  const double cz = p.cx < 0 ? 0.5 * (p.nz - 1) : p.cz;
  int64_t inside = 0;
  for (int z = 0; z < p.nz; ++z)
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const double dx = x - cx, dy = y - cy, dz = z - cz;
        inside += dx * dx + dy * dy + dz * dz < p.radius * p.radius;
      }
  R.min_cc = (int32_t)std::max<int64_t>(1, (inside + 99) / 100);
  return R;
}

void destroy_graphs(lbm_ctx* c) {
  for (auto& kv : c->graphs) hipGraphExecDestroy(kv.second);
  for (auto& kv : c->graph_src) hipGraphDestroy(kv.second);
  c->graphs.clear();
  c->graph_src.clear();
}

// Tile table: canonical order (run, tz, ty, tx), cut into rounds of the
// workgroups the GPU holds at once (a persistent grid's size, else CUs x
// workgroups per CU); within a round the workgroups one XCD receives
// (dispatch is round-robin over the 8 XCDs) own a contiguous block of tiles.
// A round then covers one contiguous stretch of the lattice: the halo rows
// between XCD blocks are read by both at about the same time, and only the
// rows where one round meets the next are read at different times.
int build_tiles(lbm_ctx* c) {
  const lbm_launch& l = c->launch;
  std::vector<Tile> canon;
  for (int r = 0; r < c->nruns; ++r) {
    const RunDev& R = c->runs[r];
    const int bzr = l.bz > 0 ? l.bz : R.nz;   // bz = 0: whole columns
    for (int z = 0; z < R.nz; z += bzr)
      for (int y = 0; y < R.ny; y += l.by)
        for (int x = 0; x < R.nx; x += l.bx)
          canon.push_back(Tile{r, x, y, z, std::min(z + bzr, R.nz)});
  }
  const int64_t T = (int64_t)canon.size();
  int64_t cap = 0;   // workgroups resident at once
  if (l.persistent > 0) {
    cap = std::max(8, l.persistent / 8 * 8);
  } else {
    int per_cu = 0;
    bool wide = l.grouped != 0, trt = false;
    for (const RunDev& R : c->runs) {
      wide |= (int64_t)lbm::Q * R.ld * (int64_t)(c->prec == LBM_FP64 ? 8 : c->prec == LBM_FP32 ? 4 : 2) >=
              (int64_t)1 << 32;
      trt |= R.tau_m[0] != R.tau[0] || R.tau_m[1] != R.tau[1];
    }
    by_precision(c->prec, [&](auto* tt, auto* ss) {
      using T_ = std::remove_pointer_t<decltype(tt)>;
      using S_ = std::remove_pointer_t<decltype(ss)>;
      per_cu = lbm::step_blocks_per_cu<T_, S_>(l.bx, l.by, wide, trt);
    });
    cap = (int64_t)std::max(1, per_cu) * c->n_cu / 8 * 8;
  }
  cap = std::max<int64_t>(cap, 8);
  std::vector<Tile> table;
  table.reserve(T + 8 * (T / cap + 1));
  for (int64_t r0 = 0; r0 < T; r0 += cap) {
    const int64_t n = std::min(cap, T - r0);
    const int64_t per = (n + 7) / 8;   // tiles per XCD in this round
    for (int64_t p = 0; p < 8 * per; ++p) {
      const int64_t cidx = (p % 8) * per + p / 8;
      table.push_back(cidx < n ? canon[r0 + cidx] : Tile{-1, 0, 0, 0, 0});
    }
  }
  const int64_t Tp = (int64_t)table.size();
  if (Tp > c->L.tiles_cap) return LBM_EINVAL;
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->at<Tile>(c->L.tiles), table.data(), Tp * sizeof(Tile), hipMemcpyHostToDevice));
  c->ntiles = Tp;
  destroy_graphs(c);
  return LBM_OK;
}

// Enqueue the per-run step targets and reset the device step counter.
int set_targets(lbm_ctx* c, const int32_t* target) {
  for (int first = 0; first < c->nruns; first += MAX_TARGETS) {
    const int count = std::min(MAX_TARGETS, c->nruns - first);
    Targets t{};
    for (int i = 0; i < count; ++i) {
      t.target[i] = target[first + i];
      t.base[i] = (int32_t)(c->done[first + i] & 0x7fffffff);
      c->runs[first + i].target = t.target[i];
      c->runs[first + i].base = t.base[i];
    }
    k_set_targets<<<1, MAX_TARGETS, 0, c->stream>>>(c->at<RunDev>(c->L.runs), first, count, t,
                                                    c->at<int32_t>(c->L.gstep));
  }
  return hip_ok(hipGetLastError());
}

// One step: the fused step kernel, then the step counter.
void enqueue_step(lbm_ctx* c, hipStream_t s) {
  const dim3 grid = step_grid(c), block(c->launch.bx, c->launch.by);
  by_precision(c->prec, [&](auto* tt, auto* ss) {
    using T = std::remove_pointer_t<decltype(tt)>;
    using S = std::remove_pointer_t<decltype(ss)>;
    lbm::launch_step<T, S>(step_args<T, S>(c), grid, block, s);
  });
  lbm::launch_inc_step(c->at<int32_t>(c->L.gstep), s);
}

int get_graph(lbm_ctx* c, int chunk, hipGraphExec_t* out) {
  auto it = c->graphs.find(chunk);
  if (it != c->graphs.end()) { *out = it->second; return LBM_OK; }
  if (!c->cap) HIPCHK(hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
  for (int k = 0; k < chunk; ++k) enqueue_step(c, c->cap);
  const hipError_t e = hipStreamEndCapture(c->cap, &g);
  if (e != hipSuccess || !g) return LBM_EHIP;
  hipGraphExec_t ex = nullptr;
  if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
    hipGraphDestroy(g);
    return LBM_EHIP;
  }
  c->graph_src[chunk] = g;
  c->graphs[chunk] = ex;
  *out = ex;
  return LBM_OK;
}

int run_steps(lbm_ctx* c, const int32_t* target) {
  int32_t m = 0;
  for (int r = 0; r < c->nruns; ++r) {
    if (target[r] < 0) return LBM_EINVAL;
    m = std::max(m, target[r]);
  }
  if (m == 0) return LBM_OK;
  int e = set_targets(c, target);
  if (e) return e;
  int remaining = m;
  for (int chunk : GRAPH_CHUNKS) {
    while (remaining >= chunk) {
      hipGraphExec_t ex;
      e = get_graph(c, chunk, &ex);
      if (e) return e;
      HIPCHK(hipGraphLaunch(ex, c->stream));
      remaining -= chunk;
    }
  }
  for (int r = 0; r < c->nruns; ++r) c->done[r] += target[r];
  return LBM_OK;
}

// Physical velocity of every run at its current state (observe, export).
int refresh_flow(lbm_ctx* c) {
  std::vector<int32_t> zero(c->nruns, 0);
  const int e = set_targets(c, zero.data());
  if (e) return e;
  by_precision(c->prec, [&](auto* tt, auto* ss) {
    using T = std::remove_pointer_t<decltype(tt)>;
    using S = std::remove_pointer_t<decltype(ss)>;
    lbm::launch_flow<T, S>(aux_args<T, S>(c, 1), c->stream);
  });
  return hip_ok(hipGetLastError());
}

void finish_obs(const lbm_ctx* c, int r, const double* o, lbm_obs* out) {
  const lbm_params& p = c->prm[r];
  std::memset(out, 0, sizeof(*out));
  out->step = c->done[r];
  out->mass[0] = o[lbm::OB_MA];
  out->mass[1] = o[lbm::OB_MB];
  const double W = o[lbm::OB_W];
  out->weight = W;
  const double hx = 0.5 * (p.nx - 1), hy = 0.5 * (p.ny - 1), hz = 0.5 * (p.nz - 1);
  if (W > 0.0) {
    const double X = o[lbm::OB_WX] / W, Y = o[lbm::OB_WY] / W, Z = o[lbm::OB_WZ] / W;
    const double Ixx = o[lbm::OB_WXX] - W * X * X;
    const double Ixz = o[lbm::OB_WXZ] - W * X * Z;
    const double Izz = o[lbm::OB_WZZ] - W * Z * Z;
    out->centroid[0] = X + hx; out->centroid[1] = Y + hy; out->centroid[2] = Z + hz;
    out->inertia[0] = Ixx; out->inertia[1] = Ixz; out->inertia[2] = Izz;
    const double mean = 0.5 * (Ixx + Izz);
    const double rad = std::sqrt(0.25 * (Ixx - Izz) * (Ixx - Izz) + Ixz * Ixz);
    const double lp = mean + rad, lm = std::max(mean - rad, 0.0);
    const double sp = std::sqrt(lp), sm = std::sqrt(lm);
    out->D = sp + sm > 0.0 ? (sp - sm) / (sp + sm) : 0.0;
    out->theta_deg = 0.5 * std::atan2(2.0 * Ixz, Ixx - Izz) * (180.0 / M_PI);
  }
  out->Lp = o[lbm::OB_XMAX] >= o[lbm::OB_XMIN] ? o[lbm::OB_XMAX] - o[lbm::OB_XMIN] + 1.0 : 0.0;
  out->umax = std::sqrt(o[lbm::OB_U2MAX]);
  out->trC_max = o[lbm::OB_TRCMAX];
  out->n_components = -1;
  for (int i = 0; i < 4; ++i) out->piece_nodes[i] = 0;
}

}  // namespace

// ============================================================================
extern "C" {

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_EUNSUP: return "unsupported device or combination";
    case LBM_ENAN: return "non-finite value in the state";
    case LBM_EFENE: return "conformation trace reached L^2";
    default: return "unknown status";
  }
}

int lbm_validate(const lbm_params* p) { return validate(p); }

int lbm_batch_workspace_bytes(const lbm_params* runs, int32_t nruns, size_t* bytes) {
  if (!bytes) return LBM_EINVAL;
  const int e = validate_all(runs, nruns);
  if (e) return e;
  *bytes = make_layout(runs, nruns).total;
  return LBM_OK;
}

int lbm_workspace_bytes(const lbm_params* p, size_t* bytes) { return lbm_batch_workspace_bytes(p, 1, bytes); }

int lbm_batch_init(const lbm_params* runs, int32_t nruns, void* ws, size_t bytes, void* stream,
                   lbm_ctx** out) {
  if (!out || !ws) return LBM_EINVAL;
  *out = nullptr;
  int e = validate_all(runs, nruns);
  if (e) return e;
  const Layout L = make_layout(runs, nruns);
  if (bytes < L.total) return LBM_ENOMEM;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return LBM_EUNSUP;

  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return LBM_EINVAL;
  c->nruns = nruns;
  c->prec = runs[0].precision;
  // default launch: whole-column tiles of the shape the autotuner picks for
  // single lattices (32x8; 16x8 in FP64, whose rings are twice as large)
  c->launch = c->prec == LBM_FP64 ? lbm_launch{16, 8, 0, 0, 0} : lbm_launch{32, 8, 0, 0, 0};
  c->n_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->stream = (hipStream_t)stream;
  c->ws = (char*)ws;
  c->L = L;
  c->prm.assign(runs, runs + nruns);
  c->done.assign(nruns, 0);
  int64_t off = 0;
  std::vector<double> rc(4 * nruns), rinit(4 * nruns);
  for (int r = 0; r < nruns; ++r) {
    c->runs.push_back(make_run(runs[r], off));
    off += c->runs.back().ld;
    const lbm_params& p = runs[r];
    const bool centre = p.cx < 0;
    rc[4 * r] = p.radius;
    rc[4 * r + 1] = centre ? 0.5 * (p.nx - 1) : p.cx;
    rc[4 * r + 2] = centre ? 0.5 * (p.ny - 1) : p.cy;
    rc[4 * r + 3] = centre ? 0.5 * (p.nz - 1) : p.cz;
    rinit[4 * r] = p.rho_major;
    rinit[4 * r + 1] = p.rho_minor;
    rinit[4 * r + 2] = p.init_noise;
    std::memcpy(&rinit[4 * r + 3], &p.seed, 8);   // the seed's bits
  }
  auto fail = [&](int code) { lbm_destroy(c); return code; };
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(LBM_EHIP);
  if (hipMemcpy(c->at<RunDev>(L.runs), c->runs.data(), nruns * sizeof(RunDev), hipMemcpyHostToDevice) ||
      hipMemcpy(c->at<double>(L.rc), rc.data(), rc.size() * 8, hipMemcpyHostToDevice) ||
      hipMemcpy(c->at<double>(L.rinit), rinit.data(), rinit.size() * 8, hipMemcpyHostToDevice))
    return fail(LBM_EHIP);
  e = build_tiles(c);
  if (e) return fail(e);
  lbm::launch_fill_u32(c->at<uint32_t>(L.status), 0u, nruns, c->stream);
  by_precision(c->prec, [&](auto* tt, auto* ss) {
    using T = std::remove_pointer_t<decltype(tt)>;
    using S = std::remove_pointer_t<decltype(ss)>;
    lbm::launch_init<T, S>(aux_args<T, S>(c, 0), c->stream);
  });
  if (hipGetLastError() != hipSuccess) return fail(LBM_EHIP);
  *out = c;
  return LBM_OK;
}

int lbm_init(const lbm_params* p, void* ws, size_t bytes, void* stream, lbm_ctx** out) {
  return lbm_batch_init(p, 1, ws, bytes, stream, out);
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream || c->cap) hipStreamSynchronize(c->stream);
  destroy_graphs(c);
  if (c->cap) hipStreamDestroy(c->cap);
  delete c;
}

int32_t lbm_batch_nruns(const lbm_ctx* c) { return c ? c->nruns : 0; }

int lbm_get_launch(const lbm_ctx* c, lbm_launch* out) {
  if (!c || !out) return LBM_EINVAL;
  *out = c->launch;
  return LBM_OK;
}

int lbm_set_launch(lbm_ctx* c, const lbm_launch* in) {
  if (!c || !in) return LBM_EINVAL;
  const lbm_launch l = *in;
  // block shapes with a compiled step-kernel instance for this precision
  const bool shape_ok = lbm::step_shape_ok(l.bx, l.by, c->prec == LBM_FP64);
  if (!shape_ok || l.bz < 0 || l.bz > 1024 || l.persistent < 0) return LBM_EINVAL;
  if (l.grouped != 0 && l.grouped != 1) return LBM_EINVAL;
  const lbm_launch old = c->launch;
  c->launch = l;
  const int e = build_tiles(c);
  if (e) { c->launch = old; build_tiles(c); }
  return e;
}

int lbm_steps_done(const lbm_ctx* c, int32_t run, int64_t* out) {
  if (!c || !out || run < 0 || run >= c->nruns) return LBM_EINVAL;
  *out = c->done[run];
  return LBM_OK;
}

int lbm_batch_step(lbm_ctx* c, const int32_t* steps) {
  if (!c || !steps) return LBM_EINVAL;
  return run_steps(c, steps);
}

int lbm_step_profiled(lbm_ctx* c, int32_t nsteps, double* ms_step) {
  if (!c || nsteps < 0 || !ms_step) return LBM_EINVAL;
  *ms_step = 0.0;
  if (nsteps == 0) return LBM_OK;
  std::vector<int32_t> t(c->nruns, nsteps);
  int e = set_targets(c, t.data());
  if (e) return e;
  std::vector<hipEvent_t> ev(2 * (size_t)nsteps, nullptr);
  for (auto& x : ev)
    if (hipEventCreate(&x) != hipSuccess) { e = LBM_EHIP; break; }
  const dim3 grid = step_grid(c), block(c->launch.bx, c->launch.by);
  for (int k = 0; k < nsteps && !e; ++k) {
    by_precision(c->prec, [&](auto* tt, auto* ss) {
      using T = std::remove_pointer_t<decltype(tt)>;
      using S = std::remove_pointer_t<decltype(ss)>;
      hipEventRecord(ev[2 * k], c->stream);
      lbm::launch_step<T, S>(step_args<T, S>(c), grid, block, c->stream);
      hipEventRecord(ev[2 * k + 1], c->stream);
    });
    lbm::launch_inc_step(c->at<int32_t>(c->L.gstep), c->stream);
  }
  if (!e && hipStreamSynchronize(c->stream) != hipSuccess) e = LBM_EHIP;
  for (int k = 0; k < nsteps && !e; ++k) {
    float v = 0.f;
    if (hipEventElapsedTime(&v, ev[2 * k], ev[2 * k + 1]) != hipSuccess) { e = LBM_EHIP; break; }
    *ms_step += v;
  }
  for (auto& x : ev)
    if (x) hipEventDestroy(x);
  if (e) return e;
  for (int r = 0; r < c->nruns; ++r) c->done[r] += nsteps;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int32_t nsteps) {
  if (!c || nsteps < 0) return LBM_EINVAL;
  std::vector<int32_t> t(c->nruns, nsteps);
  return run_steps(c, t.data());
}

int lbm_batch_observe(lbm_ctx* c, int32_t want_cc, lbm_obs* out) {
  if (!c || !out) return LBM_EINVAL;
  int e = refresh_flow(c);
  if (e) return e;
  by_precision(c->prec, [&](auto* tt, auto* ss) {
    using T = std::remove_pointer_t<decltype(tt)>;
    using S = std::remove_pointer_t<decltype(ss)>;
    const auto a = aux_args<T, S>(c, 1);
    lbm::launch_observe<T, S>(a, c->stream);
    if (want_cc) lbm::launch_components<T, S>(a, c->stream);
  });
  HIPCHK(hipGetLastError());
  std::vector<double> o((size_t)c->nruns * lbm::NOBS);
  std::vector<uint32_t> st(c->nruns);
  std::vector<int32_t> nc(c->nruns), pc((size_t)c->nruns * lbm::MAX_PIECES);
  HIPCHK(hipMemcpyAsync(o.data(), c->at<double>(c->L.obs), o.size() * 8, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(st.data(), c->at<uint32_t>(c->L.status), st.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(nc.data(), c->at<int32_t>(c->L.ncomp), nc.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipMemcpyAsync(pc.data(), c->at<int32_t>(c->L.pieces), pc.size() * 4, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  int first = LBM_OK;
  for (int r = 0; r < c->nruns; ++r) {
    finish_obs(c, r, o.data() + (size_t)r * lbm::NOBS, out + r);
    if (want_cc) {
      out[r].n_components = nc[r];
      // sizes of the largest pieces, in descending order
      const int k = std::min<int>(nc[r], lbm::MAX_PIECES);
      std::vector<int32_t> sz(pc.begin() + (size_t)r * lbm::MAX_PIECES,
                              pc.begin() + (size_t)r * lbm::MAX_PIECES + k);
      std::sort(sz.begin(), sz.end(), [](int32_t p, int32_t q) { return p > q; });
      for (int i = 0; i < 4 && i < k; ++i) out[r].piece_nodes[i] = sz[i];
    }
    int s = LBM_OK;
    if ((st[r] & lbm::ST_NAN) || o[(size_t)r * lbm::NOBS + lbm::OB_NONFINITE] > 0) s = LBM_ENAN;
    else if (st[r] & lbm::ST_FENE) s = LBM_EFENE;
    else if (want_cc && (st[r] & lbm::ST_CC)) s = LBM_EHIP;
    out[r].status = s;
    if (s && !first) first = s;
  }
  return first;
}

int lbm_observe(lbm_ctx* c, int32_t want_cc, lbm_obs* out) {
  if (!c || !out) return LBM_EINVAL;
  std::vector<lbm_obs> all(c->nruns);
  const int e = lbm_batch_observe(c, want_cc, all.data());
  *out = all[0];
  return e == LBM_EINVAL || e == LBM_EHIP ? e : all[0].status;
}

static int64_t field_elems(const lbm_params& p, int field) {
  const int64_t n = (int64_t)p.nx * p.ny * p.nz;
  switch (field) {
    case LBM_FIELD_F: return 38 * n;
    case LBM_FIELD_C: return 6 * n;
    case LBM_FIELD_RHO: return 2 * n;
    case LBM_FIELD_U: return 3 * n;
    default: return -1;
  }
}

}  // extern "C"

namespace {

// Storage units of the shifted populations (FP16 keeps g * 2^12).
double pop_scale(int prec) { return prec == LBM_FP16S ? 4096.0 : 1.0; }

// Host views of device element types: S (populations) and T (other fields).
double get_elem(size_t bytes, const char* buf, int64_t k) {
  if (bytes == 8) return ((const double*)buf)[k];
  if (bytes == 4) return (double)((const float*)buf)[k];
  return (double)__half2float(((const __half*)buf)[k]);
}
void put_elem(size_t bytes, char* buf, int64_t k, double v) {
  if (bytes == 8) ((double*)buf)[k] = v;
  else if (bytes == 4) ((float*)buf)[k] = (float)v;
  else ((__half*)buf)[k] = __float2half_rn((float)v);
}

// Device <-> host copies of a run's block of `comps` arrays (stride ld).
int copy_out(const lbm_ctx* c, size_t dev_off, size_t elem, int comps, const RunDev& R, char* host) {
  const size_t w = (size_t)R.n * elem;
  return hipMemcpy2D(host, w, c->ws + dev_off, (size_t)R.ld * elem, w, comps,
                     hipMemcpyDeviceToHost) == hipSuccess ? LBM_OK : LBM_EHIP;
}
int copy_in(lbm_ctx* c, size_t dev_off, size_t elem, int comps, const RunDev& R, const char* host) {
  const size_t w = (size_t)R.n * elem;
  return hipMemcpy2D(c->ws + dev_off, (size_t)R.ld * elem, host, w, w, comps,
                     hipMemcpyHostToDevice) == hipSuccess ? LBM_OK : LBM_EHIP;
}

// Clear one run's status after its state was replaced.
int after_state_change(lbm_ctx* c, int run) {
  lbm::launch_fill_u32(c->at<uint32_t>(c->L.status) + run, 0u, 1, c->stream);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

// Raw state blob: header, then populations as stored, densities, momenta
// and C.
struct StateHeader {
  uint64_t magic;
  int32_t precision, nx, ny, nz, visc, pad;
  int64_t done;
};
constexpr uint64_t STATE_MAGIC = 0x32534d564d424cull;   // "LBMVMS2"

size_t state_bytes(const lbm_ctx* c, int run) {
  const int64_t N = c->runs[run].n;
  return sizeof(StateHeader) + (size_t)N * (38 * elem_S(c->prec) + 14 * elem_T(c->prec));
}

// Shift of direction i against the node moments: w_i (rho + 3 c_i.j).
double pop_shift(int i, double rho, double jx, double jy, double jz) {
  return lbm::wgt<double>(i) *
         (rho + 3.0 * (lbm::CX[i] * jx + lbm::CY[i] * jy + lbm::CZ[i] * jz));
}

}  // namespace

extern "C" {

int lbm_batch_export(lbm_ctx* c, int32_t run, int32_t field, double* host, size_t n) {
  if (!c || !host || run < 0 || run >= c->nruns) return LBM_EINVAL;
  const int64_t want = field_elems(c->prm[run], field);
  if (want < 0 || (int64_t)n != want) return LBM_EINVAL;
  const RunDev& R = c->runs[run];
  const int par = (int)(c->done[run] & 1);
  const int64_t N = R.n;
  if (field == LBM_FIELD_U) {
    const int e = refresh_flow(c);
    if (e) return e;
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  const size_t st = elem_S(c->prec), tt = elem_T(c->prec);
  std::vector<char> buf;
  int e = LBM_OK;
  if (field == LBM_FIELD_F) {
    // f_i = g_i + w_i (rho_s + 3 c_i.j_s), decoded in FP64
    std::vector<char> rb((size_t)2 * N * tt), jb((size_t)6 * N * tt);
    buf.resize((size_t)want * st);
    e = copy_out(c, c->L.f[par] + (size_t)R.off * 38 * st, st, 38, R, buf.data());
    if (!e) e = copy_out(c, c->L.rho[par] + (size_t)R.off * 2 * tt, tt, 2, R, rb.data());
    if (!e) e = copy_out(c, c->L.j[par] + (size_t)R.off * 6 * tt, tt, 6, R, jb.data());
    if (e) return e;
    const double isc = 1.0 / pop_scale(c->prec);
    for (int64_t k = 0; k < want; ++k) {
      const int s = (int)(k / (19 * N)), i = (int)((k / N) % 19);
      const int64_t m = k % N;
      host[k] = get_elem(st, buf.data(), k) * isc +
                pop_shift(i, get_elem(tt, rb.data(), s * N + m),
                          get_elem(tt, jb.data(), (3 * s) * N + m),
                          get_elem(tt, jb.data(), (3 * s + 1) * N + m),
                          get_elem(tt, jb.data(), (3 * s + 2) * N + m));
    }
    return LBM_OK;
  }
  size_t src = 0;
  int comps = 0;
  if (field == LBM_FIELD_C) { src = c->L.C[R.visc >= 0 ? par : 0] + (size_t)R.off * 6 * tt; comps = 6; }
  else if (field == LBM_FIELD_RHO) { src = c->L.rho[par] + (size_t)R.off * 2 * tt; comps = 2; }
  else { src = c->L.u + (size_t)R.off * 3 * tt; comps = 3; }
  buf.resize((size_t)want * tt);
  e = copy_out(c, src, tt, comps, R, buf.data());
  if (e) return e;
  for (int64_t k = 0; k < want; ++k) host[k] = get_elem(tt, buf.data(), k);
  return LBM_OK;
}

int lbm_export(lbm_ctx* c, int32_t field, double* host, size_t n) {
  return lbm_batch_export(c, 0, field, host, n);
}

int lbm_batch_import(lbm_ctx* c, int32_t run, int32_t field, const double* host, size_t n) {
  if (!c || !host || run < 0 || run >= c->nruns) return LBM_EINVAL;
  if (field != LBM_FIELD_F && field != LBM_FIELD_C) return LBM_EINVAL;
  const int64_t want = field_elems(c->prm[run], field);
  if ((int64_t)n != want) return LBM_EINVAL;
  const RunDev& R = c->runs[run];
  const int par = (int)(c->done[run] & 1);
  const int64_t N = R.n;
  const size_t st = elem_S(c->prec), tt = elem_T(c->prec);
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<char> buf;
  int e = LBM_OK;
  if (field == LBM_FIELD_F) {
    // node moments rho_s = sum_i f_i, j_s = sum_i c_i f_i (FP64, rounded to
    // the field type), then the shifted values g_i = f_i - w_i (rho + 3 c_i.j)
    // against the rounded moments
    std::vector<char> rb((size_t)2 * N * tt), jb((size_t)6 * N * tt);
    for (int s = 0; s < 2; ++s)
      for (int64_t m = 0; m < N; ++m) {
        double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        for (int i = 0; i < 19; ++i) {
          const double v = host[((int64_t)s * 19 + i) * N + m];
          r += v;
          jx += lbm::CX[i] * v;
          jy += lbm::CY[i] * v;
          jz += lbm::CZ[i] * v;
        }
        put_elem(tt, rb.data(), s * N + m, r);
        put_elem(tt, jb.data(), (3 * s) * N + m, jx);
        put_elem(tt, jb.data(), (3 * s + 1) * N + m, jy);
        put_elem(tt, jb.data(), (3 * s + 2) * N + m, jz);
      }
    buf.resize((size_t)want * st);
    const double sc = pop_scale(c->prec);
    for (int64_t k = 0; k < want; ++k) {
      const int s = (int)(k / (19 * N)), i = (int)((k / N) % 19);
      const int64_t m = k % N;
      const double sh = pop_shift(i, get_elem(tt, rb.data(), s * N + m),
                                  get_elem(tt, jb.data(), (3 * s) * N + m),
                                  get_elem(tt, jb.data(), (3 * s + 1) * N + m),
                                  get_elem(tt, jb.data(), (3 * s + 2) * N + m));
      put_elem(st, buf.data(), k, (host[k] - sh) * sc);
    }
    e = copy_in(c, c->L.f[par] + (size_t)R.off * 38 * st, st, 38, R, buf.data());
    if (!e) e = copy_in(c, c->L.rho[par] + (size_t)R.off * 2 * tt, tt, 2, R, rb.data());
    if (!e) e = copy_in(c, c->L.j[par] + (size_t)R.off * 6 * tt, tt, 6, R, jb.data());
  } else {
    buf.resize((size_t)want * tt);
    for (int64_t k = 0; k < want; ++k) put_elem(tt, buf.data(), k, host[k]);
    // a Newtonian run never updates C, which stays at parity 0
    const int cp = R.visc >= 0 ? par : 0;
    e = copy_in(c, c->L.C[cp] + (size_t)R.off * 6 * tt, tt, 6, R, buf.data());
  }
  if (e) return e;
  return after_state_change(c, run);
}

int lbm_batch_state_bytes(const lbm_ctx* c, int32_t run, size_t* bytes) {
  if (!c || !bytes || run < 0 || run >= c->nruns) return LBM_EINVAL;
  *bytes = state_bytes(c, run);
  return LBM_OK;
}

int lbm_batch_save_state(lbm_ctx* c, int32_t run, void* host, size_t bytes) {
  if (!c || !host || run < 0 || run >= c->nruns || bytes != state_bytes(c, run)) return LBM_EINVAL;
  const RunDev& R = c->runs[run];
  const lbm_params& p = c->prm[run];
  const int par = (int)(c->done[run] & 1);
  const size_t st = elem_S(c->prec), tt = elem_T(c->prec);
  HIPCHK(hipStreamSynchronize(c->stream));
  StateHeader h{STATE_MAGIC, c->prec, p.nx, p.ny, p.nz, R.visc, 0, c->done[run]};
  char* out = static_cast<char*>(host);
  std::memcpy(out, &h, sizeof h);
  char* q = out + sizeof h;
  int e = copy_out(c, c->L.f[par] + (size_t)R.off * 38 * st, st, 38, R, q);
  q += (size_t)R.n * 38 * st;
  if (!e) e = copy_out(c, c->L.rho[par] + (size_t)R.off * 2 * tt, tt, 2, R, q);
  q += (size_t)R.n * 2 * tt;
  if (!e) e = copy_out(c, c->L.j[par] + (size_t)R.off * 6 * tt, tt, 6, R, q);
  q += (size_t)R.n * 6 * tt;
  const int cp = R.visc >= 0 ? par : 0;
  if (!e) e = copy_out(c, c->L.C[cp] + (size_t)R.off * 6 * tt, tt, 6, R, q);
  return e;
}

int lbm_batch_load_state(lbm_ctx* c, int32_t run, const void* host, size_t bytes) {
  if (!c || !host || run < 0 || run >= c->nruns || bytes != state_bytes(c, run)) return LBM_EINVAL;
  const RunDev& R = c->runs[run];
  const lbm_params& p = c->prm[run];
  StateHeader h;
  std::memcpy(&h, host, sizeof h);
  if (h.magic != STATE_MAGIC || h.precision != c->prec || h.nx != p.nx || h.ny != p.ny ||
      h.nz != p.nz || h.visc != R.visc || h.done < 0)
    return LBM_EINVAL;
  const size_t st = elem_S(c->prec), tt = elem_T(c->prec);
  HIPCHK(hipStreamSynchronize(c->stream));
  c->done[run] = h.done;
  const int par = (int)(h.done & 1);
  const char* q = static_cast<const char*>(host) + sizeof h;
  int e = copy_in(c, c->L.f[par] + (size_t)R.off * 38 * st, st, 38, R, q);
  q += (size_t)R.n * 38 * st;
  if (!e) e = copy_in(c, c->L.rho[par] + (size_t)R.off * 2 * tt, tt, 2, R, q);
  q += (size_t)R.n * 2 * tt;
  if (!e) e = copy_in(c, c->L.j[par] + (size_t)R.off * 6 * tt, tt, 6, R, q);
  q += (size_t)R.n * 6 * tt;
  const int cp = R.visc >= 0 ? par : 0;
  if (!e) e = copy_in(c, c->L.C[cp] + (size_t)R.off * 6 * tt, tt, 6, R, q);
  if (e) return e;
  return after_state_change(c, run);
}

int lbm_import(lbm_ctx* c, int32_t field, const double* host, size_t n) {
  return lbm_batch_import(c, 0, field, host, n);
}

}  // extern "C"
