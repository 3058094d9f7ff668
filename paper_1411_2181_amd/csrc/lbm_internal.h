// Internal interface between the host library and the kernel translation
// units (not part of the public C ABI).
#pragma once

#include "lbm_device.h"

namespace lbm {

template <typename T, typename S>
struct StepArgs {
  Pools<T, S> P;
  const RunDev* runs;
  const Tile* tiles;
  int32_t ntiles;
  const int32_t* gstep;   // step index within the current step call
  int32_t any_visc;       // some run of the batch carries a polymer phase
  int32_t wide;           // some run's 19 population arrays span >= 4 GiB
  int32_t trt;            // some run has tau^- != tau (two-relaxation-time)
};

// Population addressing of the step kernel: direction i of a run is read
// from a 64-bit base of its group of G direction arrays plus a 32-bit byte
// offset, so G arrays of one run must span less than 4 GiB.  G = Q (one base
// for all directions: fewest scalar registers) when a run's 19 arrays fit;
// runs up to the library's limit use G = DG_WIDE.
constexpr int DG_WIDE = 4;

// Number of per-block partial values of the observable reduction.
constexpr int NOBS = 16;
enum ObsSlot {
  OB_MA = 0, OB_MB, OB_W, OB_WX, OB_WY, OB_WZ, OB_WXX, OB_WXZ, OB_WZZ,
  OB_U2MAX, OB_TRCMAX, OB_XMIN, OB_XMAX, OB_NONFINITE, OB_PAD0, OB_PAD1
};
// blocks per run of the per-node auxiliary kernels (init, moments, observe,
// component labelling)
constexpr int AUX_BLOCKS = 128;
constexpr int AUX_THREADS = 256;

constexpr int MAX_PIECES = 8;   // pieces whose sizes are kept per run

template <typename T, typename S>
struct AuxArgs {
  Pools<T, S> P;
  const RunDev* runs;
  int32_t nruns;
  int32_t use_parity;      // parity of each run = (runs[r].base) & 1 when 1, else 0
  double* partials;        // [nruns][AUX_BLOCKS][NOBS]
  double* obs;             // [nruns][NOBS]
  int32_t* labels;         // per node (component labelling)
  int32_t* counts;         // per node
  int32_t* ncomp;          // per run: pieces counted
  int32_t* pieces;         // [nruns][MAX_PIECES]: node counts of counted pieces, unordered
  const double* radius_centre;  // [nruns][4]: R, cx, cy, cz  (init only)
  const double* rho_init;       // [nruns][4]: rho_major, rho_minor, init_noise, seed bits (init only)
};

// One time step over the tile table: grid.x workgroups (two per tile slot,
// one per component; see k_step), block (bx, by).
template <typename T, typename S>
void launch_step(const StepArgs<T, S>& a, dim3 grid, dim3 block, hipStream_t s);
// Tile shapes (bx, by) with a compiled instance of the step kernel for the
// compute type T (the FP64 instance has fewer: its LDS rings are twice as
// large).
bool step_shape_ok(int bx, int by, bool fp64);
template <typename T, typename S>
int step_blocks_per_cu(int bx, int by, bool wide, bool trt);

template <typename T, typename S>
void launch_init(const AuxArgs<T, S>& a, hipStream_t s);
// Physical velocity u of every run at its current parity (observe, export).
template <typename T, typename S>
void launch_flow(const AuxArgs<T, S>& a, hipStream_t s);
template <typename T, typename S>
void launch_observe(const AuxArgs<T, S>& a, hipStream_t s);
template <typename T, typename S>
void launch_components(const AuxArgs<T, S>& a, hipStream_t s);

void launch_set_step(int32_t* gstep, int32_t v, hipStream_t s);
void launch_inc_step(int32_t* gstep, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

}  // namespace lbm
