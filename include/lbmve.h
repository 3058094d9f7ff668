/*
 * lbmve — MI355X (gfx950) library for the per-timestep hot path of the
 * hybrid lattice-Boltzmann / finite-difference solver of viscoelastic
 * droplets in confined shear (Gupta & Sbragaglia, arXiv:1411.2181).
 *
 * One step advances, on every lattice node, two immiscible lattice-Boltzmann
 * components (Shan-Chen interaction, Section 2) and the FENE-P conformation
 * tensor of the viscoelastic phase (Eqs. (2) and (4), Peterlin factor
 * f = (L^2-3)/(L^2 - tr C) defined below Eq. (2)), with the polymer stress
 * fed back as the body force (eta_P/tau_P) div[f C] of Eqs. (1) and (3).
 * The flow is the confined shear of Section 3: walls at z = 0 and z = W
 * moving at -U_w and +U_w along x, periodic in x and y, a sphere of radius R
 * at mid-gap at t = 0.
 *
 * Discrete scheme: D3Q19, BGK with one relaxation time per component,
 * Shan-Chen force with interaction weights 3 w_i and psi = rho, Shan-Chen
 * velocity-shift forcing, half-way moving-wall bounce-back (walls half a
 * link outside z = 0 and z = nz-1, so W = nz), explicit Euler FENE-P with
 * first-order upwind advection and centred velocity gradients.
 *
 * All calls return an int status (LBM_OK = 0 or a negative LBM_E* code);
 * lbm_strerror() gives its text.  No call throws.  Every pointer argument is
 * a plain host pointer unless its name ends in _dev (device memory) or is the
 * workspace / stream pair of an init call.
 *
 * Memory ownership:
 *   - the caller owns the device workspace passed to *_init (it must stay
 *     allocated until lbm_destroy) and the HIP stream (hipStream_t passed as
 *     void*; NULL = the null stream);
 *   - the library owns the opaque context and the HIP graphs it builds;
 *   - parameter structs are copied at init; host buffers are only read or
 *     written during the call that receives them.
 *
 * Threading: a context is not thread-safe; calls on one context must be
 * serialised by the caller.  Step calls are asynchronous on the context's
 * stream; observe / export / import synchronise that stream.
 */
#ifndef LBMVE_H
#define LBMVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,  /* invalid argument or parameter set (nothing touched)  */
  LBM_ENOMEM = -2,  /* workspace too small                                   */
  LBM_EHIP = -3,    /* a HIP runtime call failed                             */
  LBM_EUNSUP = -4,  /* unsupported combination (e.g. no gfx950 device)       */
  LBM_ENAN = -5,    /* a non-finite value appeared in the state              */
  LBM_EFENE = -6    /* tr C reached L^2 (Peterlin factor undefined)          */
};

/* ---- storage precision of the populations and of C -------------------- */
enum {
  LBM_FP64 = 0,   /* populations FP64, C FP64, arithmetic FP64                */
  LBM_FP32 = 1,   /* populations FP32, C FP32, arithmetic FP32                */
  LBM_FP16S = 2   /* populations FP16 stored as
                     (f_i - w_i (rho_s(x) + 3 c_i.j_s(x))) * 2^12, the shift
                     taken from the FP32 density and momentum of the node
                     holding the value and rounded stochastically; densities,
                     momenta and C FP32, arithmetic FP32                      */
};
/* In every precision the Peterlin factor f(tr C) and all observable
 * reductions are evaluated in FP64. */

/* ---- exportable fields (FP64, oracle order, x fastest) ---------------- */
enum {
  LBM_FIELD_F = 0,    /* f[2][19][nz][ny][nx]  post-stream populations      */
  LBM_FIELD_C = 1,    /* C[6][nz][ny][nx]      xx, yy, zz, xy, xz, yz        */
  LBM_FIELD_RHO = 2,  /* rho[2][nz][ny][nx]    (export only)                 */
  LBM_FIELD_U = 3     /* u[3][nz][ny][nx]      physical velocity
                         (j_A + j_B + (F_A + F_B)/2)/rho (export only)       */
};

/*
 * Parameters of one run (lattice units).  Component A is the droplet
 * component, B the matrix component.  The direction order of the
 * populations is: 0 rest; 1,2 = +-x; 3,4 = +-y; 5,6 = +-z; 7,8 = +-(1,1,0);
 * 9,10 = +-(1,-1,0); 11,12 = +-(1,0,1); 13,14 = +-(1,0,-1);
 * 15,16 = +-(0,1,1); 17,18 = +-(0,1,-1).
 */
typedef struct {
  int32_t nx, ny, nz;    /* fluid nodes, each >= 3; W = nz; nx*ny*nz < 2^31
                            and nx*ny*nz*(bytes per stored population) < 2^32 */
  int32_t precision;     /* LBM_FP64 | LBM_FP32 | LBM_FP16S                  */
  double u_wall;         /* top wall +u_wall, bottom wall -u_wall (x); |.|<0.2 */
  double radius;         /* droplet radius R (0 = no droplet); R < nz/2      */
  double cx, cy, cz;     /* droplet centre; cx < 0 => box centre
                            ((nx-1)/2, (ny-1)/2, (nz-1)/2)                   */
  double rho_major;      /* majority density of each component (> 0)         */
  double rho_minor;      /* minority density (> 0)                            */
  double G;              /* Shan-Chen coupling (>= 0)                         */
  double tau[2];         /* relaxation time of A and B, > 0.5: BGK, or the
                            rate of the parts of f even under c -> -c (it
                            sets the viscosity) when tau_minus is given     */
  double tau_P[2];       /* polymer relaxation time of phase A, B (> 0)      */
  double eta_P[2];       /* polymer viscosity of phase A, B; a phase is
                            viscoelastic iff eta_P > 0; at most one may be   */
  double L2[2];          /* FENE-P extensibility L^2 of phase A, B (> 3)     */
  double chi_lo, chi_hi; /* bounds of the polymer-phase indicator: chi =
                            clamp((x_p - chi_lo)/(chi_hi - chi_lo), 0, 1),
                            x_p the mass fraction of the polymer phase's
                            component; both 0 => mean-field coexistence
                            fractions at (G, rho_major + rho_minor)          */
  uint64_t seed;         /* seed of the optional initial density noise       */
  double init_noise;     /* its relative amplitude a, 0 <= a < 0.1 (0: none):
                            component s's initial density at node n (x
                            fastest) is rho (1 + a u), u = (w >> 11) 2^-52 - 1
                            in [-1, 1) with w the SplitMix64 word of counter
                            2 n + s: mix(seed + (2 n + s + 1) 0x9e3779b97f4a7c15)
                            (Steele, Lea and Flood 2014, its finaliser)      */
  double tau_minus[2];   /* two-relaxation-time collision (a model variant
                            beyond the paper's BGK): relaxation time of the
                            parts of f odd under c -> -c for A and B, > 0.5;
                            0 selects tau (BGK).  The odd parts carry the
                            momentum, so the velocity shift of the forcing
                            takes tau_minus where BGK takes tau.  With
                            Lambda = (tau - 1/2)(tau_minus - 1/2) = 3/16 the
                            half-way bounce-back walls hold a force-driven
                            channel parabola exactly                        */
} lbm_params;

/* Observables of one run at the current state. */
typedef struct {
  int64_t step;          /* steps taken since init                           */
  double mass[2];        /* sum over nodes of rho_A, rho_B                   */
  double weight;         /* sum of w = max(phi, 0), phi = (rhoA-rhoB)/rho    */
  double centroid[3];    /* sum w x / sum w (unwrapped node coordinates)     */
  double inertia[3];     /* I_xx, I_xz, I_zz = sum w (x_a-X_a)(x_b-X_b)      */
  double D;              /* (sqrt l+ - sqrt l-)/(sqrt l+ + sqrt l-) of I     */
  double theta_deg;      /* atan2(2 I_xz, I_xx - I_zz)/2 in degrees          */
  double Lp;             /* x_max - x_min + 1 over nodes with phi > 0        */
  double umax;           /* max |u| of the physical velocity                 */
  double trC_max;        /* max tr C                                          */
  int32_t n_components;  /* droplet pieces >= 1% of the initial droplet
                            volume (6-connected, periodic x, y); -1 if not
                            requested                                         */
  int32_t piece_nodes[4];/* node counts of the largest such pieces in
                            descending order (0 past n_components or if not
                            requested): the daughter-size spread of a
                            break-up (Section 3)                              */
  int32_t status;        /* LBM_OK, LBM_ENAN or LBM_EFENE for this run       */
} lbm_obs;

/* Launch shape of the step kernel (chosen by the autotuner).  A tile is
 * bx * by columns of nodes advanced by one workgroup of 2 * bx * by threads
 * (one half per component), which marches up bz planes in z; persistent > 0
 * caps the grid at that many workgroups (rounded down to a multiple of 8, at
 * least 8), which then loop over the tile table.  The kernel reads a run's
 * population arrays from one base when its 19 arrays of one component span
 * less than 4 GiB, and from a base per group of four arrays otherwise;
 * grouped = 1 takes the grouped addressing for every run (same results). */
typedef struct {
  int32_t bx, by;        /* (32,8) (16,16) (16,8) (8,16); FP64 (16,8) (8,16) */
  int32_t bz;            /* planes per tile, 1 <= bz <= 1024; 0: each tile
                            spans its run's whole height                      */
  int32_t persistent;    /* 0 = one workgroup per tile                        */
  int32_t grouped;       /* 0 = as the run sizes need, 1 = always grouped     */
} lbm_launch;

typedef struct lbm_ctx lbm_ctx;

const char* lbm_strerror(int code);

/* Host-only validation of one parameter set; touches no device. */
int lbm_validate(const lbm_params* p);

/* ---- single run -------------------------------------------------------
 * Equivalent to the batched calls below with nruns = 1. */
int lbm_workspace_bytes(const lbm_params* p, size_t* bytes);
/* Initialise the set-up of Section 3 (a spherical droplet at mid-gap, shear
 * started from rest): sphere |x - c|^2 < R^2 holds rho_A = rho_major,
 * rho_B = rho_minor, the rest the reverse; f = w_i rho_s (fluid at rest);
 * C = I.  workspace_dev: device memory of at least lbm_workspace_bytes,
 * owned by the caller until lbm_destroy (else LBM_ENOMEM); hip_stream: the
 * caller's stream.  Enqueued on the stream; returns after enqueueing. */
int lbm_init(const lbm_params* p, void* workspace_dev, size_t bytes,
             void* hip_stream, lbm_ctx** out);
/* Advance nsteps >= 0 steps of the coupled scheme (asynchronous): the
 * lattice-Boltzmann steps of the two components with the Shan-Chen and
 * polymer forces (Section 2, Eqs. (1) and (3)), then the FENE-P update of C
 * (Eqs. (2) and (4)), with the moving walls of Section 3.  Faults surface
 * at the next observe. */
int lbm_step(lbm_ctx* ctx, int32_t nsteps);
/* Observables of run 0 (the quantities the paper reports in Section 3:
 * deformation and orientation of the droplet, its projected length L_p in
 * the flow direction as in Fig. 4, and break-up into pieces), reduced in
 * FP64 with a fixed order; synchronises.  want_components != 0 also labels
 * the droplet's connected components.  Returns LBM_ENAN / LBM_EFENE when the
 * run's status word is set (out is still filled). */
int lbm_observe(lbm_ctx* ctx, int32_t want_components, lbm_obs* out);
/* Copy a field of run 0 to / from a host FP64 buffer of n elements (the
 * exact element count of the field, else LBM_EINVAL); synchronises.  Only F
 * and C can be imported.  Populations are held as
 * g_i = f_i - w_i (rho_s(x) + 3 c_i.j_s(x)) against the node's density and
 * momentum: export of F decodes them in FP64; import of F sets
 * rho_s = sum_i f_i and j_s = sum_i c_i f_i (FP64, rounded to the field
 * type) and the shifted values against them.  Status is cleared on import.
 * An F export/import round trip is exact up to that rounding; for a
 * bit-exact restart use lbm_batch_save_state / lbm_batch_load_state. */
int lbm_export(lbm_ctx* ctx, int32_t field, double* host, size_t n);
int lbm_import(lbm_ctx* ctx, int32_t field, const double* host, size_t n);
void lbm_destroy(lbm_ctx* ctx);

/* ---- launch shape ----------------------------------------------------- */
int lbm_get_launch(const lbm_ctx* ctx, lbm_launch* out);
int lbm_set_launch(lbm_ctx* ctx, const lbm_launch* in);
/* Advance every run by nsteps with eager launches and HIP events around
 * each launch of the step kernel; *ms_step receives the summed kernel
 * durations in milliseconds (for roofline accounting).  Synchronises. */
int lbm_step_profiled(lbm_ctx* ctx, int32_t nsteps, double* ms_step);
/* Steps actually taken by run r since init. */
int lbm_steps_done(const lbm_ctx* ctx, int32_t run, int64_t* out);

/* ---- batched independent runs (uneven boxes, one precision) ------------
 * All runs share the context's stream and precision (taken from runs[0]);
 * each run has its own box and parameters. */
int lbm_batch_workspace_bytes(const lbm_params* runs, int32_t nruns,
                              size_t* bytes);
int lbm_batch_init(const lbm_params* runs, int32_t nruns,
                   void* workspace_dev, size_t bytes, void* hip_stream,
                   lbm_ctx** out);
/* Advance run r by steps_per_run[r] >= 0 steps.  All runs advance together
 * through one HIP-graph replay sequence; a run that has taken its steps is
 * masked for the remaining launches. */
int lbm_batch_step(lbm_ctx* ctx, const int32_t* steps_per_run);
/* Observables of every run into out[nruns]; synchronises.  Returns the first
 * non-OK run status (each out[r].status holds its own). */
int lbm_batch_observe(lbm_ctx* ctx, int32_t want_components, lbm_obs* out);
int lbm_batch_export(lbm_ctx* ctx, int32_t run, int32_t field, double* host,
                     size_t n);
int lbm_batch_import(lbm_ctx* ctx, int32_t run, int32_t field,
                     const double* host, size_t n);
int32_t lbm_batch_nruns(const lbm_ctx* ctx);

/* ---- checkpoint / restart ------------------------------------------------
 * The raw state of one run: populations as stored, node densities, momenta
 * and C, behind a header (precision, box, viscoelastic phase, step count).
 * A load restores the run bit for bit, including its step count, into a
 * context of the same precision whose run has the same box and viscoelastic
 * phase (else LBM_EINVAL), and clears the run's status.
 * The host buffer is the caller's; bytes must equal lbm_batch_state_bytes.
 * Both synchronise the context's stream. */
int lbm_batch_state_bytes(const lbm_ctx* ctx, int32_t run, size_t* bytes);
int lbm_batch_save_state(lbm_ctx* ctx, int32_t run, void* host, size_t bytes);
int lbm_batch_load_state(lbm_ctx* ctx, int32_t run, const void* host,
                         size_t bytes);

#ifdef __cplusplus
}
#endif
#endif /* LBMVE_H */
