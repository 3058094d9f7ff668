/*
 * lbmve surrogate — a small learned model that proposes where to bracket the
 * critical capillary number Ca_cr of droplet break-up (the quantity the
 * paper locates by pre/post-critical wall speeds, Section 3).  The plain
 * simulation stays the arbiter: every proposal is verified by full runs.
 *
 * Network: inputs (Ca, De, lambda, 2R/W, L^2, polymer fraction) -- the
 * dimensionless groups of Sections 2-3, z-scored by the caller -- through
 * 6 -> 128 -> 128 -> 3 with tanh hidden units to (steady D, orientation,
 * break-up logit).  Weights and biases are used in bfloat16 (round to nearest
 * even) with float32 accumulation; a float32 master copy is updated by Adam.
 *
 * Loss on n rows: (1/n) sum_r [ m_r ((z0-t0)^2 + (z1-t1)^2)/2
 *                               + softplus(z2) - t2 z2 ]
 * with m_r = 1 for runs that did not break (deformation and angle are
 * undefined after break-up) and t2 in {0, 1} the break-up label.
 *
 * Parameter vector (float32, sg_param_count() entries): W1[6][128], b1[128],
 * W2[128][128], b2[128], W3[128][3], b3[3]; W[k][j] multiplies input k into
 * unit j.  Row-major device arrays: x[n][6], targets t[n][3], mask m[n],
 * outputs z[n][3], all float32.
 *
 * Ownership and errors as in lbmve.h: the caller owns the device workspace
 * and the stream; calls return LBM_OK (0) or a negative LBM_E* code;
 * n must be in [1, batch_max] (else LBM_EINVAL).
 */
#ifndef LBMVE_SURROGATE_H
#define LBMVE_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sg_ctx sg_ctx;

int32_t sg_param_count(void);
int sg_workspace_bytes(int32_t batch_max, size_t* bytes);
int sg_init(int32_t batch_max, void* workspace_dev, size_t bytes, void* hip_stream, sg_ctx** out);
/* Load float32 master parameters (host); resets the Adam state. */
int sg_set_params(sg_ctx* s, const float* host, size_t n);
/* Copy the float32 master parameters, or their bfloat16-rounded working copy
 * widened to float32, to the host. */
int sg_get_params(sg_ctx* s, float* host, size_t n);
int sg_get_working_params(sg_ctx* s, float* host, size_t n);
/* z_dev[n][3] = network(x_dev[n][6]) with the working (bf16) parameters.
 * Asynchronous on the context's stream. */
int sg_forward(sg_ctx* s, const float* x_dev, int32_t n, float* z_dev);
/* Loss and its gradient w.r.t. the parameters (at the working parameters)
 * into grad_host[sg_param_count()] and *loss_host; synchronises. */
int sg_gradient(sg_ctx* s, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                float* grad_host, float* loss_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the loss of the batch;
 * *loss_host receives the loss before the update; synchronises. */
int sg_train_step(sg_ctx* s, const float* x_dev, const float* t_dev, const float* m_dev, int32_t n,
                  float lr, float* loss_host);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the loss
 * and gradient of sg_gradient, written to caller-owned float32 device buffers
 * grad_dev[sg_param_count()] and loss_dev[1] instead of host memory.  The
 * per-row intermediates (activations, deltas, row losses) live in a fixed
 * device array of the library (about 2 MB on each GPU it runs on, kept until
 * the process ends), not in the context's workspace: n must be in
 * [1, SG_NOALLOC_MAX_ROWS] (else LBM_EINVAL).  Asynchronous on the context's
 * stream; allocates nothing and does not synchronise.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (on different
 * streams) race.  Results are bit-identical to sg_gradient's. */
#define SG_NOALLOC_MAX_ROWS 1024
int sg_gradient_noalloc(sg_ctx* s, const float* x_dev, const float* t_dev, const float* m_dev,
                        int32_t n, float* grad_dev, float* loss_dev);
void sg_destroy(sg_ctx* s);

#ifdef __cplusplus
}
#endif
#endif /* LBMVE_SURROGATE_H */
