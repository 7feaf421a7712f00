/*
 * lbm_mlp.h -- C ABI of the sigma surrogate network.
 *
 * Purpose: the paper picks the constant sigma of its improved forcing scheme
 * (Sec. IV.B, Eq. 31) by running simulations with different sigma and keeping
 * the one whose coexistence densities fit the Maxwell construction (Eq. 7).
 * This network learns that map from batched lattice runs, so that sigma can be
 * proposed for a new (T/Tc, tau) and then checked by a lattice run.
 *
 * Network: 3 -> 64 -> 64 -> 2, GELU (exact, erf form) after the two hidden
 * layers.  Inputs (T/Tc, tau, sigma) and outputs (log rho_l, log rho_g) are
 * standardised with the caller's mean and standard deviation.  Every matrix
 * product rounds both operands to bfloat16 (round to nearest even) and
 * accumulates in FP32; the 64x64 products run on MFMA.  Parameters are FP32
 * master weights in one vector of 4546 floats: W1 (64x3, row = output unit),
 * b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2).
 * Loss: sum over rows and outputs of (y - t)^2 / (2 B) in standardised units.
 * Optimiser: Adam (Kingma and Ba, 2015).
 *
 * Memory: device workspace owned by the caller (mlp_workspace_bytes); batch
 * arrays are device pointers, row-major (X: B x 3, targets and outputs:
 * B x 2, FP32).  Work is enqueued on the caller's stream; the functions that
 * return values to host memory synchronise.  Status codes as in lbm.h.
 */
#ifndef LBM_MLP_H
#define LBM_MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLP_NPARAMS 4546

typedef struct mlp_ctx mlp_ctx;

typedef struct {
  float in_mean[3], in_std[3];    /* (T/Tc, tau, sigma) */
  float out_mean[2], out_std[2];  /* (log rho_l, log rho_g) */
} mlp_norm;

/* Workspace for batches of up to max_batch rows (max_batch >= 1). */
int mlp_workspace_bytes(int32_t max_batch, size_t* bytes);

/* host_params: MLP_NPARAMS floats (initial weights); Adam moments start at 0. */
int mlp_init(const float* host_params, const mlp_norm* norm, int32_t max_batch, void* dev_workspace,
             size_t ws_bytes, void* hip_stream, mlp_ctx** out);

/* Replace the parameters (and reset Adam) / copy them to host (synchronous). */
int mlp_set_params(mlp_ctx* c, const float* host_params);
int mlp_get_params(mlp_ctx* c, float* host_params);
int mlp_set_norm(mlp_ctx* c, const mlp_norm* norm);

/* Y = network(X) in output units (log rho_l, log rho_g); 1 <= B <= max_batch. */
int mlp_forward(mlp_ctx* c, const float* dev_X, float* dev_Y, int32_t B);

/* Gradient of the loss for targets dev_T (log rho) into dev_grad (MLP_NPARAMS
 * floats) and the loss into dev_loss (1 float); deterministic (fixed-order
 * reductions, no atomics). */
int mlp_gradient(mlp_ctx* c, const float* dev_X, const float* dev_T, int32_t B, float* dev_grad,
                 float* dev_loss);

/* One Adam step with the gradient in dev_grad (step count kept by the context). */
int mlp_adam(mlp_ctx* c, const float* dev_grad, float lr, float beta1, float beta2, float eps);

/* Gradient + Adam (beta1 0.9, beta2 0.999, eps 1e-8); loss to dev_loss (nullable). */
int mlp_train_step(mlp_ctx* c, const float* dev_X, const float* dev_T, int32_t B, float lr,
                   float* dev_loss);

int mlp_destroy(mlp_ctx* c);

#ifdef __cplusplus
}
#endif
#endif /* LBM_MLP_H */
