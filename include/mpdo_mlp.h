/* Surrogate MLP of the simulator: (QAOA angles, noise rates) -> (energy per site, success
 * probability), trained on the simulator's own outputs.  Forward, backward and optimiser run
 * on the GPU in the library's own kernels: FP32 parameters and activations, BF16 matrix-core
 * products with FP32 accumulation.
 *
 * Network: h_0 = x; z_l = h_l W_l^T + b_l; h_{l+1} = tanh(z_l) on hidden layers; the output
 * layer is linear.  W_l is widths[l+1] x widths[l], row-major.  Parameters are packed as
 * W_0, b_0, W_1, b_1, ... (float, host).  Loss: mean squared error over batch and outputs.
 * Optimiser: Adam (beta1 0.9, beta2 0.999, eps 1e-8), bias-corrected.
 *
 * Host arrays are row-major, batch x width, and are copied before a call returns.  Calls
 * that return host data synchronise the handle's stream.  Status codes as in mpdo.h:
 *   MPDO_E_ARG    bad sizes, a batch above max_batch, null pointers, non-finite inputs;
 *   MPDO_E_NOMEM  device or pinned allocation failed;
 *   MPDO_E_DEVICE a HIP error.
 * mpdo_mlp_last_error() describes the last failure. */
#ifndef MPDO_MLP_H
#define MPDO_MLP_H

#include <stddef.h>

#include "mpdo.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mpdo_mlp_s* mpdo_mlp;

/* Number of packed parameters of a network with n_layers layers and widths[0..n_layers]. */
size_t mpdo_mlp_param_count(int n_layers, const int* widths);

/* Create a network (parameters zero, Adam state zero).  Device memory for max_batch rows is
 * allocated here and owned by the handle.  hip_stream may be null (the default stream). */
mpdo_status mpdo_mlp_create(int n_layers, const int* widths, int max_batch, void* hip_stream,
                            mpdo_mlp* out);
mpdo_status mpdo_mlp_destroy(mpdo_mlp net);

/* Set all parameters (resets the Adam state) / read them back. */
mpdo_status mpdo_mlp_set_params(mpdo_mlp net, const float* params);
mpdo_status mpdo_mlp_get_params(mpdo_mlp net, float* params);

/* y (batch x widths[L]) = network(x (batch x widths[0])). */
mpdo_status mpdo_mlp_forward(mpdo_mlp net, int batch, const float* x, float* y);

/* MSE loss against targets t and its gradient with respect to the packed parameters
 * (grads may be null: the gradient then stays on the device). */
mpdo_status mpdo_mlp_loss_grad(mpdo_mlp net, int batch, const float* x, const float* t,
                               float* loss, float* grads);

/* One Adam step of size lr on the loss of this batch; *loss (may be null) is the loss
 * before the step. */
mpdo_status mpdo_mlp_train_step(mpdo_mlp net, int batch, const float* x, const float* t,
                                float lr, float* loss);

/* Gradient with respect to the inputs of sum_k w_out[k] y[:, k], per row: dx (batch x
 * widths[0]); y (may be null) receives the outputs.  Used to search over the inputs. */
mpdo_status mpdo_mlp_input_grad(mpdo_mlp net, int batch, const float* x, const float* w_out,
                                float* y, float* dx);

const char* mpdo_mlp_last_error(mpdo_mlp net);

#ifdef __cplusplus
}
#endif

#endif /* MPDO_MLP_H */
