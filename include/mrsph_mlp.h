/* C-ABI of the sub-step surrogate network (gfx950, BF16 matrix cores with
 * FP32 accumulation).
 *
 * A per-solid-particle multilayer perceptron in_dim -> 128 -> 128 -> 128 ->
 * out_dim with SiLU (z sigmoid(z)) after each hidden layer and a linear
 * output.  It is trained on trajectories of the plain method and predicts the
 * time-averaged velocity and acceleration of a solid particle over one
 * acoustic step in place of the kappa sub-steps (the learned extension of the
 * paper's multi-time-step scheme, Section 3.2; the paper itself has no
 * learned part).
 *
 * Precision: FP32 master weights, Adam moments and gradients; the operands of
 * every matrix product (layer inputs, weights, back-propagated errors) are
 * rounded to bfloat16 (nearest, ties to even) and multiplied on the matrix
 * cores with FP32 accumulation; biases, SiLU and the loss are FP32.
 *
 * Memory: the caller owns all device memory (one arena sized by
 * mlp_arena_bytes).  Matrices are row-major FP32 unless stated.  Calls enqueue
 * on the caller's stream unless they say they synchronise.  Status codes are
 * those of mrsph.h (0 = OK, -1 argument, -2 HIP, -3 order).
 */
#ifndef MRSPH_MLP_H
#define MRSPH_MLP_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mlp_ctx mlp_ctx;

/* Bytes of device memory for a network with in_dim <= 32 inputs, out_dim <=
 * 16 outputs and up to max_rows rows per call (0 for invalid sizes). */
size_t mlp_arena_bytes(int in_dim, int out_dim, int max_rows);

/* Create a network in the caller's arena (weights zero until mlp_set_params).
 * stream is a hipStream_t (NULL = default stream). */
int mlp_init(int in_dim, int out_dim, int max_rows, void *dev_arena, size_t arena_bytes, void *stream,
             mlp_ctx **out);

/* Number of parameters: in*128 + 128 + 2*(128*128 + 128) + 128*out + out. */
size_t mlp_param_count(const mlp_ctx *m);

/* Host FP32 parameters in the order W1, b1, W2, b2, W3, b3, W4, b4, each W
 * row-major (fan_in x fan_out).  n must equal mlp_param_count.  Setting the
 * parameters resets the Adam moments and step.  Both synchronise. */
int mlp_set_params(mlp_ctx *m, const float *host, size_t n);
int mlp_get_params(mlp_ctx *m, float *host, size_t n);

/* Inference: y (rows x out_dim, device) = network(x (rows x in_dim, device)),
 * 1 <= rows <= max_rows. */
int mlp_forward(mlp_ctx *m, const float *x_dev, float *y_dev, int rows);

/* Forward with stored activations, loss L = 0.5 mean_rows sum_cols (y - t)^2
 * and back-propagation of its gradient into the gradient buffers (replaced,
 * not accumulated).  t is rows x out_dim on the device.  loss_host (may be
 * NULL) receives L, which synchronises. */
int mlp_backward(mlp_ctx *m, const float *x_dev, const float *t_dev, int rows, double *loss_host);

/* Copy the gradients of the last mlp_backward to host memory, in the
 * parameter order of mlp_set_params.  Synchronises. */
int mlp_get_grads(mlp_ctx *m, float *host, size_t n);

/* One Adam step (bias-corrected moments, Kingma & Ba) on the FP32 master
 * parameters with the last gradients; refreshes the bfloat16 copies. */
int mlp_adam(mlp_ctx *m, float lr, float beta1, float beta2, float eps);

/* Training step: mlp_backward followed by mlp_adam. */
int mlp_train_step(mlp_ctx *m, const float *x_dev, const float *t_dev, int rows, float lr, float beta1,
                   float beta2, float eps, double *loss_host);

int mlp_sync(mlp_ctx *m);
void mlp_destroy(mlp_ctx *m);

#ifdef __cplusplus
}
#endif

#endif
