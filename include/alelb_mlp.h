/*
 * alelb_mlp.h -- C-ABI of the surrogate network trained on the solver's force
 * histories: a fully connected network (tanh hidden layers, linear output)
 * whose forward and backward passes run as BF16 matrix-core (MFMA) products
 * with FP32 accumulation on gfx950, trained by Adam on the GPU.
 *
 * The network maps a case's motion and flow parameters to its lift and
 * moment coefficient histories; the ALE lattice-Boltzmann solver of
 * alelb.h produces the training data and remains the reference (the
 * surrogate's error is measured against it, and it is the fallback).
 *
 * Conventions:
 *   widths[0] inputs, widths[n-1] outputs, n >= 2; layer l maps widths[l] to
 *   widths[l+1]; hidden layers apply tanh, the last layer is linear.
 *   Parameters (host, FP32) are packed layer by layer: W_l [widths[l+1]][widths[l]]
 *   row-major, then b_l [widths[l+1]].
 *   Batches are row-major [batch][features], FP32.
 *   Loss: mean squared error over the batch and the outputs,
 *   L = sum (y - t)^2 / (batch * outputs).
 * Products: every layer's inputs (activations, weights, back-propagated
 * errors) are rounded to BF16 (round to nearest even) and multiplied with FP32
 * accumulation; biases, activations kept for the backward pass, gradients,
 * master weights and Adam moments are FP32.
 *
 * All functions return an int status (0 = OK, < 0 = ALE_LB_E* of alelb.h);
 * the message of the last failure is ale_lb_last_error().  The handle owns its
 * device memory (hipMalloc) and runs on the stream given at create (NULL = the
 * null stream); every call returns after that stream has drained.
 */
#ifndef ALELB_MLP_H
#define ALELB_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ale_mlp ale_mlp_t; /* opaque handle */

/* Network of n_widths layers' widths (each 1..4096, at most 16 layers) for
 * batches of up to max_batch rows (1..4194240 = 65535 tiles of 64 rows).
 * Parameters start at zero: set them with ale_mlp_set_params().  EINVAL for
 * a bad shape, ENOMEM when device memory runs out. */
int ale_mlp_create(const int32_t *widths, int32_t n_widths, int32_t max_batch, void *stream, ale_mlp_t **out);
void ale_mlp_destroy(ale_mlp_t *h);

/* number of parameters, out[0]; out[1] Adam steps taken */
int ale_mlp_info(ale_mlp_t *h, int64_t *out, int32_t n);

/* Copy the n FP32 parameters in (and reset the Adam moments) / out. */
int ale_mlp_set_params(ale_mlp_t *h, const float *params, int64_t n);
int ale_mlp_get_params(ale_mlp_t *h, float *params, int64_t n);

/* y [batch][outputs] = network(x [batch][inputs]).  on_device != 0: x and y
 * are device pointers; else host pointers. */
int ale_mlp_forward(ale_mlp_t *h, const float *x, int32_t batch, float *y, int32_t on_device);

/* Loss and its gradient with respect to every parameter (host FP32, packed
 * like the parameters) for the batch (x, t); no update.  on_device refers to
 * x and t; grads and loss are host pointers (loss may be NULL). */
int ale_mlp_gradients(ale_mlp_t *h, const float *x, const float *t, int32_t batch, float *grads, double *loss,
                      int32_t on_device);

/* One Adam step (Kingma & Ba) on the batch's loss gradient:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps), k = steps taken.
 * *loss (may be NULL) receives the loss before the step. */
int ale_mlp_train_step(ale_mlp_t *h, const float *x, const float *t, int32_t batch, float lr, float beta1,
                       float beta2, float eps, double *loss, int32_t on_device);

/* n Adam steps on one batch (x, t), with learning rate lr[k] (host array of
 * n) at step k: the same arithmetic, in the same order, as n calls of
 * ale_mlp_train_step, without a host synchronization per step.  The batch is
 * staged once.  losses (host array of n, or NULL) receives each step's loss
 * before its update, copied back every 1024 steps.  EINVAL for a null
 * pointer, n < 1, a batch outside 1..max_batch or bad hyper-parameters (the
 * parameters are then unchanged). */
int ale_mlp_train_steps(ale_mlp_t *h, const float *x, const float *t, int32_t batch, int32_t n, const float *lr,
                        float beta1, float beta2, float eps, double *losses, int32_t on_device);

/* The network's matrix product on its own (tests): C [M][N] (FP32, device) =
 * A [M][K] B [K][N] with A and B device arrays of BF16 bit patterns,
 * row-major, FP32 accumulation.  Runs on the null stream. */
int ale_mlp_gemm_bf16(const uint16_t *A, const uint16_t *B, float *C, int32_t M, int32_t N, int32_t K);

#ifdef __cplusplus
}
#endif
#endif /* ALELB_MLP_H */
