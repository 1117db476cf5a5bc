/*
 * pdhcg_mlp.h -- C ABI of the warm-start network for parametric QP families.
 *
 * A multilayer perceptron n_in -> n_hid -> n_hid -> n_out (ReLU on the two
 * hidden layers, linear output) that maps the parameter of a QP family to a
 * predicted primal-dual pair (x, y), used as the start point of restarted
 * PDHCG.  Weights and activations are bfloat16 in the matrix products (MFMA,
 * FP32 accumulation); FP32 master weights are updated by Adam.  Training and
 * inference run in the library's HIP kernels.
 *
 * Parameter packing (FP32, used by set/get and by the gradient output):
 * W1 (n_in x n_hid, row-major), b1 (n_hid), W2 (n_hid x n_hid), b2 (n_hid),
 * W3 (n_hid x n_out), b3 (n_out); a layer maps a row batch H to H W + b.
 *
 * Conventions: return 0 on success or a negative PDHCG_ERR_* code (see
 * pdhcg.h); pdhcg_last_error() gives the message.  X, T and Y are FP32
 * row-major device arrays (batch rows).  All work is issued on the stream
 * given at creation; each call returns after that stream has finished,
 * except pdhcg_mlp_train_step, which only queues its work (its arrays must
 * stay valid until the stream reaches it).  The handle owns its device
 * buffers; it is not thread-safe.
 */
#ifndef PDHCG_MLP_H
#define PDHCG_MLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdhcg_mlp pdhcg_mlp;

/* Allocate a network and its workspace for batches of up to max_batch rows.
 * Weights start at zero: call pdhcg_mlp_set_params before use. */
int pdhcg_mlp_create(pdhcg_mlp** h, int32_t n_in, int32_t n_hid, int32_t n_out, int32_t max_batch,
                     void* hip_stream);

/* Number of FP32 values in the packed parameter vector. */
int64_t pdhcg_mlp_num_params(const pdhcg_mlp* h);

/* Copy packed FP32 parameters from / to host memory; set also resets Adam. */
int pdhcg_mlp_set_params(pdhcg_mlp* h, const float* params);
int pdhcg_mlp_get_params(const pdhcg_mlp* h, float* params);

/* Y (batch x n_out, FP32) = network(X (batch x n_in)). */
int pdhcg_mlp_forward(pdhcg_mlp* h, const float* X, int32_t batch, float* Y);

/* A start point for `batch` members of a parametric family, on the device:
 * Z = network(X) (X: batch x n_in FP32, any batch size; run in chunks of
 * max_batch rows), each output column de-standardised as z * out_sd + out_mu
 * (FP64, product and sum rounded separately), then columns 0..n-1 are x and
 * the rest encode y: column n + p (p < n_pair) holds the multiplier lam of the
 * p-th equality row pair, y[plus[p]] = max(lam, 0), y[minus[p]] = max(-lam, 0);
 * column n + n_pair + q holds y[rest[q]] before its projection max(., 0).
 * out_mu, out_sd: n_out FP64 device arrays; plus, minus (n_pair) and rest
 * (n_rest): int32 device arrays of rows of y, every row 0..m-1 exactly once;
 * x0 (batch x n) and y0 (batch x m): FP64 row-major device outputs (the
 * packed start points of a batch of same-sized members).  INVALID_ARGUMENT
 * unless n + n_pair + n_rest = n_out and 2 n_pair + n_rest = m. */
int pdhcg_mlp_predict_start(pdhcg_mlp* h, const float* X, int32_t batch, const double* out_mu,
                            const double* out_sd, int32_t n, int32_t n_pair, const int32_t* plus,
                            const int32_t* minus, int32_t n_rest, const int32_t* rest, int32_t m, double* x0,
                            double* y0);

/* Mean-squared-error loss of network(X) against targets T (batch x n_out)
 * and its gradient with respect to every parameter (kept on the device for
 * pdhcg_mlp_adam_step; copied to host `grads` in the packed layout unless
 * grads is NULL).  *loss receives the loss (may be NULL). */
int pdhcg_mlp_loss_grad(pdhcg_mlp* h, const float* X, const float* T, int32_t batch, float* loss, float* grads);

/* One Adam step with the gradient of the last pdhcg_mlp_loss_grad call. */
int pdhcg_mlp_adam_step(pdhcg_mlp* h, float lr, float beta1, float beta2, float eps);

/* One training step queued on the network's stream without waiting: the
 * loss and gradient of pdhcg_mlp_loss_grad on the rows rows[0..batch) of X
 * (n_in per row) and T (n_out per row) -- rows is an int32 device array, or
 * NULL for the first batch rows -- then one Adam step.  The minibatch is
 * gathered by the library's own kernels.  The step's loss is added to the
 * running sum that pdhcg_mlp_take_loss returns. */
int pdhcg_mlp_train_step(pdhcg_mlp* h, const float* X, const float* T, const int32_t* rows, int32_t batch, float lr,
                         float beta1, float beta2, float eps);

/* Wait for the stream; *sum receives the sum of the losses of the
 * pdhcg_mlp_train_step and pdhcg_mlp_loss_grad calls since the last call (or
 * since creation) and *steps their number; both are then reset.  Either
 * pointer may be NULL. */
int pdhcg_mlp_take_loss(pdhcg_mlp* h, double* sum, int64_t* steps);

void pdhcg_mlp_destroy(pdhcg_mlp* h);

#ifdef __cplusplus
}
#endif

#endif /* PDHCG_MLP_H */
