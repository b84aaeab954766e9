/*
 * hprqp_mlp.h -- C ABI of the warm-start surrogate in libhprqp.so: a
 * fully connected network x -> GELU(W1 x + b1) -> GELU(W2 h + b2) -> W3 h + b3
 * that maps the parameters of a parametric QP family to a starting point
 * (y, z, w) of HPR-QP.  The surrogate only changes the starting point of
 * Algorithm 4; the solver itself stays FP64 and decides convergence.
 *
 * Arithmetic: GEMM operands (inputs, activations, weights, back-propagated
 * gradients) are rounded to BF16 (round to nearest even) and multiplied on
 * the gfx950 matrix cores (v_mfma_f32_32x32x16_bf16) with FP32
 * accumulation; biases, GELU, the loss and Adam run in FP32 on FP32 master
 * weights.
 *
 * Parameter vector (FP32, flat): W1 (h1 x n_in, row-major: output-major,
 * like a y = W x layer), b1 (h1), W2 (h2 x h1), b2 (h2), W3 (n_out x h2), b3.
 * Activations are row-major (batch x features).  All data pointers are
 * DEVICE pointers unless the name ends in _host.  Errors: see hprqp.h
 * (hprqp_status, hprqp_last_error).
 */
#ifndef HPRQP_MLP_H
#define HPRQP_MLP_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>
#include "hprqp.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hprqp_mlp hprqp_mlp;

/* dims = {n_in, h1, h2, n_out}; max_batch bounds the batch of every call;
 * params_host: initial FP32 parameter vector (NULL: all zeros). */
hprqp_status hprqp_mlp_create(const int32_t dims[4], int32_t max_batch, const float *params_host,
                              hipStream_t stream, hprqp_mlp **out);

/* Number of parameters (length of the flat vector). */
int64_t hprqp_mlp_num_params(const hprqp_mlp *net);

/* Y (batch x n_out, FP32) = network(X (batch x n_in, FP32)). */
hprqp_status hprqp_mlp_forward(hprqp_mlp *net, int32_t batch, const float *X, float *Y);

/* Forward + backward of the weighted mean-squared error
 *   loss = sum_{b,j} out_w[j] (Y[b,j] - T[b,j])^2 / (batch * n_out)
 * (out_w may be NULL: all ones).  The gradient (same layout as the
 * parameter vector) is kept for hprqp_mlp_adam and copied to grad (device,
 * may be NULL); loss_host may be NULL. */
hprqp_status hprqp_mlp_loss_grad(hprqp_mlp *net, int32_t batch, const float *X, const float *T,
                                 const float *out_w, float *loss_host, float *grad);

/* Per-feature standardization applied inside the library (host arrays):
 * the network sees (x - in_mean)/in_std and is trained on (t - out_mean)/out_std;
 * hprqp_mlp_forward returns out_mean + out_std * output.  A std <= 1e-12
 * marks a constant feature (scaled to 0).  Default: identity. */
hprqp_status hprqp_mlp_set_scaling(hprqp_mlp *net, const float *in_mean, const float *in_std,
                                   const float *out_mean, const float *out_std);

/* Warm start of HPR-QP for `batch` family members from their parameter
 * vectors X: with the prediction (y, z, w) = forward(X) (n_out = m + 2n),
 * writes the FP64 starting point y0 = y (batch x m), w0 = w and
 * x0 = Pi_C(w) = clamp(w, L, U) (batch x n each; the z part is not used by
 * Algorithm 4).  bad[s] = 1 flags a sample whose prediction is not finite:
 * the caller starts it cold instead. */
hprqp_status hprqp_mlp_warm_start(hprqp_mlp *net, int32_t batch, const float *X, int32_t n, int32_t m,
                                  const double *L, const double *U, double *y0, double *w0, double *x0,
                                  int32_t *bad);

/* One Adam step (bias-corrected) on the FP32 master parameters with the
 * last gradient; refreshes the BF16 weight copies. */
hprqp_status hprqp_mlp_adam(hprqp_mlp *net, float lr, float beta1, float beta2, float eps);

hprqp_status hprqp_mlp_get_params(hprqp_mlp *net, float *params_host);
hprqp_status hprqp_mlp_set_params(hprqp_mlp *net, const float *params_host);

/* Time (HIP events, ms) and useful FLOPs of the GEMM launches of the last
 * forward / loss_grad call. */
hprqp_status hprqp_mlp_gemm_stats(hprqp_mlp *net, double *ms_host, double *flop_host);

void hprqp_mlp_destroy(hprqp_mlp *net);

/* Plain BF16 GEMM with FP32 accumulation on the matrix cores (exposed for
 * tests): C[i*ldc + j] (+)= sum_k A[i*a_rs + k*a_cs] * B[k*b_rs + j*b_cs],
 * A, B stored as BF16 bit patterns; accumulate = 1 adds to C. */
hprqp_status hprqp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t a_rs, int64_t a_cs,
                             const uint16_t *B, int64_t b_rs, int64_t b_cs, float *C, int64_t ldc,
                             int32_t accumulate, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HPRQP_MLP_H */
