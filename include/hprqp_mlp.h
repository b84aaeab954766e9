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

/* Standardization from training data: the column means and standard
 * deviations (divisor rows - 1) of X (rows x n_in) and T (rows x n_out,
 * device, FP32), accumulated in FP64 on the device in a fixed order, set as by
 * hprqp_mlp_set_scaling.  stats_host (may be NULL) receives them as
 * [in_mean, in_std, out_mean, out_std] (2 n_in + 2 n_out floats). */
hprqp_status hprqp_mlp_fit_scaling(hprqp_mlp *net, int64_t rows, const float *X, const float *T,
                                   float *stats_host);

/* Network input of `batch` family members: X[s] = [c_s (n); u_s (m)] as FP32
 * (c: batch x n, u: batch x m, FP64, concatenated by member; X: batch x (n+m)). */
hprqp_status hprqp_family_features(int32_t batch, int32_t n, int32_t m, const double *c, const double *u,
                                   float *X, hipStream_t stream);

/* Training targets: T[s] = [y_s (m); z_s (n); w_s (n)] as FP32 from the FP64
 * solutions (concatenated by member), T: batch x (m + 2n).  With iters (device,
 * batch entries, the iteration count of the solve that produced each
 * solution; may be NULL) T has one more column, log(max(iters_s, 1)): the
 * network then also learns the length of a member's solve. */
hprqp_status hprqp_family_targets(int32_t batch, int32_t n, int32_t m, const double *y, const double *z,
                                  const double *w, const int64_t *iters, float *T, hipStream_t stream);

/* Warm start of HPR-QP for `batch` family members from their parameter
 * vectors X: with the prediction (y, z, w) = forward(X) (n_out = m + 2n, or
 * m + 2n + 1 with a last column that predicts the log iteration count of the
 * member's solve), writes the FP64 starting point y0 = y (batch x m), w0 = w
 * and x0 = Pi_C(w) = clamp(w, L, U) (batch x n each; the z part is not used
 * by Algorithm 4).  bad[s] = 1 flags a sample whose predicted y or w is not
 * finite: its start is written as the origin (the cold start).  score (device,
 * batch floats, may be NULL; needs n_out = m + 2n + 1) receives the predicted
 * log iteration count, the priority hprqp_batch_set_priority takes to start
 * the longest solves first. */
hprqp_status hprqp_mlp_warm_start(hprqp_mlp *net, int32_t batch, const float *X, int32_t n, int32_t m,
                                  const double *L, const double *U, double *y0, double *w0, double *x0,
                                  int32_t *bad, float *score);

/* One Adam step (bias-corrected) on the FP32 master parameters with the
 * last gradient; refreshes the BF16 weight copies. */
hprqp_status hprqp_mlp_adam(hprqp_mlp *net, float lr, float beta1, float beta2, float eps);

hprqp_status hprqp_mlp_get_params(hprqp_mlp *net, float *params_host);
hprqp_status hprqp_mlp_set_params(hprqp_mlp *net, const float *params_host);

/* Time (HIP events, ms) and useful FLOPs of the GEMM launches of the last
 * forward / loss_grad call. */
hprqp_status hprqp_mlp_gemm_stats(hprqp_mlp *net, double *ms_host, double *flop_host);

void hprqp_mlp_destroy(hprqp_mlp *net);

/* A stage tensor of the last forward / loss_grad call (exposed for tests, so
 * that every stage can be checked with its own inputs), written to out
 * (rows x cols FP32, device; may be NULL to query the shape): which = 0 the
 * standardized input (BF16), 1 Z1 = W1 x + b1, 2 A1 = GELU(Z1) (BF16), 3 Z2,
 * 4 A2 (BF16), 5 the standardized output, 6 dY = d loss / d output (FP32),
 * 7 its BF16 copy, 8 dA2, 9 dZ2 = dA2 * GELU'(Z2), 10 its BF16 copy, 11 dA1,
 * 12 dZ1, 13 its BF16 copy, 14 the standardized targets.  BF16 values are
 * widened exactly.  rows_host / cols_host (may be NULL) receive the shape. */
hprqp_status hprqp_mlp_intermediate(hprqp_mlp *net, int32_t which, float *out, int32_t *rows_host,
                                    int32_t *cols_host);

/* Plain BF16 GEMM with FP32 accumulation on the matrix cores (exposed for
 * tests): C[i*ldc + j] (+)= sum_k A[i*a_rs + k*a_cs] * B[k*b_rs + j*b_cs],
 * A, B stored as BF16 bit patterns; accumulate = 1 adds to C.  split_k in
 * [1, 64]: the K range is cut into that many slices of whole 16-steps, each
 * slice's partial product goes to workspace (device, split_k M N floats;
 * may be NULL when split_k = 1) and a second kernel adds the partials in slice
 * order (deterministic).  The network's own GEMMs choose their split from
 * the shape (enough waves to fill the CUs) and use the handle's workspace. */
hprqp_status hprqp_gemm_bf16(int32_t M, int32_t N, int32_t K, const uint16_t *A, int64_t a_rs, int64_t a_cs,
                             const uint16_t *B, int64_t b_rs, int64_t b_cs, float *C, int64_t ldc,
                             int32_t accumulate, int32_t split_k, float *workspace, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* HPRQP_MLP_H */
