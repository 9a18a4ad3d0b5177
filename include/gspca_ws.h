/*
 * gspca_ws.h -- learned warm start for the iterative PCA library (gspca.h).
 *
 * Not part of the paper: the paper starts component k from a column of the
 * residual (Secs. 2.2-2.3, the pseudo-code's T^(k) <- R^(k)); gspca.h's
 * GSPCA_INIT_GIVEN accepts any start vector instead.  This header produces
 * one per component from a random sketch of X:
 *
 *   Y = X Omega                          M x r, r = 32 or 64, Omega N x r given
 *   Y^T Y = Q diag(g) Q^T                 FP64 Jacobi, g decreasing
 *   Z = sqrt(M) Y Q diag(g)^(-1/2)        whitened rows (unit-variance columns)
 *   [refinement, `power` times: Y = X (X^T Z / sqrt(M)), whiten again -- one
 *    step of subspace iteration (Halko, Martinsson & Tropp 2011, Alg. 4.4),
 *    which turns the sketch's directions into Ritz vectors of X X^T]
 *   o_m = z_m[:d3] + W3^T relu(W2^T relu(W1^T z_m[:32] + b1) + b2) + b3  (row m)
 *   T0[:, k] = (o_0k, ..., o_(M-1)k)      start of component k (sign free)
 *
 * The network is row-wise (the same map for every row and every matrix): the
 * first d3 whitened directions (Ritz vectors of the sketch) plus a learned
 * correction; with W3 = 0 it returns the un-learned sketch start.
 * Products run on bfloat16 matrix cores with FP32 accumulation; rounding
 * points (round to nearest even): the input rows z_m, the weights W1..W3, the
 * stored hidden activations, and in the backward pass the incoming gradient
 * dL/do and the masked hidden gradients.  Biases, outputs and parameter
 * gradients are FP32.  relu'(0) = 0.
 *
 * Training loss for one matrix with converged unit scores v_k (column k of
 * the GS-PCA result T divided by sigma_k):
 *   L = sum_k 1 - (o_k . v_k)^2 / (|o_k|^2 |v_k|^2)
 * (a column with |o_k| = 0 or |v_k| = 0 contributes 1 and no gradient),
 * averaged over the matrices of a step; Adam (Kingma & Ba) on FP32 master
 * weights.
 *
 * All array arguments are device pointers owned by the caller; `stream` is a
 * hipStream_t passed as void*.  Negative status codes come from host-side
 * validation and enqueue nothing.  Nothing here synchronises the stream; no
 * entry point allocates memory.
 */
#ifndef GSPCA_WS_H
#define GSPCA_WS_H

#include "gspca.h"

#ifdef __cplusplus
extern "C" {
#endif

#define GSPCA_WS_RANK 32 /* network input width d0 (the first d0 whitened directions) */
#define GSPCA_WS_RMAX 64 /* widest sketch: r is 32 or 64 */

/* Network state.  Parameters are packed in one FP32 array in the order
 * W1, b1, W2, b2, W3, b3; W_l is row-major d_(l-1) x d_l (W[i*d_l + j] maps
 * input i to output j).  theta_bf16, grad, adam_m and adam_v use the same
 * packing.  d0 must be 32, d1 and d2 in [16, 1024], d3 (the number of
 * components predicted) in [1, 32]. */
typedef struct {
    int32_t d0, d1, d2, d3;
    float *theta;      /* FP32 master parameters (caller initialises)          */
    uint16_t *theta_bf16; /* bfloat16 bit patterns of theta (gspca_mlp_sync)   */
    float *grad;       /* dL/dtheta of the last gspca_mlp_loss_grad             */
    float *adam_m;     /* first moments, zero before the first step             */
    float *adam_v;     /* second moments, zero before the first step            */
    int32_t step;      /* Adam steps taken; gspca_mlp_adam increments it        */
    int32_t pad;
} gspca_mlp;

/* Number of parameters: d0*d1 + d1 + d1*d2 + d2 + d2*d3 + d3. */
int64_t gspca_mlp_param_count(int32_t d0, int32_t d1, int32_t d2, int32_t d3);

/* Workspace of gspca_mlp_forward / gspca_mlp_loss_grad over `rows` rows in
 * `ninst` matrices (cols = 0), and of gspca_ws_predict for an M x N matrix
 * (rows = M, ninst = 1, cols = N).  0 when the sizes or the network widths
 * are invalid (d0 = 32, d1 and d2 in [16, 1024], d3 in [1, 32]). */
size_t gspca_mlp_workspace_bytes(const gspca_mlp *net, int64_t rows, int32_t ninst,
                                 int64_t cols);

/* Y = X Omega.  X FP32 column-major M x N (ldx >= M), Omega FP32 row-major
 * N x r (Omega[j*r + c]), Y FP32 row-major M x r.  r is 32 or 64. */
gspca_status gspca_sketch(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Omega,
                          int32_t r, float *Y, void *stream);

/* Device workspace of gspca_sketch_refine for an M x N matrix and width r;
 * it also covers gspca_whiten_sketch of M rows (0 for invalid sizes). */
size_t gspca_sketch_workspace_bytes(int64_t M, int64_t N, int32_t r);

/* Refinement step: W = X^T Z / sqrt(M) (N x r, row-major; FP32 sums over row
 * slices, added in slice order) and Y = X W (M x r, row-major) for a whitened
 * sketch Z (row-major M x r, r = 32 or 64).  Whiten Y again to finish the
 * step.  ws: gspca_sketch_workspace_bytes(M, N, r) bytes. */
gspca_status gspca_sketch_refine(const float *X, int64_t ldx, int64_t M, int64_t N,
                                 const float *Z, int32_t r, float *W, float *Y, void *ws,
                                 size_t ws_bytes, void *stream);

/* Z = sqrt(M) Y Q diag(g)^(-1/2) with the eigenpairs of Y^T Y (FP64, cyclic
 * Jacobi) ordered by decreasing g, each eigenvector's largest entry made
 * positive.  Y, Z row-major M x r (r = 32 or 64; M >= r); gamma (nullable) receives
 * g (r doubles); *flag (nullable) is set to 1 on the device if some g is not
 * positive and finite (the matching columns of Z are then 0), else 0.  Y^T Y
 * is summed in FP64 over row slices, added in slice order.  ws: at least
 * gspca_sketch_workspace_bytes(M, 1, r) bytes. */
gspca_status gspca_whiten_sketch(const float *Y, int64_t M, int32_t r, float *Z, double *gamma,
                                 int32_t *flag, void *ws, size_t ws_bytes, void *stream);

/* theta_bf16 <- bf16(theta). */
gspca_status gspca_mlp_sync(const gspca_mlp *net, void *stream);

/* O = network(Z): Z FP32 row-major rows x d0, O FP32 column-major rows x d3
 * (O[m + k*rows]).  Uses theta_bf16 for the weights, theta for the biases. */
gspca_status gspca_mlp_forward(const gspca_mlp *net, const float *Z, int64_t rows, float *O,
                               void *ws, size_t ws_bytes, void *stream);

/* Forward, loss and backward over ninst matrices of rows_per_inst rows each:
 * Z row-major (ninst*rows_per_inst) x d0, matrix b owning rows
 * [b*rows_per_inst, (b+1)*rows_per_inst); V the converged unit scores,
 * column-major per matrix: V[b*rows_per_inst*d3 + m + k*rows_per_inst].
 * Writes net->grad (gradient of the mean loss over the matrices) and
 * *loss (device double, nullable) = that mean loss. */
gspca_status gspca_mlp_loss_grad(const gspca_mlp *net, const float *Z, const float *V,
                                 int32_t ninst, int64_t rows_per_inst, double *loss, void *ws,
                                 size_t ws_bytes, void *stream);

/* One Adam step from net->grad (lr > 0, 0 <= beta < 1, eps > 0); refreshes
 * theta_bf16 and increments net->step. */
gspca_status gspca_mlp_adam(gspca_mlp *net, float lr, float beta1, float beta2, float eps,
                            void *stream);

/* Start vectors for one matrix: sketch of width r (32 or 64), whiten, `power`
 * refinement steps (0..4), forward on the first 32 whitened directions.  X
 * FP32 column-major M x N (M >= r), Omega FP32 row-major N x r, T0 FP32
 * column-major M x d3 (ready for gspca_options.T0 with
 * init = GSPCA_INIT_GIVEN).  A width above K oversamples the subspace. */
gspca_status gspca_ws_predict(const gspca_mlp *net, const float *X, int64_t ldx, int64_t M,
                              int64_t N, const float *Omega, int32_t r, int32_t power, float *T0,
                              void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* GSPCA_WS_H */
