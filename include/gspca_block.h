/*
 * gspca_block.h -- block form of the iteration: the K leading singular
 * triplets of X from one block of r vectors iterated together.
 *
 * Not in the paper, whose GS-PCA (Sec. 2.3) iterates one component at a time
 * and deflates; this is the block (subspace) iteration with Rayleigh-Ritz
 * that reads X twice per iteration for all r vectors at once (Halko,
 * Martinsson & Tropp 2011, Alg. 4.4, with the orthonormalisation done by
 * whitening).  With V_j the M x r orthonormal block (V_0 from Y = X Omega or
 * from given start vectors Y = Z0):
 *
 *   Y   = X (X^T V_j)                      two products over X
 *   Y^T Y = Q diag(g) Q^T                  FP64 Jacobi, g decreasing
 *   V_(j+1) = Y Q diag(g)^(-1/2)           orthonormal, in Ritz order
 *
 * g holds the Ritz values of (X X^T)^2 on the block, so s_i = g_i^(1/4)
 * estimates sigma_i.  Stop tests, for every i < K at once:
 *   GSPCA_STOP_SIGMA_REL: |s_i^(j) - s_i^(j-1)| < tol * s_i^(j) (the paper's
 *     relative test on the K leading estimates; s^(0) = 0).  The estimates
 *     settle quadratically faster than the vectors, so in FP32 this test
 *     suits tolerances down to ~1e-7, i.e. vectors to ~3e-4.
 *   GSPCA_STOP_LOADING: |v_i^(j) - s v_i^(j-1)| < tol, s = +-1 aligning the
 *     signs: the unit Ritz vectors moved less than tol (FP64 dot products).
 * At the end
 *   w_i = X^T v_i,  sigma_i = |w_i|,  P[:, i] = w_i / sigma_i,
 *   T[:, i] = sigma_i v_i,  lambda_i = sigma_i^2          (i < K)
 * -- the same output conventions as gspca_fit_ex (T = V Lambda, unit
 * loadings, lambda = sigma^2), columns in decreasing Ritz order, signs free.
 *
 * Precision: X FP32; products accumulate in FP32, the Gram matrix, the
 * eigen-decomposition and the output norms in FP64.  Block widths r = 32 or
 * 64 (K <= r <= M; a width above K oversamples, which speeds convergence by
 * the factor (sigma_(r+1) / sigma_K)^2 per iteration).
 *
 * All arrays are device pointers owned by the caller; `stream` is a
 * hipStream_t passed as void*.  No entry point allocates memory.
 */
#ifndef GSPCA_BLOCK_H
#define GSPCA_BLOCK_H
#include "gspca.h"
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t r;          /* block width: 32 or 64, K <= r <= M                  */
    int32_t max_iter;   /* >= 1 block iterations                               */
    int32_t stop;       /* gspca_stop (see above)                              */
    int32_t reserved;
    double tol;         /* >= 0; 0 runs exactly max_iter iterations            */
    const float *Omega; /* N x r row-major start sketch (used when Z0 is NULL) */
    const float *Z0;    /* M x r row-major start vectors (nullable); whitened
                           before the first iteration                          */
} gspca_block_options;

/* Device workspace of gspca_fit_block (0 for invalid sizes). */
size_t gspca_block_workspace_bytes(int64_t M, int64_t N, int32_t r);

/* Fit the K leading components of X (FP32 column-major M x N, ldx >= M).
 * Outputs: T (M x K, leading dimension M), P (N x K, leading dimension N),
 * lambda (K doubles), sigma (K doubles, nullable), *iters (host, nullable):
 * the iterations run.  The host reads the K estimates after every iteration,
 * so the call synchronises `stream` and returns when the fit is done.
 * Returns OK, NOT_CONVERGED (max_iter reached with tol > 0), EINVAL (bad
 * arguments, or a Ritz value among the first K that is not positive and
 * finite: X of rank below K to the last bit, e.g. zero, or non-finite),
 * EWORKSPACE, or EDEVICE. */
gspca_status gspca_fit_block(const float *X, int64_t ldx, int64_t M, int64_t N, int64_t K,
                             const gspca_block_options *opt, float *T, float *P, double *lambda,
                             double *sigma, int32_t *iters, void *ws, size_t ws_bytes,
                             void *stream);

#ifdef __cplusplus
}
#endif
#endif /* GSPCA_BLOCK_H */
