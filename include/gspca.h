/*
 * gspca.h -- C ABI of the MI355X (gfx950) iterative-PCA library.
 *
 * Method: M. Andrecut, "Parallel GPU Implementation of Iterative PCA
 * Algorithms", arXiv:0811.1081.
 *   NIPALS-PCA: Sec. 2.2 (eqs. 3-4 and its pseudo-code).
 *   GS-PCA:     Sec. 2.3 (eq. 5 and its pseudo-code): per component k, repeat
 *       p <- R^T t; p <- p - P_(k) (P_(k)^T p); p <- p / |p|;
 *       t <- R p;   t <- t - V_(k) (V_(k)^T t); sigma <- |t|; v <- t / sigma
 *     until |sigma - mu| < tol * sigma (mu = previous sigma, 0 at the start;
 *     the relative test of the host programs in Appendices 1 and 3), then
 *     deflate R <- R - sigma v p^T; finally T = V diag(sigma), P = U.
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major: element (m, n) of X is X[m + n*ldx].
 *     T is M x K with leading dimension M, P is N x K with leading dimension N.
 *   - Every array argument is a DEVICE pointer (memory of the GPU that is
 *     current on the calling thread), owned by the caller; the library never
 *     frees caller memory.  `stream` is a hipStream_t passed as void*
 *     (NULL = the default stream).
 *   - lambda[k] = sigma_k^2 where sigma_k = |t_k| (the paper's "eigenvalue"
 *     lambda_k is the norm of the score, i.e. a singular value of X).
 *   - Start vector: column of the residual with the largest norm (ties to the
 *     lowest index) unless options say otherwise.  A zero start column falls
 *     back to the largest-norm column.
 *   - Degenerate component (loading or score norm below DBL_MIN for FP64 data,
 *     FLT_MIN otherwise): sigma_k = 0, T[:,k] = 0 and P[:,k] = the first unit
 *     vector e_i (ascending i) whose Gram-Schmidt residual against P[:, :k]
 *     has squared norm >= (N-k)/(2N), after one projection, normalised.
 *   - No sign normalisation is applied (the paper applies none).
 *   - Errors: negative status codes are returned after host-side validation
 *     and enqueue nothing; outputs are then unspecified.  NOT_CONVERGED means
 *     some component stopped at max_iter; its outputs are the last iterate.
 *   - Calls on one stream are serialised; calls on different streams are
 *     independent as long as they use distinct workspaces.
 */
#ifndef GSPCA_H
#define GSPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSPCA_OK = 0,
    GSPCA_NOT_CONVERGED = 1,
    GSPCA_EINVAL = -1,     /* bad size, pointer, tolerance or option           */
    GSPCA_EWORKSPACE = -2, /* workspace smaller than gspca_workspace_bytes()   */
    GSPCA_EDEVICE = -3,    /* a HIP runtime call failed                        */
    GSPCA_ENONFINITE = -4, /* X holds NaN or Inf                               */
    GSPCA_ENOMEM = -5      /* the convenience entry points could not allocate  */
} gspca_status;

typedef enum {
    GSPCA_F64 = 0, /* X, T, P, T0 double                                       */
    GSPCA_F32 = 1  /* X, T, P, T0 float; Gram-Schmidt and norms in FP64        */
} gspca_dtype;

typedef enum { GSPCA_GS = 0, GSPCA_NIPALS = 1 } gspca_algo;

typedef enum {
    GSPCA_INIT_MAXNORM = 0,  /* largest-norm residual column (default)        */
    GSPCA_INIT_COLUMN_K = 1, /* column k of the residual (the pseudo-code's R^(k)) */
    GSPCA_INIT_GIVEN = 2     /* column k of options.T0                        */
} gspca_init;

/* Optional per-kernel timing (host memory, filled when options.profile is
 * non-NULL).  Each launch of the two streaming kernels that did work is
 * bracketed by HIP events on the fit's stream; launches enqueued past a
 * component's stop are not counted.  Adds a few microseconds per launch. */
typedef struct {
    double pass_ms;         /* single-pass path: summed duration of the fused  */
    int64_t pass_launches;  /*   t <- R p, q <- R^T t launches                 */
    double gemv_t_ms;       /* two-pass path: p <- R^T t launches              */
    double gemv_n_ms;       /* two-pass path: t <- R p launches                */
    int64_t gemv_t_launches;
    int64_t gemv_n_launches;
    int64_t iterations;     /* iterations run, summed over components          */
    int64_t bytes_per_pass; /* algorithmic bytes of one read of the data, M*N*size */
    int32_t single_pass;    /* 1 when the single-pass path ran                 */
    int32_t reserved;
} gspca_profile;

/* The data.  X is read, never written. */
typedef struct {
    int32_t dtype;   /* gspca_dtype                                         */
    const void *X;   /* M x N, leading dimension ldx >= M                   */
    int64_t ldx;
    int64_t M, N, K; /* 1 <= K <= min(M, N)                                 */
} gspca_problem;

typedef struct {
    int32_t algo;       /* gspca_algo                                          */
    int32_t init;       /* gspca_init                                          */
    /* 0: explicit deflation R <- R - t p^T after each component (Secs. 2.2-2.3).
     * 1: implicit: R = X - T P^T is never formed; the products use X on
     *    Gram-Schmidt-projected vectors, for which the T P^T terms vanish in
     *    exact arithmetic (GS-PCA only; N <= 8192 for FP32, N <= 4096 for FP64). */
    int32_t implicit_deflation;
    const void *T0;     /* M x K start scores (GIVEN only), dtype of X         */
    double tol;         /* >= 0; 0 runs exactly max_iter iterations            */
    int32_t max_iter;   /* >= 1: number of (R^T t, R p) product pairs          */
    /* Replay (testing): when non-NULL, component k runs exactly
     * replay_iters[k] iterations without the convergence test, starting from
     * residual column replay_start_col[k] (entries < 0: use `init`).  Device
     * arrays of K int32 each; they are read before the fit starts. */
    const int32_t *replay_iters;
    const int32_t *replay_start_col;
    gspca_profile *profile; /* host pointer, nullable (see gspca_profile)      */
} gspca_options;

/* Outputs (device pointers).  T, P and lambda are required. */
typedef struct {
    void *T;            /* M x K scores T = V diag(sigma) (NIPALS: the score t) */
    void *P;            /* N x K unit loadings                                  */
    double *lambda;     /* K: sigma_k^2                                         */
    double *sigma;      /* K: sigma_k (nullable)                                */
    int32_t *iters;     /* K: iteration at which component k stopped (nullable) */
    int32_t *start_col; /* K: start column, -1 for a given start (nullable)     */
} gspca_result;

/* Default options: GS-PCA, max-norm start, tol 1e-7 and max_iter 10000 (the
 * constants of the paper's programs), no replay. */
void gspca_default_options(gspca_options *opt);

/* Bytes of device workspace gspca_fit_ex needs for this problem and options
 * (0 if the arguments are invalid).  The workspace holds the residual R (an
 * M x N copy of X with 64-element-aligned columns), the iteration vectors,
 * reduction partials and the loop state. */
size_t gspca_workspace_bytes(const gspca_problem *prob, const gspca_options *opt);

/* Fit K components of X (Secs. 2.2-2.3).  `ws` is a device buffer of at least
 * gspca_workspace_bytes() bytes, 256-byte aligned, owned by the caller and
 * not touched after the call returns.  All work is enqueued on `stream`; the
 * host reads a small status word once per batch of iterations to test
 * convergence, so the call returns only after the fit has completed on the
 * GPU (the stream is synchronised).  Returns OK, NOT_CONVERGED or an error. */
gspca_status gspca_fit_ex(const gspca_problem *prob, const gspca_options *opt,
                          const gspca_result *res, void *ws, size_t ws_bytes, void *stream);

/* Convenience forms: GS-PCA with the max-norm start and the relative
 * sigma test, FP64 or FP32 data (ldx = M).  They allocate and free their own
 * workspace with hipMalloc/hipFree (ENOMEM if that fails) and synchronise
 * `stream`. */
gspca_status gspca_fit(const double *X, int64_t M, int64_t N, int64_t K, double tol,
                       int32_t max_iter, double *T, double *P, double *lambda, void *stream);
gspca_status gspca_fit_f32(const float *X, int64_t M, int64_t N, int64_t K, double tol,
                           int32_t max_iter, float *T, float *P, double *lambda, void *stream);

/* Human-readable name of a status code (static string). */
const char *gspca_status_string(int status);

/* Library ABI version (major * 10000 + minor * 100 + patch). */
int gspca_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GSPCA_H */
