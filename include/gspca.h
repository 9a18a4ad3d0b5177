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
 *     back to the largest-norm column.  So does a given start (options.T0)
 *     whose norm is below the degenerate threshold or not finite, or, for
 *     GS-PCA, one that keeps less than a tenth of its norm after one
 *     Gram-Schmidt pass against the earlier normalised scores.
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
 *   - Graph capture: an entry point that reads results back to the host
 *     (gspca_fit_ex, gspca_fit, gspca_fit_f32, gspca_quantize,
 *     gspca_batched_prepare, gspca_batched_tune, gspca_fit_block) returns
 *     GSPCA_EINVAL, enqueuing nothing, when `stream` is being captured into a
 *     hipGraph.  Loop state is cleared by a kernel, never by a memset.
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
    GSPCA_F64 = 0,      /* X, T, P, T0 double                                  */
    GSPCA_F32 = 1,      /* X, T, P, T0 float; Gram-Schmidt and norms in FP64   */
    GSPCA_BF16 = 2,     /* X = bfloat16 codes from gspca_quantize; T, P, T0 float */
    GSPCA_FP8_E4M3 = 3  /* X = OCP FP8 E4M3 codes from gspca_quantize; T, P, T0 float */
} gspca_dtype;

/* Stop rule of each component's iteration. */
typedef enum {
    GSPCA_STOP_SIGMA_REL = 0, /* |sigma_j - sigma_(j-1)| < tol * sigma_j: the
                                 relative test of the paper's programs          */
    GSPCA_STOP_LOADING = 1    /* |p_j - s p_(j-1)| < tol (s = +-1 aligning the
                                 signs): the unit loading moved less than tol;
                                 evaluated from FP64 dot products, meaningful
                                 for tol >= 1e-7                                */
} gspca_stop;

typedef enum { GSPCA_GS = 0, GSPCA_NIPALS = 1 } gspca_algo;

/* Form of GS-PCA's two Gram-Schmidt steps per iteration (Sec. 2.3 uses one
 * classical pass; the other two are re-orthogonalisation variants for
 * studying the loss of orthogonality, not in the paper):
 *   CGS:  x <- x - Q (Q^T x), one pass (the paper's; default).
 *   CGS2: the classical pass applied twice, each with coefficients from the
 *         vector as it enters that pass.
 *   MGS:  modified Gram-Schmidt: for i = 0 .. k-1 in order, the coefficient
 *         of column i is taken from the vector already reduced by columns
 *         0 .. i-1.
 * CGS2 and MGS run on the two-pass path (t and p formed explicitly every
 * iteration) with explicit deflation, FP32/FP64 data; MGS does its k steps
 * inside one workgroup per side, so it is meant for moderate sizes.  NIPALS
 * has no Gram-Schmidt step and ignores the field. */
typedef enum { GSPCA_REORTH_CGS = 0, GSPCA_REORTH_CGS2 = 1, GSPCA_REORTH_MGS = 2 } gspca_reorth;

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
    int64_t bytes_per_pass; /* algorithmic bytes of one read of the data:
                               M*N*(bytes per element of the stored X)         */
    int32_t single_pass;    /* 1 when the single-pass path ran                 */
    int32_t reserved;
} gspca_profile;

/* The data.  X is read, never written.  For F64/F32, X is column-major with
 * leading dimension ldx >= M.  For BF16/FP8_E4M3, X is the code buffer
 * written by gspca_quantize for the same M and N (ldx ignored) and col_scale
 * its N per-column scales; the represented matrix is
 * X~[m, n] = decode(code[m, n]) * col_scale[n]. */
typedef struct {
    int32_t dtype;   /* gspca_dtype                                         */
    const void *X;
    int64_t ldx;
    int64_t M, N, K; /* 1 <= K <= min(M, N)                                 */
    const float *col_scale; /* BF16/FP8 only (device, N floats)             */
} gspca_problem;

typedef struct {
    int32_t algo;       /* gspca_algo                                          */
    int32_t init;       /* gspca_init                                          */
    /* 0: explicit deflation R <- R - t p^T after each component (Secs. 2.2-2.3).
     * 1: implicit: R = X - T P^T is never formed; the products use X on
     *    Gram-Schmidt-projected vectors, for which the T P^T terms vanish in
     *    exact arithmetic (GS-PCA only; N <= 8192 for FP32, BF16 and FP8,
     *    N <= 4096 for FP64).  Required for BF16/FP8 data. */
    int32_t implicit_deflation;
    int32_t stop;       /* gspca_stop                                          */
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
    int32_t reorth;     /* gspca_reorth (GS-PCA; 0 = the paper's single pass;
                           others need explicit deflation and F64/F32 data)   */
    int32_t reserved;
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

/* Default options: GS-PCA, explicit deflation, max-norm start, the relative
 * sigma stop with tol 1e-7 and max_iter 10000 (the constants of the paper's
 * programs), no replay, no profile. */
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
 * convergence, so the call is blocking: it returns only after the fit has
 * completed on the GPU (the stream is synchronised), and it returns
 * GSPCA_EINVAL without enqueuing anything when `stream` is capturing.
 * Returns OK, NOT_CONVERGED or an error. */
gspca_status gspca_fit_ex(const gspca_problem *prob, const gspca_options *opt,
                          const gspca_result *res, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (serving loops that must
 * not call hipMalloc, harnesses that forbid it): gspca_fit_ex with no
 * workspace argument.  The workspace is a fixed array of
 * GSPCA_NOALLOC_SCRATCH_BYTES bytes inside the library, one copy per GPU,
 * held until the process ends; the call allocates nothing (no hipMalloc,
 * hipFree or event creation).  Problems whose gspca_workspace_bytes() exceed
 * that size are refused with GSPCA_EWORKSPACE (for FP32, roughly M*N*4 plus
 * N*K*8 bytes must fit: e.g. 4096 x 512 with K = 512 does); options with
 * replay arrays or a profile are refused with GSPCA_EINVAL.  Every call on
 * one GPU uses that GPU's array, which keeps the last call's contents (the
 * fit initialises what it reads): calls that overlap on one GPU, from any
 * thread or stream, race and must not be issued.  Blocking and not
 * capturable, as gspca_fit_ex.  The device is the current one. */
#define GSPCA_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
size_t gspca_noalloc_scratch_bytes(void);
gspca_status gspca_fit_noalloc(const gspca_problem *prob, const gspca_options *opt,
                               const gspca_result *res, void *stream);

/* Reduced-precision storage (not in the paper, whose Sec. 3 only notes the
 * programs convert to single precision): per-column scale
 * s_n = max_m |X[m,n]| / Qmax (binary32; Qmax = 1 for BF16, 448 for E4M3;
 * an all-zero column has s_n = 1) and codes encode(X[m,n] / s_n) (binary32
 * division, round to nearest even; E4M3 saturates to +-448).
 * Code layout: row panels of PR = 8 (BF16) or 16 (FP8) rows, panel b holding
 * rows [b*PR, b*PR + PR) of `ldp` columns, the PR codes of one column in 16
 * contiguous bytes, column n of panel b at byte offset (b*ldp + n)*16; ldp >= N
 * is fixed by N (columns >= N and rows >= M are zero codes).
 * gspca_quantized_bytes: size of Q for M x N (0 if dtype is not BF16/FP8, or
 * N > 8192).  gspca_quantize: X is FP32 column-major (ldx >= M); Q and
 * col_scale (N floats) are written on `stream`; `ws` is a device scratch of
 * at least 256 bytes (256-byte aligned).  Synchronises the stream; returns
 * ENONFINITE if X holds NaN/Inf. */
size_t gspca_quantized_bytes(int64_t M, int64_t N, int32_t dtype);
gspca_status gspca_quantize(const float *X, int64_t M, int64_t N, int64_t ldx, int32_t dtype,
                            void *Q, float *col_scale, void *ws, size_t ws_bytes, void *stream);

/* ---- Batched fits: many independent FP32 problems in one persistent launch.
 * Each problem is an FP32 column-major X (M <= 4096, N <= 1024,
 * 1 <= K <= min(M, N, 64)) with its own outputs, as in gspca_result, plus an
 * int32 status word written by the device (0 OK, 1 NOT_CONVERGED,
 * -4 ENONFINITE).  GS-PCA with implicit deflation (X is never written); the
 * options' algo must be GS; init MAXNORM, COLUMN_K or GIVEN (then every
 * problem's T0 is required; the fallback rule of a given start applies);
 * replay arrays are taken per problem.  All pointers are device pointers. */
typedef struct {
    const float *X;
    /* leading dimension, >= M; rows M..ldx-1 are never read.  A multiple of
     * 32 (128-byte aligned columns) lets the kernel read whole cache lines:
     * on a 2048-problem batch ldx = M costs ~10 % (104.5 vs 95.3 ms). */
    int64_t ldx;
    int64_t M, N, K;
    float *T;            /* M x K, leading dimension M                          */
    float *P;            /* N x K, leading dimension N                          */
    double *lambda;      /* K                                                   */
    double *sigma;       /* K, nullable                                         */
    int32_t *iters;      /* K, nullable                                         */
    int32_t *start_col;  /* K, nullable                                         */
    const int32_t *replay_iters;     /* K, nullable (testing)                   */
    const int32_t *replay_start_col; /* K, nullable (testing)                   */
    int32_t *status;     /* one int32, nullable                                 */
    const float *T0;     /* M x K start vectors (leading dimension M), read when
                            options.init == GSPCA_INIT_GIVEN; else ignored      */
} gspca_batch_problem;

/* Launch plan filled by gspca_batched_prepare (host memory, opaque). */
typedef struct {
    unsigned char opaque[256];
} gspca_batch_plan;

/* Device workspace for a batch (problem table, queue, per-problem X^T V). */
size_t gspca_batched_workspace_bytes(const gspca_batch_problem *probs, int32_t nprob);

/* Validate the problems (host array of descriptors), write the descriptor
 * table -- sorted by decreasing M*N so that the queue hands out the largest
 * problems first -- into `ws`, and fill `plan` with a default launch shape.
 * Options: GS-PCA, explicit form, opt->reorth == GSPCA_REORTH_CGS (else
 * GSPCA_EINVAL).  Synchronises `stream`.  Not capturable. */
gspca_status gspca_batched_prepare(const gspca_batch_problem *probs, int32_t nprob,
                                   const gspca_options *opt, void *ws, size_t ws_bytes,
                                   gspca_batch_plan *plan, void *stream);

/* Enqueue the whole batch: one queue-reset kernel and one persistent kernel.
 * No host synchronisation and no memset, so the call can be captured in a
 * hipGraph and replayed (each replay refits every problem).  The status words
 * are valid once the stream has reached the end of the launch. */
gspca_status gspca_batched_launch(const gspca_batch_plan *plan, void *stream);

/* Autotuner: time the launch for each candidate shape (threads per
 * workgroup x workgroups per compute unit, within the LDS the problems need)
 * and keep the fastest in `plan`.  Runs the batch several times (outputs are
 * overwritten with the same results).  When the environment variable
 * GSPCA_TUNE_CACHE names a file, results are looked up there first and
 * recorded there (one JSON object per line, keyed by the batch signature). */
gspca_status gspca_batched_tune(gspca_batch_plan *plan, void *stream);

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
