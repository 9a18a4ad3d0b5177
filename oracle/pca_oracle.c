/*
 * pca_oracle.c -- plain, slow FP64 CPU oracle for iterative PCA.
 *
 * TEST INFRASTRUCTURE.  This file is the reference the GPU library is checked
 * against; it is not part of the library.  Only the test-suite, the package's
 * smoke check and the benchmark's CPU-baseline leg load it.  It shares no
 * code, header, table or helper with the GPU library.
 *
 * Source: M. Andrecut, "Parallel GPU Implementation of Iterative PCA
 * Algorithms", arXiv:0811.1081.
 *   - Sec. 2.1, eq. (2): PCA model X = T P^T.
 *   - Sec. 2.2, eqs. (3)-(4) and the NIPALS-PCA pseudo-code: power iteration
 *     P <- R^T T, normalise P, T <- R P, eigenvalue estimate = ||T||, then the
 *     rank-1 deflation R <- R - T P^T.
 *   - Sec. 2.3, eq. (5) and the GS-PCA pseudo-code: the same loop with one
 *     classical Gram-Schmidt pass of the loading U against U_(k) and of the
 *     score V against V_(k) in every iteration, V normalised by lambda_k,
 *     deflation R <- R - lambda_k V U^T, and finally T = V Lambda, P = U.
 *   - Appendices 1 and 3 (host programs): the convergence test is relative,
 *     |a - lambda| < er * lambda with a = previous estimate (0 at the start).
 *
 * Readings where the paper is silent or inconsistent (all mirrored by the GPU
 * library and listed in the design notes):
 *   - "eigenvalue" lambda_k of the paper is the norm of the score vector, i.e.
 *     the singular value sigma_k; the oracle returns sigma_k (lambda = sigma^2
 *     is formed by the caller).
 *   - max_iter counts (R^T, R) product pairs; iters[k] is the pair at which
 *     the test passed (or max_iter).
 *   - start vector: column k of the residual (the pseudo-code's R^(k)), the
 *     column of largest norm (ties to the lowest index), or a given vector;
 *     a zero start column falls back to the largest-norm column.  A given
 *     vector (the learned warm start) also falls back to the largest-norm
 *     column if its norm is below `tiny` or not finite, or, for GS-PCA, if
 *     one Gram-Schmidt pass against the earlier normalised scores V_(k)
 *     leaves less than a tenth of its norm.
 *   - degenerate component: if the loading or score norm is below `tiny`
 *     (DBL_MIN or FLT_MIN by the caller's choice), sigma_k = 0, t_k = 0 and
 *     p_k is the first canonical vector e_i (ascending i) whose Gram-Schmidt
 *     residual against P_(k) has squared norm >= (N-k)/(2N), normalised.
 *   - loading stop (not in the paper; optional): component k stops at the
 *     first iteration j >= 2 where |p_j - s p_(j-1)| < tol, s = +-1 aligning
 *     the signs of successive unit loadings.
 *   - implicit deflation (not in the paper): R is never formed; products use
 *     R p = X p - T (P^T p) and R^T t = X^T t - P (T^T t), identical in exact
 *     arithmetic.
 *   - re-orthogonalisation (not in the paper, which uses one classical pass;
 *     optional): the iteration's two Gram-Schmidt steps may instead run two
 *     classical passes (CGS2, each pass with coefficients from the vector as
 *     it enters that pass) or the modified process (MGS: for i = 0, 1, ...,
 *     the coefficient of column i is taken from the vector already reduced
 *     by columns 0..i-1).  The start-vector test and the degenerate rule
 *     keep one classical pass.
 *
 * Arithmetic: FP64, sequential loops in increasing index order; build with
 * -O2 -fno-fast-math -ffp-contract=off.  Matrices are column-major:
 * element (m, n) of an M x N matrix with leading dimension ld is A[m + n*ld].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_NOT_CONVERGED 1
#define OR_EINVAL (-1)
#define OR_ENONFINITE (-4)

#define OR_ALGO_GS 0
#define OR_ALGO_NIPALS 1

#define OR_STOP_SIGMA 0
#define OR_STOP_LOADING 1

#define OR_INIT_MAXNORM 0
#define OR_INIT_COLUMN_K 1
#define OR_INIT_GIVEN 2

#define OR_REORTH_CGS 0
#define OR_REORTH_CGS2 1
#define OR_REORTH_MGS 2

/* ------------------------------------------------------------------ */
/* Level-1 helpers (plain loops).                                      */

static double dot(const double *a, const double *b, int64_t n)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += a[i] * b[i];
    return s;
}

static double nrm2(const double *a, int64_t n) { return sqrt(dot(a, a, n)); }

/* ------------------------------------------------------------------ */
/* The residual operator R, either stored (explicit deflation) or      */
/* represented as X - T P^T over the finished components (implicit).   */

typedef struct {
    int implicit;
    int64_t M, N;
    const double *X; int64_t ldx; /* implicit: the data               */
    double *R;                    /* explicit: working copy, ld = M   */
    const double *T;              /* implicit: finished scores, M x k */
    const double *P;              /* implicit: finished loadings      */
    int64_t k;                    /* number of finished components    */
    double *tmp;                  /* K-length scratch                 */
} resid_op;

/* y = R^T x  (N-vector from M-vector) */
static void resid_t_mul(const resid_op *op, const double *x, double *y)
{
    const int64_t M = op->M, N = op->N;
    if (!op->implicit) {
        for (int64_t n = 0; n < N; ++n)
            y[n] = dot(op->R + n * M, x, M);
        return;
    }
    for (int64_t n = 0; n < N; ++n)
        y[n] = dot(op->X + n * op->ldx, x, M);
    /* minus P (T^T x) */
    for (int64_t i = 0; i < op->k; ++i)
        op->tmp[i] = dot(op->T + i * M, x, M);
    for (int64_t n = 0; n < N; ++n) {
        double s = 0.0;
        for (int64_t i = 0; i < op->k; ++i)
            s += op->P[n + i * N] * op->tmp[i];
        y[n] -= s;
    }
}

/* y = R x  (M-vector from N-vector) */
static void resid_mul(const resid_op *op, const double *x, double *y)
{
    const int64_t M = op->M, N = op->N;
    const double *A = op->implicit ? op->X : op->R;
    const int64_t ld = op->implicit ? op->ldx : M;
    for (int64_t m = 0; m < M; ++m)
        y[m] = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        const double xn = x[n];
        const double *col = A + n * ld;
        for (int64_t m = 0; m < M; ++m)
            y[m] += col[m] * xn;
    }
    if (!op->implicit)
        return;
    /* minus T (P^T x) */
    for (int64_t i = 0; i < op->k; ++i)
        op->tmp[i] = dot(op->P + i * N, x, N);
    for (int64_t m = 0; m < M; ++m) {
        double s = 0.0;
        for (int64_t i = 0; i < op->k; ++i)
            s += op->T[m + i * M] * op->tmp[i];
        y[m] -= s;
    }
}

/* out = R[:, n] */
static void resid_column(const resid_op *op, int64_t n, double *out)
{
    const int64_t M = op->M, N = op->N;
    if (!op->implicit) {
        memcpy(out, op->R + n * M, (size_t)M * sizeof(double));
        return;
    }
    for (int64_t m = 0; m < M; ++m) {
        double s = 0.0;
        for (int64_t i = 0; i < op->k; ++i)
            s += op->T[m + i * M] * op->P[n + i * N];
        out[m] = op->X[m + n * op->ldx] - s;
    }
}

/* Column of largest Euclidean norm (ties to the lowest index); its norm in *nrm. */
static int64_t resid_maxnorm_column(const resid_op *op, double *col, double *nrm)
{
    int64_t best = 0;
    double bestsq = -1.0;
    for (int64_t n = 0; n < op->N; ++n) {
        resid_column(op, n, col);
        const double sq = dot(col, col, op->M);
        if (sq > bestsq) {
            bestsq = sq;
            best = n;
        }
    }
    *nrm = sqrt(bestsq);
    return best;
}

/* ------------------------------------------------------------------ */
/* One classical Gram-Schmidt pass: x <- x - Q (Q^T x), Q n x k        */
/* orthonormal columns (Sec. 2.3: A <- U_(k)^T U, U <- U - U_(k) A).  */

static void cgs_pass(const double *Q, int64_t n, int64_t k, double *x, double *coef)
{
    for (int64_t i = 0; i < k; ++i)
        coef[i] = dot(Q + i * n, x, n);
    for (int64_t m = 0; m < n; ++m) {
        double s = 0.0;
        for (int64_t i = 0; i < k; ++i)
            s += Q[m + i * n] * coef[i];
        x[m] -= s;
    }
}

/* The iteration's Gram-Schmidt step in the chosen form: one classical pass
 * (the paper's), two classical passes, or the modified process. */
static void gs_step(const double *Q, int64_t n, int64_t k, double *x, double *coef, int reorth)
{
    if (reorth == OR_REORTH_MGS) {
        for (int64_t i = 0; i < k; ++i) {
            const double c = dot(Q + i * n, x, n);
            for (int64_t m = 0; m < n; ++m)
                x[m] -= Q[m + i * n] * c;
        }
        return;
    }
    cgs_pass(Q, n, k, x, coef);
    if (reorth == OR_REORTH_CGS2)
        cgs_pass(Q, n, k, x, coef);
}

/* One Gram-Schmidt step of the vector x (n) against the k columns of Q (n x
 * k, leading dimension n), in place, in the chosen form (for the tests). */
int oracle_gs_step(const double *Q, int64_t n, int64_t k, double *x, int reorth)
{
    if (!Q || !x || n < 1 || k < 0 || reorth < OR_REORTH_CGS || reorth > OR_REORTH_MGS)
        return OR_EINVAL;
    double *coef = malloc((size_t)(k + 1) * sizeof(double));
    if (!coef)
        return OR_EINVAL;
    gs_step(Q, n, k, x, coef, reorth);
    free(coef);
    return OR_OK;
}

/* Loading for a degenerate component: first e_i whose residual against P_(k)
 * has squared norm >= (N-k)/(2N), after one Gram-Schmidt pass, normalised. */
static void degenerate_loading(const double *P, int64_t N, int64_t k, double *p, double *coef)
{
    const double thresh = (double)(N - k) / (2.0 * (double)N);
    for (int64_t i = 0; i < N; ++i) {
        for (int64_t n = 0; n < N; ++n)
            p[n] = 0.0;
        p[i] = 1.0;
        cgs_pass(P, N, k, p, coef);
        const double sq = dot(p, p, N);
        if (sq >= thresh) {
            const double inv = 1.0 / sqrt(sq);
            for (int64_t n = 0; n < N; ++n)
                p[n] *= inv;
            return;
        }
    }
    /* Unreachable for k < N: the squared residuals sum to N - k. */
    for (int64_t n = 0; n < N; ++n)
        p[n] = 0.0;
}

/* ------------------------------------------------------------------ */
/* The fit.                                                             */

int oracle_fit(int algo, int implicit,
               const double *X, int64_t M, int64_t N, int64_t ldx, int64_t K,
               double tol, int32_t max_iter, int init, const double *T0,
               const int32_t *replay_iters, const int32_t *replay_start,
               double tiny, int stop, int reorth,
               double *T, double *P, double *sigma, int32_t *iters, int32_t *start_col,
               double *R_out)
{
    if (!X || !T || !P || !sigma || !iters || !start_col)
        return OR_EINVAL;
    if (M < 1 || N < 1 || K < 1 || K > M || K > N || ldx < M || max_iter < 1 || !(tol >= 0.0))
        return OR_EINVAL;
    if (algo != OR_ALGO_GS && algo != OR_ALGO_NIPALS)
        return OR_EINVAL;
    if (stop != OR_STOP_SIGMA && stop != OR_STOP_LOADING)
        return OR_EINVAL;
    if (reorth < OR_REORTH_CGS || reorth > OR_REORTH_MGS)
        return OR_EINVAL;
    if (init == OR_INIT_GIVEN && !T0)
        return OR_EINVAL;
    for (int64_t n = 0; n < N; ++n)
        for (int64_t m = 0; m < M; ++m)
            if (!isfinite(X[m + n * ldx]))
                return OR_ENONFINITE;
    if (!(tiny > 0.0))
        tiny = 2.2250738585072014e-308; /* DBL_MIN */

    double *t = malloc((size_t)M * sizeof(double));
    double *p = malloc((size_t)N * sizeof(double));
    double *pprev = malloc((size_t)N * sizeof(double));
    double *coef = malloc((size_t)(K + 1) * sizeof(double));
    double *tmp = malloc((size_t)(K + 1) * sizeof(double));
    double *Tfin = implicit ? malloc((size_t)M * K * sizeof(double)) : NULL;
    double *R = implicit ? NULL : malloc((size_t)M * N * sizeof(double));
    if (!t || !p || !pprev || !coef || !tmp || (implicit && !Tfin) || (!implicit && !R)) {
        free(t); free(p); free(pprev); free(coef); free(tmp); free(Tfin); free(R);
        return OR_EINVAL;
    }
    /* Sec. 2.2/2.3: R <- X. */
    if (!implicit)
        for (int64_t n = 0; n < N; ++n)
            memcpy(R + n * M, X + n * ldx, (size_t)M * sizeof(double));

    resid_op op = { implicit, M, N, X, ldx, R, Tfin, P, 0, tmp };
    int status = OR_OK;
    const int gs = (algo == OR_ALGO_GS);

    /* V (normalised scores, GS) or T (NIPALS) lives in T until the end. */
    for (int64_t k = 0; k < K; ++k) {
        op.k = k;
        double *tk = T + k * M;
        double *pk = P + k * N;
        int degenerate = 0;

        /* Start vector (Sec. 2.2 / 2.3 pseudo-code: T^(k) <- R^(k)). */
        int64_t sc = -1;
        double snrm = 0.0;
        if (replay_start && replay_start[k] >= 0 && replay_start[k] < N) {
            sc = replay_start[k];
            resid_column(&op, sc, t);
            snrm = nrm2(t, M);
        } else if (init == OR_INIT_GIVEN) {
            memcpy(t, T0 + k * M, (size_t)M * sizeof(double));
            snrm = nrm2(t, M);
            sc = -1;
            int fall = !(snrm >= tiny) || !isfinite(snrm);
            if (!fall && gs && k > 0) {
                /* residual of one CGS pass against v_0 .. v_(k-1) */
                double *r = malloc((size_t)M * sizeof(double));
                if (!r) { status = OR_EINVAL; break; }
                memcpy(r, t, (size_t)M * sizeof(double));
                for (int64_t i = 0; i < k; ++i) {
                    const double c = dot(T + i * M, t, M);
                    for (int64_t m = 0; m < M; ++m)
                        r[m] -= c * T[m + i * M];
                }
                fall = nrm2(r, M) < 0.1 * snrm;
                free(r);
            }
            if (fall)
                sc = resid_maxnorm_column(&op, t, &snrm), resid_column(&op, sc, t);
        } else if (init == OR_INIT_COLUMN_K) {
            sc = k;
            resid_column(&op, sc, t);
            snrm = nrm2(t, M);
            if (!(snrm >= tiny))
                sc = resid_maxnorm_column(&op, t, &snrm), resid_column(&op, sc, t);
        } else {
            sc = resid_maxnorm_column(&op, t, &snrm);
            resid_column(&op, sc, t);
        }
        start_col[k] = (int32_t)sc;
        if (!(snrm >= tiny))
            degenerate = 1;

        double mu = 0.0, s = 0.0;
        int32_t j = 0;
        int converged = 0;
        const int32_t limit = replay_iters ? replay_iters[k] : max_iter;
        if (limit < 1)
            degenerate = 1;
        while (!degenerate && j < limit) {
            ++j;
            /* P^(k) <- R^T T^(k) */
            resid_t_mul(&op, t, p);
            /* GS-PCA: A <- U_(k)^T U^(k); U^(k) <- U^(k) - U_(k) A */
            if (gs && k > 0)
                gs_step(P, N, k, p, coef, reorth);
            /* normalise the loading */
            const double pn = nrm2(p, N);
            if (!(pn >= tiny)) { degenerate = 1; break; }
            for (int64_t n = 0; n < N; ++n)
                p[n] /= pn;
            /* loading stop (not in the paper): the change |p_j - s p_(j-1)|
             * of the unit loading, s = +-1 aligning the signs */
            double dp = INFINITY;
            if (j >= 2) {
                const double sgn = dot(p, pprev, N) >= 0.0 ? 1.0 : -1.0;
                double ss = 0.0;
                for (int64_t n = 0; n < N; ++n)
                    ss += (p[n] - sgn * pprev[n]) * (p[n] - sgn * pprev[n]);
                dp = sqrt(ss);
            }
            memcpy(pprev, p, (size_t)N * sizeof(double));
            /* T^(k) <- R P^(k) */
            resid_mul(&op, p, t);
            /* GS-PCA: B <- V_(k)^T V^(k); V^(k) <- V^(k) - V_(k) B */
            if (gs && k > 0)
                gs_step(T, M, k, t, coef, reorth);
            /* eigenvalue estimate = score norm */
            s = nrm2(t, M);
            if (!(s >= tiny)) { degenerate = 1; break; }
            /* GS-PCA normalises the score by lambda_k */
            if (gs)
                for (int64_t m = 0; m < M; ++m)
                    t[m] /= s;
            if (replay_iters)
                continue;
            if (stop == OR_STOP_LOADING) {
                if (dp < tol) { converged = 1; break; }
            } else if (fabs(mu - s) < tol * s) {
                /* relative test of the host programs (Appendices 1, 3) */
                converged = 1;
                break;
            }
            mu = s;
        }
        if (degenerate) {
            for (int64_t m = 0; m < M; ++m)
                t[m] = 0.0;
            degenerate_loading(P, N, k, p, coef);
            s = 0.0;
            converged = 1;
        }
        if (!converged && !replay_iters)
            status = OR_NOT_CONVERGED;
        iters[k] = j;
        sigma[k] = s;
        memcpy(tk, t, (size_t)M * sizeof(double));
        memcpy(pk, p, (size_t)N * sizeof(double));

        /* Deflation: eq. (3) for NIPALS (R <- R - T P^T); Sec. 2.3 for GS
         * (R <- R - lambda_k V U^T).  Implicit: record the finished score. */
        if (!implicit) {
            for (int64_t n = 0; n < N; ++n) {
                const double pn = pk[n];
                double *col = R + n * M;
                for (int64_t m = 0; m < M; ++m)
                    col[m] -= (gs ? s * tk[m] : tk[m]) * pn;
            }
        } else {
            for (int64_t m = 0; m < M; ++m)
                Tfin[m + k * M] = gs ? s * tk[m] : tk[m];
        }
    }

    /* GS-PCA: T <- V Lambda (NIPALS scores are already unnormalised). */
    if (gs)
        for (int64_t k = 0; k < K; ++k)
            for (int64_t m = 0; m < M; ++m)
                T[m + k * M] *= sigma[k];

    if (R_out) {
        if (!implicit) {
            memcpy(R_out, R, (size_t)M * N * sizeof(double));
        } else {
            op.k = K;
            for (int64_t n = 0; n < N; ++n)
                resid_column(&op, n, R_out + n * M);
        }
    }
    free(t); free(p); free(pprev); free(coef); free(tmp); free(Tfin); free(R);
    return status;
}

/* ------------------------------------------------------------------ */
/* One score step in isolation (GS-PCA, pseudo-code of Sec. 2.3):       */
/*   t = R_k p,  R_k = X - V_(k) diag(sigma_(k)) P_(k)^T,               */
/*   t <- t - V_(k) (V_(k)^T t),  s = ||t||,  v = t / s.                */
/* Used to check a GPU fit at sizes the full oracle cannot finish:     */
/* the final score of component k is this step applied to its final    */
/* loading.  V holds normalised scores (M x k), P loadings (N x k).     */

int oracle_score_step(const double *X, int64_t M, int64_t N, int64_t ldx, int64_t k,
                      const double *V, const double *sigma, const double *P,
                      const double *p, double *v, double *s_out)
{
    if (!X || !p || !v || !s_out || M < 1 || N < 1 || k < 0 || ldx < M)
        return OR_EINVAL;
    if (k > 0 && (!V || !sigma || !P))
        return OR_EINVAL;
    double *c = malloc((size_t)(k + 1) * sizeof(double));
    if (!c)
        return OR_EINVAL;
    for (int64_t m = 0; m < M; ++m)
        v[m] = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        const double pn = p[n];
        for (int64_t m = 0; m < M; ++m)
            v[m] += X[m + n * ldx] * pn;
    }
    /* minus V diag(sigma) P^T p */
    for (int64_t i = 0; i < k; ++i)
        c[i] = sigma[i] * dot(P + i * N, p, N);
    for (int64_t m = 0; m < M; ++m) {
        double s = 0.0;
        for (int64_t i = 0; i < k; ++i)
            s += V[m + i * M] * c[i];
        v[m] -= s;
    }
    cgs_pass(V, M, k, v, c);
    const double s = nrm2(v, M);
    *s_out = s;
    if (s > 0.0)
        for (int64_t m = 0; m < M; ++m)
            v[m] /= s;
    free(c);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Brute-force reference: cyclic-by-row Jacobi eigendecomposition of a  */
/* symmetric n x n matrix (Golub & Van Loan, the textbook the paper     */
/* cites for Gram-Schmidt).  A is overwritten; on return w holds the    */
/* eigenvalues in descending order and Q (column-major) the matching   */
/* orthonormal eigenvectors.  Returns the number of sweeps.            */

int oracle_jacobi_eig(double *A, int64_t n, double *w, double *Q)
{
    if (!A || !w || !Q || n < 1)
        return OR_EINVAL;
    for (int64_t j = 0; j < n; ++j)
        for (int64_t i = 0; i < n; ++i)
            Q[i + j * n] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (int64_t i = 0; i < n * n; ++i)
        fro += A[i] * A[i];
    fro = sqrt(fro);
    int sweeps = 0;
    for (; sweeps < 100; ++sweeps) {
        double off = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < n; ++i)
                if (i != j)
                    off += A[i + j * n] * A[i + j * n];
        if (sqrt(off) <= 1e-15 * fro)
            break;
        for (int64_t p = 0; p < n - 1; ++p) {
            for (int64_t q = p + 1; q < n; ++q) {
                const double apq = A[p + q * n];
                if (apq == 0.0)
                    continue;
                /* 2x2 symmetric Schur decomposition: choose (c, s) so that the
                 * rotated (p, q) entry vanishes, smaller rotation angle. */
                const double app = A[p + p * n], aqq = A[q + q * n];
                const double tau = (aqq - app) / (2.0 * apq);
                const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                const double c = 1.0 / sqrt(1.0 + tt * tt);
                const double s = tt * c;
                /* A <- J^T A J with J = I except J_pp = J_qq = c, J_pq = s, J_qp = -s */
                for (int64_t k = 0; k < n; ++k) { /* columns p, q: A J */
                    const double akp = A[k + p * n], akq = A[k + q * n];
                    A[k + p * n] = c * akp - s * akq;
                    A[k + q * n] = s * akp + c * akq;
                }
                for (int64_t k = 0; k < n; ++k) { /* rows p, q: J^T (A J) */
                    const double apk = A[p + k * n], aqk = A[q + k * n];
                    A[p + k * n] = c * apk - s * aqk;
                    A[q + k * n] = s * apk + c * aqk;
                }
                for (int64_t k = 0; k < n; ++k) { /* Q <- Q J */
                    const double qkp = Q[k + p * n], qkq = Q[k + q * n];
                    Q[k + p * n] = c * qkp - s * qkq;
                    Q[k + q * n] = s * qkp + c * qkq;
                }
            }
        }
    }
    /* sort descending (selection sort on the diagonal) */
    for (int64_t i = 0; i < n; ++i)
        w[i] = A[i + i * n];
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = i;
        for (int64_t j = i + 1; j < n; ++j)
            if (w[j] > w[b])
                b = j;
        if (b != i) {
            const double tw = w[i]; w[i] = w[b]; w[b] = tw;
            for (int64_t r = 0; r < n; ++r) {
                const double tq = Q[r + i * n];
                Q[r + i * n] = Q[r + b * n];
                Q[r + b * n] = tq;
            }
        }
    }
    return sweeps;
}
