/*
 * oracle_sanitize.c -- driver that runs every entry point of the C oracle
 * (oracle/pca_oracle.c, codec_oracle.c, mlp_oracle.c) on small inputs, for a
 * build with -fsanitize=address,undefined.  It checks no numbers beyond a few
 * sanity conditions (the numerical pins live in the Python tests); its job is
 * to walk every code path -- both algorithms, explicit and implicit
 * deflation, every start mode, both stop rules, the three Gram-Schmidt
 * forms, replay, the degenerate and non-finite cases, the codecs, the
 * network's forward and backward passes and Adam -- under the sanitizers.
 * Test infrastructure: compiled and run by tests/test_oracle_sanitize.py.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_fit(int algo, int implicit, const double *X, int64_t M, int64_t N, int64_t ldx,
               int64_t K, double tol, int32_t max_iter, int init, const double *T0,
               const int32_t *replay_iters, const int32_t *replay_start, double tiny, int stop,
               int reorth, double *T, double *P, double *sigma, int32_t *iters,
               int32_t *start_col, double *R_out);
int oracle_gs_step(const double *Q, int64_t n, int64_t k, double *x, int reorth);
int oracle_score_step(const double *X, int64_t M, int64_t N, int64_t ldx, int64_t k,
                      const double *V, const double *sigma, const double *P, const double *p,
                      double *v, double *s_out);
int oracle_jacobi_eig(double *A, int64_t n, double *w, double *Q);
float oracle_bf16_decode(uint16_t c);
uint16_t oracle_bf16_encode(float x);
double oracle_e4m3_decode(uint8_t c);
uint8_t oracle_e4m3_encode(float x);
int oracle_quantize(const float *X, int64_t M, int64_t N, int64_t ldx, int fmt, void *codes,
                    float *scale);
int oracle_dequantize(const void *codes, const float *scale, int64_t M, int64_t N, int fmt,
                      double *Xt);
void oracle_bf16_round(const double *in, double *out, int64_t n);
void oracle_mlp_forward(const double *Z, int64_t M, int d0, int d1, int d2, int d3,
                        const double *W1, const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3, int round_bf16_act, int skip,
                        const double *Zskip, double *H1, double *H2, double *O);
double oracle_cos2_loss(const double *O, const double *V, int64_t M, int K, double *dO);
void oracle_mlp_backward(const double *Z, int64_t M, int d0, int d1, int d2, int d3,
                         const double *W1, const double *W2, const double *W3, const double *H1,
                         const double *H2, const double *dO, int round_bf16_grad, double *dW1,
                         double *db1, double *dW2, double *db2, double *dW3, double *db3,
                         double *G1, double *G2);
void oracle_adam(double *w, const double *g, double *m1, double *m2, int64_t n, double lr,
                 double beta1, double beta2, double eps, int t);

static int failures = 0;
#define CHECK(c)                                                                           \
    do {                                                                                   \
        if (!(c)) {                                                                        \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);                \
            ++failures;                                                                    \
        }                                                                                  \
    } while (0)

/* Deterministic uniform numbers in [-1, 1) (64-bit LCG, top 53 bits). */
static uint64_t lcg = 811;
static double urand(void)
{
    lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(lcg >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

static double *alloc_d(size_t n)
{
    double *p = calloc(n ? n : 1, sizeof(double));
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

/* X = sum_i 2^-i a_i b_i^T + 1e-3 noise, column-major with leading dimension ld. */
static double *lowrank(int64_t M, int64_t N, int64_t ld, int rank)
{
    double *X = alloc_d((size_t)(ld * N));
    for (int i = 0; i < rank; ++i) {
        double *a = alloc_d((size_t)M), *b = alloc_d((size_t)N);
        for (int64_t m = 0; m < M; ++m) a[m] = urand();
        for (int64_t n = 0; n < N; ++n) b[n] = urand();
        const double s = ldexp(1.0, -i);
        for (int64_t n = 0; n < N; ++n)
            for (int64_t m = 0; m < M; ++m) X[m + n * ld] += s * a[m] * b[n];
        free(a);
        free(b);
    }
    for (int64_t n = 0; n < N; ++n)
        for (int64_t m = 0; m < M; ++m) X[m + n * ld] += 1e-3 * urand();
    return X;
}

static void fits(void)
{
    const int64_t M = 37, N = 23, ld = 41, K = 6;
    double *X = lowrank(M, N, ld, 8);
    double *T = alloc_d((size_t)(M * K)), *P = alloc_d((size_t)(N * K));
    double *sig = alloc_d((size_t)K), *R = alloc_d((size_t)(M * N));
    double *T0 = alloc_d((size_t)(M * K));
    int32_t iters[6], start[6], rit[6], rst[6];
    for (int64_t i = 0; i < M * K; ++i) T0[i] = urand();
    for (int algo = 0; algo < 2; ++algo)
        for (int implicit = 0; implicit < 2; ++implicit) {
            if (implicit && algo == 1)
                continue;
            for (int init = 0; init < 3; ++init)
                for (int stop = 0; stop < 2; ++stop)
                    for (int reorth = 0; reorth < 3; ++reorth) {
                        const double tol = stop ? 1e-6 : 1e-9;
                        const int r = oracle_fit(algo, implicit, X, M, N, ld, K, tol, 500, init,
                                                 T0, NULL, NULL, 0.0, stop, reorth, T, P, sig,
                                                 iters, start, implicit ? NULL : R);
                        CHECK(r == 0 || r == 1);
                        CHECK(isfinite(sig[0]) && sig[0] > 0.0);
                    }
        }
    /* replay of a free run, with forced start columns */
    int r = oracle_fit(0, 0, X, M, N, ld, K, 1e-9, 500, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P,
                       sig, iters, start, NULL);
    CHECK(r == 0);
    for (int k = 0; k < K; ++k) {
        rit[k] = iters[k];
        rst[k] = (k * 5) % (int)N;
    }
    r = oracle_fit(0, 0, X, M, N, ld, K, 0.0, 500, 0, NULL, rit, rst, 0.0, 0, 0, T, P, sig, iters,
                   start, NULL);
    CHECK(r == 0 || r == 1);
    /* max_iter 1: not converged */
    r = oracle_fit(0, 0, X, M, N, ld, K, 1e-12, 1, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P, sig, iters,
                   start, NULL);
    CHECK(r == 1);
    /* full rank K = N on a small case, and a 1 x 1 */
    {
        const int64_t m2 = 9, n2 = 5;
        double *X2 = lowrank(m2, n2, m2, 5);
        double *T2 = alloc_d((size_t)(m2 * n2)), *P2 = alloc_d((size_t)(n2 * n2));
        double *s2 = alloc_d((size_t)n2);
        int32_t it2[5], st2[5];
        r = oracle_fit(0, 1, X2, m2, n2, m2, n2, 0.0, 200, 0, NULL, NULL, NULL, 0.0, 0, 0, T2, P2, s2,
                       it2, st2, NULL);
        CHECK(r == 0 || r == 1);
        double one = 3.0, t1, p1, s1;
        int32_t i1, c1;
        r = oracle_fit(0, 0, &one, 1, 1, 1, 1, 1e-10, 10, 0, NULL, NULL, NULL, 0.0, 0, 0, &t1, &p1,
                       &s1, &i1, &c1, NULL);
        CHECK(r == 0 && fabs(s1 - 3.0) < 1e-15);
        free(X2); free(T2); free(P2); free(s2);
    }
    /* degenerate: an all-zero matrix; non-finite: a NaN entry; invalid sizes */
    {
        double *Z = alloc_d((size_t)(M * N));
        r = oracle_fit(0, 0, Z, M, N, M, K, 1e-9, 50, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P, sig,
                       iters, start, NULL);
        CHECK(r == 0 && sig[0] == 0.0);
        Z[5] = NAN;
        r = oracle_fit(0, 0, Z, M, N, M, K, 1e-9, 50, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P, sig,
                       iters, start, NULL);
        CHECK(r == -4);
        r = oracle_fit(0, 0, Z, M, N, M, N + 1, 1e-9, 50, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P, sig,
                       iters, start, NULL);
        CHECK(r == -1);
        free(Z);
    }
    /* Gram-Schmidt steps and the isolated score step */
    {
        double x[23];
        for (int reorth = 0; reorth < 3; ++reorth) {
            for (int64_t n = 0; n < N; ++n) x[n] = urand();
            CHECK(oracle_gs_step(P, N, 3, x, reorth) == 0);
        }
        double *v = alloc_d((size_t)M), s = 0.0;
        r = oracle_fit(0, 0, X, M, N, ld, K, 1e-9, 500, 0, NULL, NULL, NULL, 0.0, 0, 0, T, P, sig,
                       iters, start, NULL);
        double *V = alloc_d((size_t)(M * K));
        for (int64_t i = 0; i < M * K; ++i) V[i] = T[i] / sig[i / M];
        CHECK(oracle_score_step(X, M, N, ld, 3, V, sig, P, P + 3 * N, v, &s) == 0);
        CHECK(fabs(s - sig[3]) < 1e-6 * sig[0]);
        free(v);
        free(V);
    }
    free(X); free(T); free(P); free(sig); free(R); free(T0);
}

static void jacobi(void)
{
    const int64_t n = 7;
    double *B = alloc_d((size_t)(n * n)), *A = alloc_d((size_t)(n * n));
    double *w = alloc_d((size_t)n), *Q = alloc_d((size_t)(n * n));
    for (int64_t i = 0; i < n * n; ++i) B[i] = urand();
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j) {
            double s = 0.0;
            for (int64_t l = 0; l < n; ++l) s += B[l + i * n] * B[l + j * n];
            A[i + j * n] = s;
        }
    CHECK(oracle_jacobi_eig(A, n, w, Q) >= 0);
    for (int64_t i = 1; i < n; ++i) CHECK(w[i - 1] >= w[i]);
    free(B); free(A); free(w); free(Q);
}

static void codecs(void)
{
    for (uint32_t c = 0; c < 65536; ++c) {
        const float f = oracle_bf16_decode((uint16_t)c);
        if (isfinite(f)) CHECK(oracle_bf16_encode(f) == (uint16_t)c || f == 0.0f);
    }
    for (uint32_t c = 0; c < 256; ++c) {
        const double d = oracle_e4m3_decode((uint8_t)c);
        if (isfinite(d) && d != 0.0) CHECK(oracle_e4m3_encode((float)d) == (uint8_t)c);
    }
    const int64_t M = 19, N = 7;
    float *X = malloc(sizeof(float) * (size_t)(M * N));
    float *sc = malloc(sizeof(float) * (size_t)N);
    uint16_t *q16 = malloc(2 * (size_t)(M * N));
    uint8_t *q8 = malloc((size_t)(M * N));
    double *Xt = alloc_d((size_t)(M * N)), *out = alloc_d((size_t)(M * N));
    for (int64_t i = 0; i < M * N; ++i) X[i] = (float)(100.0 * urand());
    for (int64_t m = 0; m < M; ++m) X[m + 3 * M] = 0.0f; /* zero column: scale 1 */
    CHECK(oracle_quantize(X, M, N, M, 0, q16, sc) == 0);
    CHECK(oracle_dequantize(q16, sc, M, N, 0, Xt) == 0);
    CHECK(oracle_quantize(X, M, N, M, 1, q8, sc) == 0);
    CHECK(oracle_dequantize(q8, sc, M, N, 1, Xt) == 0);
    CHECK(sc[3] == 1.0f);
    oracle_bf16_round(Xt, out, M * N);
    X[4] = NAN;
    CHECK(oracle_quantize(X, M, N, M, 1, q8, sc) == -4);
    free(X); free(sc); free(q16); free(q8); free(Xt); free(out);
}

static void mlp(void)
{
    const int64_t M = 13;
    const int d0 = 8, d1 = 16, d2 = 12, d3 = 4;
    double *Z = alloc_d((size_t)(M * d0));
    double *W1 = alloc_d((size_t)(d0 * d1)), *b1 = alloc_d((size_t)d1);
    double *W2 = alloc_d((size_t)(d1 * d2)), *b2 = alloc_d((size_t)d2);
    double *W3 = alloc_d((size_t)(d2 * d3)), *b3 = alloc_d((size_t)d3);
    double *H1 = alloc_d((size_t)(M * d1)), *H2 = alloc_d((size_t)(M * d2));
    double *O = alloc_d((size_t)(M * d3)), *V = alloc_d((size_t)(M * d3));
    double *dO = alloc_d((size_t)(M * d3));
    double *gW1 = alloc_d((size_t)(d0 * d1)), *gb1 = alloc_d((size_t)d1);
    double *gW2 = alloc_d((size_t)(d1 * d2)), *gb2 = alloc_d((size_t)d2);
    double *gW3 = alloc_d((size_t)(d2 * d3)), *gb3 = alloc_d((size_t)d3);
    double *G1 = alloc_d((size_t)(M * d1)), *G2 = alloc_d((size_t)(M * d2));
    double *m1 = alloc_d((size_t)(d0 * d1)), *m2 = alloc_d((size_t)(d0 * d1));
    for (int64_t i = 0; i < M * d0; ++i) Z[i] = urand();
    for (int64_t i = 0; i < d0 * d1; ++i) W1[i] = 0.3 * urand();
    for (int64_t i = 0; i < d1 * d2; ++i) W2[i] = 0.3 * urand();
    for (int64_t i = 0; i < d2 * d3; ++i) W3[i] = 0.3 * urand();
    for (int64_t i = 0; i < M * d3; ++i) V[i] = urand();
    for (int rnd = 0; rnd < 2; ++rnd)
        for (int skip = 0; skip < 2; ++skip) {
            oracle_mlp_forward(Z, M, d0, d1, d2, d3, W1, b1, W2, b2, W3, b3, rnd, skip, Z, H1, H2,
                               O);
            const double L = oracle_cos2_loss(O, V, M, d3, dO);
            CHECK(L >= 0.0 && L <= d3 + 1e-12);
            oracle_mlp_backward(Z, M, d0, d1, d2, d3, W1, W2, W3, H1, H2, dO, rnd, gW1, gb1, gW2,
                                gb2, gW3, gb3, G1, G2);
        }
    for (int t = 1; t <= 3; ++t)
        oracle_adam(W1, gW1, m1, m2, d0 * d1, 1e-3, 0.9, 0.999, 1e-8, t);
    double *Ozero = alloc_d((size_t)(M * d3)); /* a zero column adds 1 and no gradient */
    CHECK(fabs(oracle_cos2_loss(Ozero, V, M, d3, dO) - d3) < 1e-12);
    free(Z); free(W1); free(b1); free(W2); free(b2); free(W3); free(b3); free(H1); free(H2);
    free(O); free(V); free(dO); free(gW1); free(gb1); free(gW2); free(gb2); free(gW3); free(gb3);
    free(G1); free(G2); free(m1); free(m2); free(Ozero);
}

int main(void)
{
    fits();
    jacobi();
    codecs();
    mlp();
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitizer run: all paths ok\n");
    return 0;
}
