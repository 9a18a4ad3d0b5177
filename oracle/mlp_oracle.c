/*
 * mlp_oracle.c -- FP64 reference of the warm-start network.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite loads this file; it shares no
 * code with the GPU library.
 *
 * The warm start is not in the paper (whose start vector is a residual
 * column, Secs. 2.2-2.3).  It is this project's learned initial score: a
 * row-wise multilayer perceptron maps each row z_m of a whitened random
 * sketch of X to row m of the K initial scores,
 *     h1 = relu(z W1 + b1), h2 = relu(h1 W2 + b2), o = z[:d3] + h2 W3 + b3
 * (the skip term z[:d3] -- the first d3 inputs -- only when `skip` is set),
 * and is trained with the sign-invariant loss
 *     L = sum_k [ 1 - (o_k . v_k)^2 / (|o_k|^2 |v_k|^2) ]
 * between each output column o_k (over the rows) and the converged
 * normalised score v_k.  relu'(0) = 0.
 *
 * Layout: row-major, samples in rows: Z[m*d0 + i], W1[i*d1 + j], H1[m*d1 + j],
 * O[m*d3 + k], V[m*d3 + k].  If round_bf16_act is non-zero, the stored
 * activations H1, H2 are rounded to bfloat16 (round to nearest even) after the
 * ReLU; if round_bf16_grad is non-zero, so are the masked hidden gradients G2,
 * G1 in the backward pass: the points where a bf16 implementation stores them.
 * Rounding the inputs, weights and dL/dO is left to the caller.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

uint16_t oracle_bf16_encode(float x);
float oracle_bf16_decode(uint16_t c);

static double round_bf16(double x)
{
    return (double)oracle_bf16_decode(oracle_bf16_encode((float)x));
}

/* Y (M x dout) = act(X (M x din) W (din x dout) + b) */
static void layer(const double *X, int64_t M, int din, int dout, const double *W,
                  const double *b, int relu, int rnd, double *Y)
{
    for (int64_t m = 0; m < M; ++m)
        for (int j = 0; j < dout; ++j) {
            double s = b[j];
            for (int i = 0; i < din; ++i)
                s += X[m * din + i] * W[(int64_t)i * dout + j];
            if (relu && !(s > 0.0))
                s = 0.0;
            if (rnd)
                s = round_bf16(s);
            Y[m * dout + j] = s;
        }
}

void oracle_mlp_forward(const double *Z, int64_t M, int d0, int d1, int d2, int d3,
                        const double *W1, const double *b1, const double *W2, const double *b2,
                        const double *W3, const double *b3, int round_bf16_act, int skip,
                        const double *Zskip, double *H1, double *H2, double *O)
{
    layer(Z, M, d0, d1, W1, b1, 1, round_bf16_act, H1);
    layer(H1, M, d1, d2, W2, b2, 1, round_bf16_act, H2);
    layer(H2, M, d2, d3, W3, b3, 0, 0, O);
    if (skip)
        for (int64_t m = 0; m < M; ++m)
            for (int k = 0; k < d3; ++k)
                O[m * d3 + k] += Zskip[m * d0 + k];
}

/* Loss and its gradient dO = dL/dO (M x K). */
double oracle_cos2_loss(const double *O, const double *V, int64_t M, int K, double *dO)
{
    double L = 0.0;
    for (int k = 0; k < K; ++k) {
        double ov = 0.0, oo = 0.0, vv = 0.0;
        for (int64_t m = 0; m < M; ++m) {
            ov += O[m * K + k] * V[m * K + k];
            oo += O[m * K + k] * O[m * K + k];
            vv += V[m * K + k] * V[m * K + k];
        }
        if (!(oo > 0.0) || !(vv > 0.0)) {
            L += 1.0;
            if (dO)
                for (int64_t m = 0; m < M; ++m)
                    dO[m * K + k] = 0.0;
            continue;
        }
        const double c = ov * ov / (oo * vv);
        L += 1.0 - c;
        /* d/do [ -(o.v)^2 / (|o|^2 |v|^2) ] = -2 (o.v) v / (|o|^2|v|^2) + 2 (o.v)^2 o / (|o|^4 |v|^2) */
        if (dO)
            for (int64_t m = 0; m < M; ++m)
                dO[m * K + k] = -2.0 * ov * V[m * K + k] / (oo * vv) +
                                2.0 * ov * ov * O[m * K + k] / (oo * oo * vv);
    }
    return L;
}

/* Backward through the three layers given the stored activations. */
void oracle_mlp_backward(const double *Z, int64_t M, int d0, int d1, int d2, int d3,
                         const double *W1, const double *W2, const double *W3, const double *H1,
                         const double *H2, const double *dO, int round_bf16_grad, double *dW1,
                         double *db1, double *dW2, double *db2, double *dW3, double *db3,
                         double *G1, double *G2)
{
    /* layer 3: O = H2 W3 + b3 */
    for (int i = 0; i < d2; ++i)
        for (int k = 0; k < d3; ++k) {
            double s = 0.0;
            for (int64_t m = 0; m < M; ++m)
                s += H2[m * d2 + i] * dO[m * d3 + k];
            dW3[(int64_t)i * d3 + k] = s;
        }
    for (int k = 0; k < d3; ++k) {
        double s = 0.0;
        for (int64_t m = 0; m < M; ++m)
            s += dO[m * d3 + k];
        db3[k] = s;
    }
    /* G2 = dL/d(pre2) = (dO W3^T) * [H2 > 0] */
    for (int64_t m = 0; m < M; ++m)
        for (int i = 0; i < d2; ++i) {
            double s = 0.0;
            for (int k = 0; k < d3; ++k)
                s += dO[m * d3 + k] * W3[(int64_t)i * d3 + k];
            s = H2[m * d2 + i] > 0.0 ? s : 0.0;
            G2[m * d2 + i] = round_bf16_grad ? round_bf16(s) : s;
        }
    for (int i = 0; i < d1; ++i)
        for (int j = 0; j < d2; ++j) {
            double s = 0.0;
            for (int64_t m = 0; m < M; ++m)
                s += H1[m * d1 + i] * G2[m * d2 + j];
            dW2[(int64_t)i * d2 + j] = s;
        }
    for (int j = 0; j < d2; ++j) {
        double s = 0.0;
        for (int64_t m = 0; m < M; ++m)
            s += G2[m * d2 + j];
        db2[j] = s;
    }
    /* G1 = (G2 W2^T) * [H1 > 0] */
    for (int64_t m = 0; m < M; ++m)
        for (int i = 0; i < d1; ++i) {
            double s = 0.0;
            for (int j = 0; j < d2; ++j)
                s += G2[m * d2 + j] * W2[(int64_t)i * d2 + j];
            s = H1[m * d1 + i] > 0.0 ? s : 0.0;
            G1[m * d1 + i] = round_bf16_grad ? round_bf16(s) : s;
        }
    for (int i = 0; i < d0; ++i)
        for (int j = 0; j < d1; ++j) {
            double s = 0.0;
            for (int64_t m = 0; m < M; ++m)
                s += Z[m * d0 + i] * G1[m * d1 + j];
            dW1[(int64_t)i * d1 + j] = s;
        }
    for (int j = 0; j < d1; ++j) {
        double s = 0.0;
        for (int64_t m = 0; m < M; ++m)
            s += G1[m * d1 + j];
        db1[j] = s;
    }
}

/* Adam step on FP64 parameters (Kingma & Ba), t = step number starting at 1. */
void oracle_adam(double *w, const double *g, double *m1, double *m2, int64_t n, double lr,
                 double beta1, double beta2, double eps, int t)
{
    const double c1 = 1.0 - pow(beta1, t), c2 = 1.0 - pow(beta2, t);
    for (int64_t i = 0; i < n; ++i) {
        m1[i] = beta1 * m1[i] + (1.0 - beta1) * g[i];
        m2[i] = beta2 * m2[i] + (1.0 - beta2) * g[i] * g[i];
        w[i] -= lr * (m1[i] / c1) / (sqrt(m2[i] / c2) + eps);
    }
}
