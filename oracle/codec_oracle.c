/*
 * codec_oracle.c -- reference encoders/decoders for the reduced-precision
 * storage of X (BF16 and OCP FP8 E4M3 "fn") with per-column FP32 scales.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite and the benchmark's CPU-baseline
 * leg load this file; it shares no code with the GPU library.
 *
 * The storage form is not in the paper (whose Sec. 3 notes only that the
 * double-precision programs convert directly to single precision); it is
 * this project's reduced-precision variant of the residual products.
 * Formats, from their public definitions:
 *   - bfloat16: the upper 16 bits of an IEEE binary32 (1 sign, 8 exponent,
 *     7 fraction bits); conversion rounds to nearest, ties to even.
 *   - E4M3 "fn" (OCP 8-bit floating point, v1.0): 1 sign, 4 exponent bits
 *     (bias 7), 3 fraction bits; no infinities; S.1111.111 is NaN; largest
 *     finite magnitude 448; subnormals (exponent field 0) are m/8 * 2^-6.
 *     Encoding here rounds to nearest, ties to even, and saturates to +-448.
 * Per-column scale: s_j = amax_j / Qmax (binary32), Qmax = 448 for E4M3 and
 * 1 for BF16; an all-zero column has s_j = 1.  Code = encode(x / s_j) with
 * the division in binary32.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static uint32_t f32_bits(float x) { uint32_t u; memcpy(&u, &x, 4); return u; }
static float bits_f32(uint32_t u) { float x; memcpy(&x, &u, 4); return x; }

float oracle_bf16_decode(uint16_t c) { return bits_f32((uint32_t)c << 16); }

/* Round-to-nearest-even on the 16 discarded bits. */
uint16_t oracle_bf16_encode(float x)
{
    uint32_t u = f32_bits(x);
    if (isnan(x))
        return (uint16_t)((u >> 16) | 0x0040u); /* quiet NaN, sign kept */
    const uint32_t upper = u >> 16, lower = u & 0xFFFFu;
    uint32_t r = upper;
    if (lower > 0x8000u || (lower == 0x8000u && (upper & 1u)))
        r = upper + 1u; /* carries into the exponent correctly, to Inf at the top */
    return (uint16_t)r;
}

double oracle_e4m3_decode(uint8_t c)
{
    const int s = (c >> 7) & 1, e = (c >> 3) & 0xF, m = c & 7;
    double v;
    if (e == 0xF && m == 7)
        return NAN;
    if (e == 0)
        v = ldexp((double)m / 8.0, -6);
    else
        v = ldexp(1.0 + (double)m / 8.0, e - 7);
    return s ? -v : v;
}

/* The 127 finite non-negative E4M3 values, indexed by code: they increase
 * with the code (exponent field above fraction field). */
static void e4m3_table(double tab[127])
{
    for (int c = 0; c <= 0x7E; ++c)
        tab[c] = oracle_e4m3_decode((uint8_t)c);
}

/* Nearest representable magnitude, ties to the code with an even fraction
 * field; values at or above 448 saturate to 448.  The bracketing pair
 * tab[lo] <= |x| < tab[lo + 1] is found by bisection of the increasing table,
 * and the nearer of the two is taken. */
static uint8_t e4m3_encode_tab(float x, const double tab[127])
{
    if (isnan(x))
        return 0x7F;
    const int neg = signbit(x) ? 1 : 0;
    const double a = fabs((double)x);
    if (a >= 448.0)
        return (uint8_t)(0x7E | (neg << 7));
    int lo = 0, hi = 0x7E; /* tab[lo] <= a < tab[hi] */
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (tab[mid] <= a)
            lo = mid;
        else
            hi = mid;
    }
    const double dlo = a - tab[lo], dhi = tab[hi] - a;
    int best;
    if (dlo < dhi)
        best = lo;
    else if (dhi < dlo)
        best = hi;
    else
        best = (lo & 1) == 0 ? lo : hi;
    return (uint8_t)(best | (neg << 7));
}

uint8_t oracle_e4m3_encode(float x)
{
    double tab[127];
    e4m3_table(tab);
    return e4m3_encode_tab(x, tab);
}

/* fmt 0 = BF16 (codes uint16), 1 = E4M3 (codes uint8).  X binary32 column-major
 * (ld >= M); codes column-major with leading dimension M. */
int oracle_quantize(const float *X, int64_t M, int64_t N, int64_t ldx, int fmt,
                    void *codes, float *scale)
{
    if (!X || !codes || !scale || M < 1 || N < 1 || ldx < M || (fmt != 0 && fmt != 1))
        return -1;
    const float qmax = fmt == 1 ? 448.0f : 1.0f;
    double tab[127];
    e4m3_table(tab);
    for (int64_t n = 0; n < N; ++n) {
        float amax = 0.0f;
        int bad = 0;
        for (int64_t m = 0; m < M; ++m) {
            const float a = fabsf(X[m + n * ldx]);
            if (!isfinite(a))
                bad = 1; /* NaN or Inf anywhere in the column */
            else if (a > amax)
                amax = a;
        }
        if (bad)
            return -4;
        const float s = amax > 0.0f ? amax / qmax : 1.0f;
        scale[n] = s;
        for (int64_t m = 0; m < M; ++m) {
            const float q = X[m + n * ldx] / s;
            if (fmt == 0)
                ((uint16_t *)codes)[m + n * M] = oracle_bf16_encode(q);
            else
                ((uint8_t *)codes)[m + n * M] = e4m3_encode_tab(q, tab);
        }
    }
    return 0;
}

/* Dequantised matrix x~ = decode(code) * s_j, exact in binary64. */
int oracle_dequantize(const void *codes, const float *scale, int64_t M, int64_t N, int fmt,
                      double *Xt)
{
    if (!codes || !scale || !Xt || M < 1 || N < 1 || (fmt != 0 && fmt != 1))
        return -1;
    double dec8[256];
    for (int c = 0; c < 256; ++c)
        dec8[c] = oracle_e4m3_decode((uint8_t)c);
    for (int64_t n = 0; n < N; ++n)
        for (int64_t m = 0; m < M; ++m) {
            const double d = fmt == 0 ? (double)oracle_bf16_decode(((const uint16_t *)codes)[m + n * M])
                                      : dec8[((const uint8_t *)codes)[m + n * M]];
            Xt[m + n * M] = d * (double)scale[n];
        }
    return 0;
}

/* out[i] = bf16(fl32(in[i])) as a double: the value an FP64 number takes when
 * it is stored as FP32 and then as bfloat16 (both round to nearest even). */
void oracle_bf16_round(const double *in, double *out, int64_t n)
{
    for (int64_t i = 0; i < n; ++i)
        out[i] = (double)oracle_bf16_decode(oracle_bf16_encode((float)in[i]));
}
