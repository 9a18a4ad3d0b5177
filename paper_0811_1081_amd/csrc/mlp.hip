// mlp.hip -- learned warm start (not in the paper, whose start vector is a
// residual column, Secs. 2.2-2.3): a whitened random sketch of X and a small
// row-wise multilayer perceptron that predicts the initial scores, with its
// training step.  The C ABI is declared in gspca_ws.h.
//
// The network's products run on bfloat16 matrix cores
// (v_mfma_f32_16x16x32_bf16, FP32 accumulation).  bf16 rounding points: the
// input rows, the weights, the stored hidden activations, the incoming
// gradient dL/do and the masked hidden gradients.  Biases, outputs and
// parameter gradients are FP32; weight gradients reduce over the rows with a
// split-K scheme whose partial sums are added in a fixed order, so a step is
// deterministic.
#include <float.h>
#include <hip/hip_bf16.h>
#include <math.h>

#include <algorithm>

#include "../../include/gspca_ws.h"
#include "internal.h"

namespace gspca {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float mf32x4_t __attribute__((ext_vector_type(4)));

__device__ inline __bf16 to_bf16(float x)
{
    const __hip_bfloat16 h = __float2bfloat16(x);
    return *reinterpret_cast<const __bf16 *>(&h);
}
__device__ inline __bf16 to_bf16(__bf16 x) { return x; }

// ---------------------------------------------------------------------------
// C = A B (+ bias, relu, mask) with bf16 operands and FP32 accumulation.
// A(i, k) = A[i*a_r + k*a_c] (M x Kd), B(k, j) = B[k*b_r + j*b_c] (Kd x N);
// strides express the transposes of the backward pass.  FP32 operands are
// rounded to bf16 as they are loaded.  A workgroup computes a 64 x 64 tile of
// C, each of its four waves a 32 x 32 quarter as 2 x 2 matrix-core tiles
// (v_mfma_f32_16x16x32_bf16).  Per 32-wide k chunk both operands are staged
// in LDS in k-contiguous bf16 rows, read from global memory along whichever
// index is contiguous (16-byte loads when the rows are aligned), so every
// lane then takes its eight k values of A and of B with one 16-byte LDS
// read.  blockIdx.z splits the k range into chunks of `kchunk` (a multiple
// of 32):
//   - split == 0: C(i, j) at Cf[i*c_r + j*c_c] (FP32, + bias, + skip(i, j) =
//     skip[i*s_r + j], relu, mask, optionally added to the old value) or Cb
//     (bf16); mask zeroes C(i, j) where the stored activation mask[i*m_r + j]
//     is not positive;
//   - split != 0: raw partial sums to part[z*M*N + i*N + j].
constexpr int kGemmTile = 64, kGemmK = 32, kGemmLdk = kGemmK + 8; // LDS row: 80 bytes

// Rows o0..o0+63 (outer index, stride so; bound no) by k0..k0+31 (stride sk;
// bound kend) of an operand into dst[o][k] as bf16, zero outside.
template <typename T>
__device__ inline void gemm_stage(const T *__restrict__ X, int64_t so, int64_t sk, int64_t o0,
                                  int64_t no, int64_t k0, int64_t kend,
                                  __bf16 (*dst)[kGemmLdk], int tid)
{
    if (sk == 1) {
        // k contiguous: thread -> outer row tid / 4, eight k from 8 (tid % 4)
        const int o = tid >> 2, seg = tid & 3;
        const int64_t og = o0 + o, kg = k0 + 8 * seg;
        bf16x8_t v;
        const T *src = X + (og < no ? og : 0) * so + kg;
        if (og < no && kg + 8 <= kend && ((uintptr_t)src & 15) == 0) {
            if constexpr (sizeof(T) == 2) {
                v = *reinterpret_cast<const bf16x8_t *>(src);
            } else {
                const mf32x4_t lo = *reinterpret_cast<const mf32x4_t *>(src);
                const mf32x4_t hi = *reinterpret_cast<const mf32x4_t *>(src + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = to_bf16(lo[e]);
                    v[4 + e] = to_bf16(hi[e]);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v[e] = (og < no && kg + e < kend) ? to_bf16(src[e]) : (__bf16)0.0f;
        }
        *reinterpret_cast<bf16x8_t *>(&dst[o][8 * seg]) = v;
    } else if (so == 1) {
        // outer index contiguous: thread -> k row tid / 8, eight outer
        // indices from 8 (tid % 8), written transposed
        const int kk = tid >> 3, seg = tid & 7;
        const int64_t kg = k0 + kk, og = o0 + 8 * seg;
        const T *src = X + (kg < kend ? kg : 0) * sk + og;
        bf16x8_t v;
        if (kg < kend && og + 8 <= no && ((uintptr_t)src & 15) == 0) {
            if constexpr (sizeof(T) == 2) {
                v = *reinterpret_cast<const bf16x8_t *>(src);
            } else {
                const mf32x4_t lo = *reinterpret_cast<const mf32x4_t *>(src);
                const mf32x4_t hi = *reinterpret_cast<const mf32x4_t *>(src + 4);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    v[e] = to_bf16(lo[e]);
                    v[4 + e] = to_bf16(hi[e]);
                }
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                v[e] = (kg < kend && og + e < no) ? to_bf16(src[e]) : (__bf16)0.0f;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
            dst[8 * seg + e][kk] = v[e];
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int idx = tid + 256 * e, o = idx >> 5, kk = idx & 31;
            const int64_t og = o0 + o, kg = k0 + kk;
            dst[o][kk] = (og < no && kg < kend) ? to_bf16(X[og * so + kg * sk]) : (__bf16)0.0f;
        }
    }
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void k_gemm_bf16(
    const TA *__restrict__ A, int64_t a_r, int64_t a_c, const TB *__restrict__ B, int64_t b_r,
    int64_t b_c, int64_t M, int64_t N, int64_t Kd, int64_t kchunk, const float *__restrict__ bias,
    int relu, const __bf16 *__restrict__ mask, int64_t m_r, const float *__restrict__ skip,
    int64_t s_r, float *__restrict__ Cf, __bf16 *__restrict__ Cb, int64_t c_r, int64_t c_c,
    int accumulate, int split, float *__restrict__ part)
{
    __shared__ __align__(16) __bf16 As[kGemmTile][kGemmLdk];
    __shared__ __align__(16) __bf16 Bs[kGemmTile][kGemmLdk];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t ib = (int64_t)blockIdx.y * kGemmTile, jb = (int64_t)blockIdx.x * kGemmTile;
    const int wi = (w >> 1) * 32, wj = (w & 1) * 32; // the wave's quarter of the tile
    const int li = lane & 15, kq = (lane >> 4) * 8;  // operand row/column, its 8 k
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = std::min<int64_t>(Kd, kbeg + kchunk);
    mf32x4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
            acc[a][b] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = kbeg; k0 < kend; k0 += kGemmK) {
        __syncthreads(); // the previous chunk's operand reads are done
        gemm_stage<TA>(A, a_r, a_c, ib, M, k0, kend, As, tid);
        gemm_stage<TB>(B, b_c, b_r, jb, N, k0, kend, Bs, tid); // Bs[j][k] = B(k, j)
        __syncthreads();
        bf16x8_t av[2], bv[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            av[t] = *reinterpret_cast<const bf16x8_t *>(&As[wi + 16 * t + li][kq]);
            bv[t] = *reinterpret_cast<const bf16x8_t *>(&Bs[wj + 16 * t + li][kq]);
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0,
                                                                     0);
    }
    // lane holds C(i0 + (lane/16)*4 + e, j0 + lane%16), e = 0..3, per tile
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) {
            const int64_t i0 = ib + wi + 16 * ta, j = jb + wj + 16 * tb + li;
            if (j >= N)
                continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int64_t i = i0 + (lane >> 4) * 4 + e;
                if (i >= M)
                    continue;
                float v = acc[ta][tb][e];
                if (split) {
                    part[(int64_t)blockIdx.z * M * N + i * N + j] = v;
                    continue;
                }
                if (bias)
                    v += bias[j];
                if (skip)
                    v += skip[i * s_r + j];
                if (relu && !(v > 0.0f))
                    v = 0.0f;
                if (mask && !((float)mask[i * m_r + j] > 0.0f))
                    v = 0.0f;
                if (Cf) {
                    float *dst = Cf + i * c_r + j * c_c;
                    *dst = accumulate ? *dst + v : v;
                } else {
                    Cb[i * c_r + j * c_c] = to_bf16(v);
                }
            }
        }
}

// C(i, j) = sum_z part[z][i][j] in increasing z (FP32, row-major M x N out
// with strides c_r, c_c).
__global__ __launch_bounds__(256) void k_split_reduce(const float *__restrict__ part, int nz,
                                                      int64_t M, int64_t N, float *__restrict__ C,
                                                      int64_t c_r, int64_t c_c)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= M * N)
        return;
    float s = 0.0f;
    for (int z = 0; z < nz; ++z)
        s += part[(int64_t)z * M * N + e];
    const int64_t i = e / N, j = e % N;
    C[i * c_r + j * c_c] = s;
}

// Column sums of a row-major rows x N matrix: block (x, z) sums columns
// [64x, 64x + 64) over its row range; partials part[z*N + j].
template <typename T>
__global__ __launch_bounds__(256) void k_colsum_part(const T *__restrict__ G, int64_t rows,
                                                     int64_t N, int64_t rchunk,
                                                     float *__restrict__ part)
{
    __shared__ float red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int64_t r0 = (int64_t)blockIdx.z * rchunk;
    const int64_t r1 = std::min<int64_t>(rows, r0 + rchunk);
    float s = 0.0f;
    if (j < N)
        for (int64_t r = r0 + w; r < r1; r += 4)
            s += (float)G[r * N + j];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N)
        part[(int64_t)blockIdx.z * N + j] = red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// Loss and dL/dO for matrix b and column k.  O row-major rows x K (FP32),
// V column-major per matrix (V[b*Mi*K + m + k*Mi]); dO row-major bf16, scaled
// by `inv` (1 / number of matrices).
__global__ __launch_bounds__(256) void k_cos2(const float *__restrict__ O,
                                              const float *__restrict__ V, int64_t Mi, int K,
                                              double inv, __bf16 *__restrict__ dO,
                                              double *__restrict__ loss_part)
{
    __shared__ double red[3][4];
    const int k = blockIdx.x, b = blockIdx.y;
    const int64_t r0 = (int64_t)b * Mi;
    const float *v = V + (int64_t)b * Mi * K + (int64_t)k * Mi;
    double ov = 0.0, oo = 0.0, vv = 0.0;
    for (int64_t m = threadIdx.x; m < Mi; m += 256) {
        const double o = O[(r0 + m) * K + k], x = v[m];
        ov += o * x;
        oo += o * o;
        vv += x * x;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        ov += __shfl_xor(ov, o, 64);
        oo += __shfl_xor(oo, o, 64);
        vv += __shfl_xor(vv, o, 64);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[0][w] = ov;
        red[1][w] = oo;
        red[2][w] = vv;
    }
    __syncthreads();
    ov = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    oo = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    vv = red[2][0] + red[2][1] + red[2][2] + red[2][3];
    const bool ok = oo > 0.0 && vv > 0.0 && isfinite(oo) && isfinite(vv);
    // d/do [-(o.v)^2 / (|o|^2 |v|^2)] = -2 (o.v) v / (|o|^2 |v|^2) + 2 (o.v)^2 o / (|o|^4 |v|^2)
    const double a = ok ? -2.0 * ov / (oo * vv) * inv : 0.0;
    const double c = ok ? 2.0 * ov * ov / (oo * oo * vv) * inv : 0.0;
    for (int64_t m = threadIdx.x; m < Mi; m += 256) {
        const double g = a * (double)v[m] + c * (double)O[(r0 + m) * K + k];
        dO[(r0 + m) * K + k] = to_bf16((float)g);
    }
    if (threadIdx.x == 0)
        loss_part[(int64_t)b * K + k] = ok ? 1.0 - ov * ov / (oo * vv) : 1.0;
}

// loss = (sum of the parts in index order) * inv.  One thread.
__global__ void k_loss_mean(const double *__restrict__ part, int64_t n, double inv,
                            double *__restrict__ loss)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += part[i];
    *loss = s * inv;
}

// Adam (Kingma & Ba) on FP32 master weights; bf16 copy refreshed.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, const float *__restrict__ g,
                                              float *__restrict__ m1, float *__restrict__ m2,
                                              __bf16 *__restrict__ wb, int64_t n, float lr,
                                              float beta1, float beta2, float eps, float c1,
                                              float c2)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n)
        return;
    const float gi = g[i];
    const float a = beta1 * m1[i] + (1.0f - beta1) * gi;
    const float b = beta2 * m2[i] + (1.0f - beta2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    const float v = w[i] - lr * (a / c1) / (sqrtf(b / c2) + eps);
    w[i] = v;
    wb[i] = to_bf16(v);
}

__global__ __launch_bounds__(256) void k_to_bf16(const float *__restrict__ x,
                                                 __bf16 *__restrict__ y, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n)
        y[i] = to_bf16(x[i]);
}

// ---------------------------------------------------------------------------
// Sketch and whitening.

// Y = X Omega (M x R, row-major) for column-major X and row-major N x R
// Omega.  Workgroup b owns rows [64b, 64b + 64): 32-column tiles of X (read
// along the rows) and the matching 32 rows of Omega are staged in LDS, and
// each of the 256 threads accumulates a 4 x (R/16) block of Y in FP32.
template <int R>
__global__ __launch_bounds__(256) void k_sketch(const float *__restrict__ X, int64_t ldx,
                                                int64_t M, int64_t N, const float *__restrict__ Om,
                                                float *__restrict__ Y)
{
    constexpr int RB = R / 16;
    __shared__ float xs[32][65];
    __shared__ float os[32][R + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4; // rows 4tx..4tx+3, sketch columns RB*ty..
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    float acc[4][RB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b)
            acc[a][b] = 0.0f;
    for (int64_t j0 = 0; j0 < N; j0 += 32) {
        __syncthreads();
        for (int e = tid; e < 32 * 64; e += 256) { // X tile, rows fastest
            const int i = e & 63, c = e >> 6;
            const int64_t m = m0 + i, j = j0 + c;
            xs[c][i] = (m < M && j < N) ? X[m + j * ldx] : 0.0f;
        }
        for (int e = tid; e < 32 * R; e += 256) { // Omega tile, sketch columns fastest
            const int c = e / R, col = e % R;
            const int64_t j = j0 + c;
            os[c][col] = j < N ? Om[j * R + col] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 32; ++c) {
            float xv[4], ov[RB];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                xv[a] = xs[c][4 * tx + a];
#pragma unroll
            for (int b = 0; b < RB; ++b)
                ov[b] = os[c][RB * ty + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b)
                    acc[a][b] += xv[a] * ov[b];
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t m = m0 + 4 * tx + a;
        if (m < M)
#pragma unroll
            for (int b = 0; b < RB; ++b)
                Y[m * R + RB * ty + b] = acc[a][b];
    }
}

// W = s X^T Z (N x R, row-major) for a row-major M x R sketch Z, as partial
// sums over row slices.  Workgroup (b, y) owns columns [64b, 64b + 64) of X
// over row slice y: 32-row tiles of X (64 columns, read along the rows) and
// of Z (R columns) are staged in LDS, and each of the 256 threads accumulates
// a 4 x (R/16) block in FP32; slice y's block goes to W + y*N*R.
template <int R>
__global__ __launch_bounds__(256) void k_sketch_t(const float *__restrict__ X, int64_t ldx,
                                                  int64_t M, int64_t N,
                                                  const float *__restrict__ Z, float s,
                                                  int64_t rows, float *__restrict__ W)
{
    constexpr int RB = R / 16; // sketch columns per thread
    __shared__ float xs[32][65];
    __shared__ float zs[32][R + 1];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4; // X columns 4tx..4tx+3, sketch columns RB*ty..
    const int64_t j0 = (int64_t)blockIdx.x * 64;
    float acc[4][RB];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b)
            acc[a][b] = 0.0f;
    // row slice blockIdx.y: rows [y*rows, y*rows + rows); W gets slice y's partial
    const int64_t rb = (int64_t)blockIdx.y * rows;
    const int64_t re = M < rb + rows ? M : rb + rows;
    W += (int64_t)blockIdx.y * N * R;
    for (int64_t r0 = rb; r0 < re; r0 += 32) {
        __syncthreads();
        for (int e = tid; e < 32 * 64; e += 256) { // X tile, rows fastest
            const int i = e & 31, c = e >> 5;
            const int64_t m = r0 + i, j = j0 + c;
            xs[i][c] = (m < re && j < N) ? X[m + j * ldx] : 0.0f;
        }
        for (int e = tid; e < 32 * R; e += 256) { // Z tile, sketch columns fastest
            const int i = e / R, c = e % R;
            const int64_t m = r0 + i;
            zs[i][c] = m < re ? Z[m * R + c] : 0.0f;
        }
        __syncthreads();
#pragma unroll 4
        for (int i = 0; i < 32; ++i) {
            float xv[4], zv[RB];
#pragma unroll
            for (int a = 0; a < 4; ++a)
                xv[a] = xs[i][4 * tx + a];
#pragma unroll
            for (int b = 0; b < RB; ++b)
                zv[b] = zs[i][RB * ty + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < RB; ++b)
                    acc[a][b] += xv[a] * zv[b];
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t j = j0 + 4 * tx + a;
        if (j < N)
#pragma unroll
            for (int b = 0; b < RB; ++b)
                W[j * R + RB * ty + b] = acc[a][b] * s;
    }
}

// The two sketch products when X's columns are 16-byte aligned (ldx a
// multiple of 4), on the FP32 matrix cores (v_mfma_f32_16x16x4f32:
// D(16x16) += A(16x4) B(4x16), FP32 operands and accumulation; lane l
// supplies A(l % 16, l / 16) and B(l / 16, l % 16) and holds
// D(4 (l / 16) + i, l % 16) in its i-th accumulator).  Chunks of BK columns
// (Y = X Om) or BK rows (W = X^T Z) of X and the matching rows of Om or Z are
// staged in two LDS buffers with 16-byte loads, the next chunk's loads in
// flight while the current one is multiplied (one barrier per chunk), and
// each chunk is BK / 4 matrix-core steps of k = 4.  The products and sums
// are FP32 as in k_sketch / k_sketch_t, in another order.  At 65536 x 8192,
// r = 64, Y = X Om takes ~0.80 ms with 32-column chunks against ~1.02 ms with
// 16 (same process, calls separated by idle gaps); W = X^T Z keeps 16-row
// chunks (~0.69 ms; 32 rows, which would read whole 128-byte lines of each
// column, halve the workgroups per CU and were not faster).

// Y = X Om, X's columns 16-byte aligned: workgroup = 64 rows of Y; wave w
// owns rows 16w..16w+15 and all R columns (R/16 tiles of 16).  Chunks of BK
// columns.
template <int R, int BK>
__global__ __launch_bounds__(256) void k_sketch_m(const float *__restrict__ X, int64_t ldx,
                                                  int64_t M, int64_t N,
                                                  const float *__restrict__ Om,
                                                  float *__restrict__ Y)
{
    constexpr int BM = 64, RT = R / 16;
    constexpr int XL = BK * BM / 4 / 256;                // float4 loads of X per thread
    constexpr int OQ = BK * R / 4, OL = (OQ + 255) / 256; // of Om
    // rows padded by 16 floats: the four k rows a wave reads at once fall in
    // different halves of the 32 banks
    __shared__ __align__(16) float xs[2][BK][BM + 16];
    __shared__ __align__(16) float os[2][BK][R + 16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t m0 = (int64_t)blockIdx.x * BM;
    mf32x4_t xr[XL], orr[OL];
#pragma unroll
    for (int u = 0; u < OL; ++u)
        orr[u] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
    auto gload = [&](int64_t j0) {
#pragma unroll
        for (int v = 0; v < XL; ++v) { // column c, rows 4q..4q+3 of the tile
            const int e = tid + 256 * v, c = e >> 4, q = e & 15;
            const int64_t m = m0 + 4 * q, j = j0 + c;
            if (j < N && m + 3 < M) {
                xr[v] = *reinterpret_cast<const mf32x4_t *>(X + m + j * ldx);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    xr[v][u] = (j < N && m + u < M) ? X[m + u + j * ldx] : 0.0f;
            }
        }
#pragma unroll
        for (int v = 0; v < OL; ++v) { // Omega row c, columns 4u..4u+3
            const int e = tid + 256 * v;
            if (e < OQ) {
                const int c = e / (R / 4), u = e % (R / 4);
                const int64_t j = j0 + c;
                if (j < N)
                    orr[v] = *reinterpret_cast<const mf32x4_t *>(Om + j * R + 4 * u);
                else
                    orr[v] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    auto sstore = [&](int b) {
#pragma unroll
        for (int v = 0; v < XL; ++v) {
            const int e = tid + 256 * v, c = e >> 4, q = e & 15;
            *reinterpret_cast<mf32x4_t *>(&xs[b][c][4 * q]) = xr[v];
        }
#pragma unroll
        for (int v = 0; v < OL; ++v) {
            const int e = tid + 256 * v;
            if (e < OQ) {
                const int c2 = e / (R / 4), u = e % (R / 4);
                *reinterpret_cast<mf32x4_t *>(&os[b][c2][4 * u]) = orr[v];
            }
        }
    };
    mf32x4_t acc[RT];
#pragma unroll
    for (int t = 0; t < RT; ++t)
        acc[t] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
    gload(0);
    sstore(0);
    __syncthreads();
    int buf = 0;
    for (int64_t j0 = 0; j0 < N; j0 += BK) {
        const bool more = j0 + BK < N;
        if (more)
            gload(j0 + BK); // in flight while this chunk is multiplied
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            const float a = xs[buf][kk + lk][16 * w + li];
#pragma unroll
            for (int t = 0; t < RT; ++t)
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, os[buf][kk + lk][16 * t + li],
                                                              acc[t], 0, 0, 0);
        }
        if (more)
            sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t m = m0 + 16 * w + 4 * lk + i;
        if (m < M)
#pragma unroll
            for (int t = 0; t < RT; ++t)
                Y[m * R + 16 * t + li] = acc[t][i];
    }
}

// W = s X^T Z over row slice y (partial sums as k_sketch_t), X's columns
// 16-byte aligned: workgroup (b, y) = 128 columns of X; wave w owns columns
// 32w..32w+31 (two tiles of 16) and all R sketch columns.  Chunks of BK rows
// (BK = 32: whole 128-byte lines of each column).
template <int R, int BK>
__global__ __launch_bounds__(256) void k_sketch_t_m(const float *__restrict__ X, int64_t ldx,
                                                    int64_t M, int64_t N,
                                                    const float *__restrict__ Z, float s,
                                                    int64_t rows, float *__restrict__ W)
{
    constexpr int BN = 128, RT = R / 16;
    constexpr int XL = BK * BN / 4 / 256;                 // float4 loads of X per thread
    constexpr int ZQ = BK * R / 4, ZL = (ZQ + 255) / 256; // of Z
    constexpr int QC = BK / 4;                            // float4 per column of a chunk
    __shared__ __align__(16) float xs[2][BK][BN + 16]; // padded as in k_sketch_m
    __shared__ __align__(16) float zs[2][BK][R + 16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t j0 = (int64_t)blockIdx.x * BN;
    const int64_t rb = (int64_t)blockIdx.y * rows;
    const int64_t re = M < rb + rows ? M : rb + rows;
    W += (int64_t)blockIdx.y * N * R;
    mf32x4_t xr[XL], zr[ZL];
#pragma unroll
    for (int u = 0; u < ZL; ++u)
        zr[u] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
    auto gload = [&](int64_t r0) {
#pragma unroll
        for (int h = 0; h < XL; ++h) { // column c, rows 4q..4q+3 of the chunk
            const int e = tid + 256 * h, c = e / QC, q = e % QC;
            const int64_t m = r0 + 4 * q, j = j0 + c;
            if (j < N && m + 3 < re) {
                xr[h] = *reinterpret_cast<const mf32x4_t *>(X + m + j * ldx);
            } else {
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    xr[h][u] = (j < N && m + u < re) ? X[m + u + j * ldx] : 0.0f;
            }
        }
#pragma unroll
        for (int v = 0; v < ZL; ++v) { // Z row c, columns 4u..4u+3
            const int e = tid + 256 * v;
            if (e < ZQ) {
                const int c = e / (R / 4), u = e % (R / 4);
                const int64_t m = r0 + c;
                if (m < re)
                    zr[v] = *reinterpret_cast<const mf32x4_t *>(Z + m * R + 4 * u);
                else
                    zr[v] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
            }
        }
    };
    auto sstore = [&](int b) {
#pragma unroll
        for (int h = 0; h < XL; ++h) {
            const int e = tid + 256 * h, c = e / QC, q = e % QC;
#pragma unroll
            for (int u = 0; u < 4; ++u)
                xs[b][4 * q + u][c] = xr[h][u];
        }
#pragma unroll
        for (int v = 0; v < ZL; ++v) {
            const int e = tid + 256 * v;
            if (e < ZQ) {
                const int c = e / (R / 4), u = e % (R / 4);
                *reinterpret_cast<mf32x4_t *>(&zs[b][c][4 * u]) = zr[v];
            }
        }
    };
    mf32x4_t acc[2][RT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int t = 0; t < RT; ++t)
            acc[h][t] = mf32x4_t{0.f, 0.f, 0.f, 0.f};
    if (rb < re) {
        gload(rb);
        sstore(0);
    }
    __syncthreads();
    int buf = 0;
    for (int64_t r0 = rb; r0 < re; r0 += BK) {
        const bool more = r0 + BK < re;
        if (more)
            gload(r0 + BK); // in flight while this chunk is multiplied
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            float zb[RT];
#pragma unroll
            for (int t = 0; t < RT; ++t)
                zb[t] = zs[buf][kk + lk][16 * t + li];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const float a = xs[buf][kk + lk][32 * w + 16 * h + li];
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    acc[h][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, zb[t], acc[h][t], 0, 0, 0);
            }
        }
        if (more)
            sstore(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t j = j0 + 32 * w + 16 * h + 4 * lk + i;
            if (j < N)
#pragma unroll
                for (int t = 0; t < RT; ++t)
                    W[j * R + 16 * t + li] = acc[h][t][i] * s;
        }
}

// G_y = Y[rows of slice y]^T Y[rows of slice y] in FP64 (products of FP32
// values are exact in FP64; only the order of the sums rounds).  64-row tiles
// are staged in LDS as doubles; four groups of 256 threads take rows i = g,
// g + 4, ... of each tile, each thread an (R/16) x (R/16) block of G_y, and
// the groups' blocks are added in group order at the end.
template <int R>
__global__ __launch_bounds__(1024) void k_gram(const float *__restrict__ Y, int64_t M,
                                               int64_t rows, double *__restrict__ part)
{
    constexpr int TB = R / 16, NG = 4;
    __shared__ __align__(16) double ys[64][R + 2];
    __shared__ double accs[NG - 1][R * R];
    const int tid = threadIdx.x, g = tid >> 8, t = tid & 255, ta = t & 15, tb = t >> 4;
    const int64_t rb = (int64_t)blockIdx.x * rows;
    const int64_t re = M < rb + rows ? M : rb + rows;
    double acc[TB][TB];
#pragma unroll
    for (int a = 0; a < TB; ++a)
#pragma unroll
        for (int b = 0; b < TB; ++b)
            acc[a][b] = 0.0;
    for (int64_t r0 = rb; r0 < re; r0 += 64) {
        __syncthreads();
        for (int e = tid; e < 64 * R; e += 1024) {
            const int i = e / R, c = e % R;
            const int64_t m = r0 + i;
            ys[i][c] = m < re ? (double)Y[m * R + c] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int i = g; i < 64; i += NG) {
            double ya[TB], yb[TB];
#pragma unroll
            for (int a = 0; a < TB; ++a)
                ya[a] = ys[i][TB * ta + a];
#pragma unroll
            for (int b = 0; b < TB; ++b)
                yb[b] = ys[i][TB * tb + b];
#pragma unroll
            for (int a = 0; a < TB; ++a)
#pragma unroll
                for (int b = 0; b < TB; ++b)
                    acc[a][b] += ya[a] * yb[b];
        }
    }
    if (g > 0)
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b)
                accs[g - 1][(TB * ta + a) * R + TB * tb + b] = acc[a][b];
    __syncthreads();
    if (g == 0) {
        double *out = part + (int64_t)blockIdx.x * R * R;
#pragma unroll
        for (int a = 0; a < TB; ++a)
#pragma unroll
            for (int b = 0; b < TB; ++b) {
                const int idx = (TB * ta + a) * R + TB * tb + b;
                double v = acc[a][b];
#pragma unroll
                for (int h = 0; h < NG - 1; ++h)
                    v += accs[h][idx];
                out[idx] = v;
            }
    }
}

// Z = Y QS (row-major, FP64 sums): 64-row tiles, QS (R x R) staged in LDS;
// each thread a 4-row by (R/16)-column block of Z.
template <int R>
__global__ __launch_bounds__(256) void k_whiten_apply(const float *__restrict__ Y, int64_t M,
                                                      const double *__restrict__ QS,
                                                      float *__restrict__ Z)
{
    constexpr int TC = R / 16;
    __shared__ double qs[R][R];
    __shared__ double ys[64][R + 1];
    const int tid = threadIdx.x, tc = tid & 15, tr = tid >> 4; // columns tc + 16 c, rows 4 tr + a
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    for (int e = tid; e < R * R; e += 256)
        qs[e / R][e % R] = QS[e];
    for (int e = tid; e < 64 * R; e += 256) {
        const int i = e / R, c = e % R;
        const int64_t m = m0 + i;
        ys[i][c] = m < M ? (double)Y[m * R + c] : 0.0;
    }
    __syncthreads();
    double z[4][TC];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int c = 0; c < TC; ++c)
            z[a][c] = 0.0;
    for (int r = 0; r < R; ++r) {
        double ya[4], qb[TC];
#pragma unroll
        for (int a = 0; a < 4; ++a)
            ya[a] = ys[4 * tr + a][r];
#pragma unroll
        for (int c = 0; c < TC; ++c)
            qb[c] = qs[r][tc + 16 * c];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int c = 0; c < TC; ++c)
                z[a][c] += ya[a] * qb[c];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const int64_t m = m0 + 4 * tr + a;
        if (m < M)
#pragma unroll
            for (int c = 0; c < TC; ++c)
                Z[m * R + tc + 16 * c] = (float)z[a][c];
    }
}

// G = the nslice partials from k_gram summed (FP64, fixed order), written
// over the first partial.  A workgroup of 256 threads owns 64 entries; wave w
// sums slices w, w + 4, w + 8, ... in increasing order and the four wave sums
// are added in wave order.  Each entry's slices are read before the barrier
// that precedes its write.
__global__ __launch_bounds__(256) void k_gram_sum(double *__restrict__ part, int nslice, int n)
{
    __shared__ double red[3][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int idx = blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (idx < n) {
#pragma unroll 8
        for (int y = w; y < nslice; y += 4)
            acc += part[(int64_t)y * n + idx];
    }
    if (w > 0)
        red[w - 1][lane] = acc;
    __syncthreads();
    if (w == 0 && idx < n)
        part[idx] = ((acc + red[0][lane]) + red[1][lane]) + red[2][lane];
}

// 1/sqrt(x) for x in [1, 2]: the hardware estimate refined by two Newton
// steps y <- y + y (1/2 - (x/2) y^2).
__device__ inline double newton_rsq(double x)
{
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = fma(y, fma(-h * y, y, 0.5), y);
    y = fma(y, fma(-h * y, y, 0.5), y);
    return y;
}

// 1/x for x in [1, 3]: the hardware estimate refined by two Newton steps
// y <- y + y (1 - x y).
__device__ inline double newton_rcp(double x)
{
    double y = __builtin_amdgcn_rcp(x);
    y = fma(y, fma(-x, y, 1.0), y);
    y = fma(y, fma(-x, y, 1.0), y);
    return y;
}

// Rotation (c, s) that zeroes the (p, q) entry of a symmetric 2 x 2 block
// (Golub & Van Loan's symmetric Schur step): with d = a_qq - a_pp and
// b = 2 a_pq, t = sign(d) b / (|d| + sqrt(d^2 + b^2)) is the smaller root of
// t^2 + 2 (d / b) t - 1 = 0, c = 1 / sqrt(1 + t^2), s = t c.  d and b are
// first scaled by about 1 / max(|d|, |b|) (t does not depend on the scale),
// so every square root and reciprocal below has its argument in [1, 3].
// The identity when a_pq = 0 or the block is below the normal range.
__device__ inline void jacobi_rotation(double app, double aqq, double apq, double &c, double &s)
{
    const double d = aqq - app, b = 2.0 * apq;
    const double m = fmax(fabs(d), fabs(b));
    const double im = __builtin_amdgcn_rcp(m);
    const double ds = d * im, bs = b * im;
    const double x = fma(ds, ds, bs * bs);
    const double r = x * newton_rsq(x);
    const double t = (ds >= 0.0 ? bs : -bs) * newton_rcp(fabs(ds) + r);
    const double cc = newton_rsq(fma(t, t, 1.0));
    const bool rot = apq != 0.0 && m >= 4.0 * DBL_MIN;
    c = rot ? cc : 1.0;
    s = rot ? t * cc : 0.0;
}

// Eigen-decomposition of the sketch's Gram matrix G (R x R, FP64, summed by
// k_gram_sum) by one workgroup of 256 threads (R = 32 or 64): parallel cyclic
// Jacobi, R/2 disjoint rotations per round applied to both sides of G in one
// step, R-1 rounds per sweep in round-robin order (index 0 fixed, the others
// advancing one place per round), until the off-diagonal mass is below 1e-28
// of |G|_F^2; eigenpairs by decreasing g, each eigenvector's largest entry
// made positive.  Writes QS = sqrt(M) Q[:, perm] diag(g)^(-1/2) (R x R,
// row-major; zero columns where g is not positive and finite), g, and the
// flag.
// G and the columns of Q are kept in round-robin position order: rotation i
// of every round acts on positions i and R-1-i, and the results are written,
// double-buffered, to the places the next round's pairing gives them
// (position u -> u - 1, position 1 -> R - 1, 0 fixed), so every LDS address
// is the same in every round; after the R-1 rounds of a sweep the positions
// are the indices again.  Every lane forms the rotation of pair
// (lane mod R/2) itself, so a round has a single barrier.
template <int R, int NT>
__global__ __launch_bounds__(NT) void k_whiten_eig(const double *__restrict__ gsum, int64_t M,
                                                     double *__restrict__ QS,
                                                     double *__restrict__ gout,
                                                     int32_t *__restrict__ flag)
{
    constexpr int NP = R / 2, EPT = R * R / NT; // Gram entries per thread
    constexpr int GB = NP * NP / NT, QB = R * NP / NT; // 2 x 2 blocks of G, Q row pairs per thread
    __shared__ double Gb[2][R][R + 1];
    __shared__ double Qb[2][R][R + 1];
    __shared__ double eig[R];
    __shared__ int perm[R];
    __shared__ double scale[R];
    __shared__ double red[2][NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, my = lane % NP;
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
        const int idx = tid + e * NT, a = idx / R, b = idx % R;
        Gb[0][a][b] = gsum[idx];
        Qb[0][a][b] = a == b ? 1.0 : 0.0;
    }
    // this lane's pair (positions p, q), the next round's places of positions
    auto next = [](int u) { return u == 0 ? 0 : (u == 1 ? R - 1 : u - 1); };
    const int p = my, q = R - 1 - my, np_ = next(p), nq = next(q);
    int b1[GB];
#pragma unroll
    for (int k = 0; k < GB; ++k)
        b1[k] = (tid + k * NT) / NP; // row pair of block k (column pair: my)
    // one round: reads from (Gc, Qc), writes to (Gn, Qn), then the barrier
    auto round_step = [&](const double(*Gc)[R + 1], double(*Gn)[R + 1],
                          const double(*Qc)[R + 1], double(*Qn)[R + 1])
        __attribute__((always_inline)) {
        const double app = Gc[p][p], aqq = Gc[q][q], apq = Gc[p][q];
        double g[GB][4], qv[QB][2];
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            const int p1 = b1[k], q1 = R - 1 - b1[k];
            g[k][0] = Gc[p1][p];
            g[k][1] = Gc[p1][q];
            g[k][2] = Gc[q1][p];
            g[k][3] = Gc[q1][q];
        }
#pragma unroll
        for (int k = 0; k < QB; ++k) {
            const int a = (tid + k * NT) / NP;
            qv[k][0] = Qc[a][p];
            qv[k][1] = Qc[a][q];
        }
        double c, sv;
        jacobi_rotation(app, aqq, apq, c, sv);
#pragma unroll
        for (int k = 0; k < GB; ++k) {
            // G <- J^T G J on the 2 x 2 block of row pair b1 and column pair
            // my: the pairs are disjoint, so it depends on rotations b1 and
            // my only (columns first, then rows)
            const double c1 = __shfl(c, b1[k], 64), s1 = __shfl(sv, b1[k], 64);
            const int p1 = next(b1[k]), q1 = next(R - 1 - b1[k]);
            const double h00 = c * g[k][0] - sv * g[k][1], h01 = sv * g[k][0] + c * g[k][1];
            const double h10 = c * g[k][2] - sv * g[k][3], h11 = sv * g[k][2] + c * g[k][3];
            Gn[p1][np_] = c1 * h00 - s1 * h10;
            Gn[q1][np_] = s1 * h00 + c1 * h10;
            Gn[p1][nq] = c1 * h01 - s1 * h11;
            Gn[q1][nq] = s1 * h01 + c1 * h11;
        }
#pragma unroll
        for (int k = 0; k < QB; ++k) { // Q <- Q J (row a, pair my)
            const int a = (tid + k * NT) / NP;
            Qn[a][np_] = c * qv[k][0] - sv * qv[k][1];
            Qn[a][nq] = sv * qv[k][0] + c * qv[k][1];
        }
        __syncthreads();
    };
    __syncthreads();
    int cur = 0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        {   // off-diagonal and total mass: per-thread entries, wave sums, the
            // waves in order (the same on every run and in every thread)
            double off = 0.0, fro = 0.0;
#pragma unroll
            for (int e = 0; e < EPT; ++e) {
                const int idx = tid + e * NT, a = idx / R, b = idx % R;
                const double v = Gb[cur][a][b];
                fro += v * v;
                off += a != b ? v * v : 0.0;
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) {
                off += __shfl_xor(off, o, 64);
                fro += __shfl_xor(fro, o, 64);
            }
            if (lane == 0) {
                red[0][w] = off;
                red[1][w] = fro;
            }
            __syncthreads();
            double so = 0.0, sf = 0.0;
            for (int i = 0; i < NT / 64; ++i) {
                so += red[0][i];
                sf += red[1][i];
            }
            if (!(so > 1e-28 * sf))
                break;
        }
        // R - 1 rounds alternating between the two buffers; each round is
        // written out for both directions so that every LDS address is a
        // fixed offset from a loop-invariant base.
        if (cur == 0) {
            for (int round = 0; round < R - 2; round += 2) {
                round_step(Gb[0], Gb[1], Qb[0], Qb[1]);
                round_step(Gb[1], Gb[0], Qb[1], Qb[0]);
            }
            round_step(Gb[0], Gb[1], Qb[0], Qb[1]);
        } else {
            for (int round = 0; round < R - 2; round += 2) {
                round_step(Gb[1], Gb[0], Qb[1], Qb[0]);
                round_step(Gb[0], Gb[1], Qb[0], Qb[1]);
            }
            round_step(Gb[1], Gb[0], Qb[1], Qb[0]);
        }
        cur ^= 1;
    }
    const double(*G)[R + 1] = Gb[cur];
    const double(*Q)[R + 1] = Qb[cur];
    // eigenvalues by decreasing g (rank of each, ties by index), then per
    // column the sign that makes its largest entry positive (first maximum in
    // row order) and the whitening scale
    __shared__ int badf;
    if (tid < R)
        eig[tid] = G[tid][tid];
    if (tid == 0)
        badf = 0;
    __syncthreads();
    if (tid < R) {
        const double gi = eig[tid];
        int rank = 0;
        for (int j = 0; j < R; ++j)
            rank += (eig[j] > gi || (eig[j] == gi && j < tid)) ? 1 : 0;
        perm[rank] = tid;
    }
    __syncthreads();
    if (tid < R) {
        const int i = tid, c = perm[i];
        double amax = -1.0, sgn = 1.0;
        for (int r = 0; r < R; ++r)
            if (fabs(Q[r][c]) > amax) {
                amax = fabs(Q[r][c]);
                sgn = Q[r][c] >= 0.0 ? 1.0 : -1.0;
            }
        const double g = eig[c];
        const bool ok = g > 0.0 && isfinite(g);
        if (!ok)
            badf = 1;
        scale[i] = ok ? sqrt((double)M) / sqrt(g) * sgn : 0.0;
        if (gout)
            gout[i] = g;
    }
    __syncthreads();
    if (tid == 0 && flag)
        *flag = badf;
    __syncthreads();
    for (int e = tid; e < R * R; e += NT) {
        const int r = e / R, b = e % R;
        QS[e] = Q[r][perm[b]] * scale[b];
    }
}

// Columns c0 .. c0 + Kc - 1 of T0 (column-major M x K) into Z (row-major
// M x R, columns Kc .. zero).
__global__ __launch_bounds__(256) void k_t0_rows(const float *__restrict__ T0, int64_t M,
                                                 int64_t c0, int64_t Kc, int R,
                                                 float *__restrict__ Z)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= M * R)
        return;
    const int64_t m = e / R, c = e % R;
    Z[e] = c < Kc ? T0[m + (c0 + c) * M] : 0.0f;
}

// The first Kc columns of W (row-major N x R) into columns c0 .. c0 + Kc - 1
// of Q0 (column-major N x K).
__global__ __launch_bounds__(256) void k_q0_cols(const float *__restrict__ W, int64_t N,
                                                 int64_t c0, int64_t Kc, int R,
                                                 float *__restrict__ Q0)
{
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= N * Kc)
        return;
    const int64_t j = e % N, c = e / N;
    Q0[(c0 + c) * N + j] = W[j * R + c];
}

// ---------------------------------------------------------------------------
// Host side.

namespace {

inline unsigned ucdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Offs {
    int64_t W1, b1, W2, b2, W3, b3, n;
};
Offs param_offsets(int d0, int d1, int d2, int d3)
{
    Offs o;
    o.W1 = 0;
    o.b1 = o.W1 + (int64_t)d0 * d1;
    o.W2 = o.b1 + d1;
    o.b2 = o.W2 + (int64_t)d1 * d2;
    o.W3 = o.b2 + d2;
    o.b3 = o.W3 + (int64_t)d2 * d3;
    o.n = o.b3 + d3;
    return o;
}

bool valid_net(const gspca_mlp *n)
{
    return n && n->d0 == GSPCA_WS_RANK && n->d1 >= 16 && n->d1 <= 1024 && n->d2 >= 16 &&
           n->d2 <= 1024 && n->d3 >= 1 && n->d3 <= n->d0 && n->theta && n->theta_bf16;
}

// Split-K partial buffer: enough for any weight gradient with <= kMaxSplit
// splits.
constexpr int kMaxSplit = 64;

struct Layout {
    size_t H1, H2, O, dO, G2, G1, lossp, part, Y, Z, W, SK, total;
};
Layout layout(const gspca_mlp *n, int64_t rows, int32_t ninst, int64_t cols)
{
    Layout L{};
    size_t o = 0;
    auto put = [&](size_t &slot, size_t bytes) {
        slot = o;
        o = align256(o + bytes);
    };
    const int64_t dmax = std::max<int64_t>(std::max<int64_t>(n->d0, n->d1),
                                           std::max<int64_t>(n->d2, n->d3));
    put(L.H1, (size_t)rows * n->d1 * 2);
    put(L.H2, (size_t)rows * n->d2 * 2);
    put(L.O, (size_t)rows * n->d3 * 4);
    put(L.dO, (size_t)rows * n->d3 * 2);
    put(L.G2, (size_t)rows * n->d2 * 2);
    put(L.G1, (size_t)rows * n->d1 * 2);
    put(L.lossp, (size_t)std::max<int32_t>(ninst, 1) * n->d3 * 8);
    put(L.part, (size_t)kMaxSplit * dmax * dmax * 4);
    put(L.Y, (size_t)rows * GSPCA_WS_RMAX * 4);
    put(L.Z, (size_t)rows * GSPCA_WS_RMAX * 4);
    put(L.W, (size_t)std::max<int64_t>(cols, 1) * GSPCA_WS_RMAX * 4);
    put(L.SK, cols > 0 ? sketch_plan(rows, cols, GSPCA_WS_RMAX).total : 0);
    L.total = o;
    return L;
}

template <typename TA, typename TB>
void gemm_launch(const TA *A, int64_t a_r, int64_t a_c, const TB *B, int64_t b_r, int64_t b_c,
                 int64_t M, int64_t N, int64_t Kd, const float *bias, int relu, const __bf16 *mask,
                 int64_t m_r, float *Cf, __bf16 *Cb, int64_t c_r, int64_t c_c, float *part,
                 hipStream_t s, const float *skip = nullptr, int64_t s_r = 0)
{
    // Split the k range when the output tiles alone cannot fill the chip
    // (weight gradients: small outputs, k = all rows).
    const int64_t tiles = (int64_t)ucdiv(M, kGemmTile) * ucdiv(N, kGemmTile);
    int nz = 1;
    if (part && tiles < 1024 && Kd >= 4096) {
        nz = (int)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, 2048 / tiles));
        nz = (int)std::min<int64_t>(nz, Kd / 1024);
    }
    const int64_t kchunk = ((Kd + nz - 1) / nz + 31) / 32 * 32;
    nz = (int)((Kd + kchunk - 1) / kchunk);
    dim3 g(ucdiv(N, kGemmTile), ucdiv(M, kGemmTile), nz);
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB>), g, dim3(256), 0, s, A, a_r, a_c, B, b_r, b_c, M, N,
                       Kd, kchunk, bias, relu, mask, m_r, skip, s_r, Cf, Cb, c_r, c_c, 0,
                       nz > 1 ? 1 : 0, part);
    if (nz > 1)
        hipLaunchKernelGGL(k_split_reduce, dim3(ucdiv(M * N, 256)), dim3(256), 0, s, part, nz, M,
                           N, Cf, c_r, c_c);
}

template <typename T>
void colsum(const T *G, int64_t rows, int64_t N, float *out, float *part, hipStream_t s)
{
    const int nz = (int)std::min<int64_t>(kMaxSplit, std::max<int64_t>(1, rows / 2048));
    const int64_t rchunk = (rows + nz - 1) / nz;
    hipLaunchKernelGGL(k_colsum_part<T>, dim3(ucdiv(N, 64), 1, nz), dim3(256), 0, s, G, rows, N,
                       rchunk, part);
    hipLaunchKernelGGL(k_split_reduce, dim3(ucdiv(N, 256)), dim3(256), 0, s, part, nz, (int64_t)1,
                       N, out, (int64_t)0, (int64_t)1);
}

// Forward over `rows` rows: H1, H2 (bf16, row-major) and the output with
// strides (o_r, o_c).
void forward(const gspca_mlp *n, const float *Z, int64_t zs, int64_t rows, __bf16 *H1,
             __bf16 *H2, float *O, int64_t o_r, int64_t o_c, hipStream_t s)
{
    const Offs of = param_offsets(n->d0, n->d1, n->d2, n->d3);
    const __bf16 *wb = reinterpret_cast<const __bf16 *>(n->theta_bf16);
    const float *th = n->theta;
    // input row m = the first d0 entries of Z's row m (row stride zs >= d0)
    gemm_launch<float, __bf16>(Z, zs, 1, wb + of.W1, n->d1, 1, rows, n->d1, n->d0, th + of.b1,
                               1, nullptr, 0, nullptr, H1, n->d1, 1, nullptr, s);
    gemm_launch<__bf16, __bf16>(H1, n->d1, 1, wb + of.W2, n->d2, 1, rows, n->d2, n->d1,
                                th + of.b2, 1, nullptr, 0, nullptr, H2, n->d2, 1, nullptr, s);
    // output = z[:d3] + W3^T h2 + b3: the whitened directions plus a learned correction
    gemm_launch<__bf16, __bf16>(H2, n->d2, 1, wb + of.W3, n->d3, 1, rows, n->d3, n->d2,
                                th + of.b3, 0, nullptr, 0, O, nullptr, o_r, o_c, nullptr, s, Z,
                                zs);
}

gspca_status launched()
{
    return hipGetLastError() == hipSuccess ? GSPCA_OK : GSPCA_EDEVICE;
}

} // namespace

// Sketch products and whitening, shared with the block iteration (block.hip).
// Row slices of the refinement's X^T Z (about 2048 workgroups) and of the Gram
// matrix (at most 256 workgroups), and the workspace they use.
SketchPlan sketch_plan(int64_t M, int64_t N, int r)
{
    SketchPlan P{};
    const int64_t cb = (N + 63) / 64;
    P.st = std::max<int64_t>(1, std::min<int64_t>((M + 255) / 256, 2048 / cb));
    P.rows_t = ((M + P.st - 1) / P.st + 31) / 32 * 32;
    P.st = (M + P.rows_t - 1) / P.rows_t;
    P.sg = std::max<int64_t>(1, std::min<int64_t>((M + 255) / 256, 256));
    P.rows_g = ((M + P.sg - 1) / P.sg + 63) / 64 * 64;
    P.sg = (M + P.rows_g - 1) / P.rows_g;
    size_t o = 0; // Gram part first: its offsets do not depend on N
    P.off_gpart = o;
    o = align256(o + (size_t)P.sg * r * r * 8);
    P.off_qs = o;
    o = align256(o + (size_t)r * r * 8);
    P.off_wpart = o;
    o = align256(o + (size_t)P.st * N * r * 4);
    P.total = o;
    return P;
}

bool valid_rank(int32_t r) { return r == 32 || r == GSPCA_WS_RMAX; }

// Chunk depths of the matrix-core sketch products (columns of X per chunk
// for Y = X Om, rows for W = X^T Z).
constexpr int kSketchBK = 32, kSketchTBK = 16;

void launch_sketch(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Om, int r,
                   float *Y, hipStream_t s)
{
    const bool aligned = ldx % 4 == 0 && ((uintptr_t)X) % 16 == 0 && ((uintptr_t)Om) % 16 == 0 &&
                         ((uintptr_t)Y) % 16 == 0;
    if (aligned) {
        if (r == 32)
            hipLaunchKernelGGL((k_sketch_m<32, kSketchBK>), dim3(ucdiv(M, 64)), dim3(256), 0, s, X,
                               ldx, M, N, Om, Y);
        else
            hipLaunchKernelGGL((k_sketch_m<64, kSketchBK>), dim3(ucdiv(M, 64)), dim3(256), 0, s, X,
                               ldx, M, N, Om, Y);
        return;
    }
    if (r == 32)
        hipLaunchKernelGGL(k_sketch<32>, dim3(ucdiv(M, 64)), dim3(256), 0, s, X, ldx, M, N, Om, Y);
    else
        hipLaunchKernelGGL(k_sketch<64>, dim3(ucdiv(M, 64)), dim3(256), 0, s, X, ldx, M, N, Om, Y);
}

void launch_sketch_t(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Z, int r,
                     float *W, unsigned char *ws, hipStream_t s, bool unit_scale)
{
    const SketchPlan P = sketch_plan(M, N, r);
    const float sc = unit_scale ? 1.0f : (float)(1.0 / sqrt((double)M));
    float *dst = P.st == 1 ? W : reinterpret_cast<float *>(ws + P.off_wpart);
    const bool aligned = ldx % 4 == 0 && ((uintptr_t)X) % 16 == 0 && ((uintptr_t)Z) % 16 == 0 &&
                         ((uintptr_t)dst) % 16 == 0 && P.rows_t % kSketchTBK == 0;
    if (aligned) {
        const dim3 g(ucdiv(N, 128), (unsigned)P.st);
        if (r == 32)
            hipLaunchKernelGGL((k_sketch_t_m<32, kSketchTBK>), g, dim3(256), 0, s, X, ldx, M, N, Z,
                               sc, P.rows_t, dst);
        else
            hipLaunchKernelGGL((k_sketch_t_m<64, kSketchTBK>), g, dim3(256), 0, s, X, ldx, M, N, Z,
                               sc, P.rows_t, dst);
    } else {
        const dim3 g(ucdiv(N, 64), (unsigned)P.st);
        if (r == 32)
            hipLaunchKernelGGL(k_sketch_t<32>, g, dim3(256), 0, s, X, ldx, M, N, Z, sc, P.rows_t,
                               dst);
        else
            hipLaunchKernelGGL(k_sketch_t<64>, g, dim3(256), 0, s, X, ldx, M, N, Z, sc, P.rows_t,
                               dst);
    }
    if (P.st > 1) // slice partials added in slice order
        hipLaunchKernelGGL(k_split_reduce, dim3(ucdiv(N * r, 256)), dim3(256), 0, s, dst,
                           (int)P.st, N, (int64_t)r, W, (int64_t)r, (int64_t)1);
}

namespace {
inline int first_loadings_width(int64_t K) { return K <= 32 ? 32 : 64; }
} // namespace

size_t first_loadings_bytes(int64_t M, int64_t N, int64_t K)
{
    const int r = first_loadings_width(K);
    return align256((size_t)M * r * 4) + align256((size_t)N * r * 4) +
           sketch_plan(M, N, r).total;
}

void launch_first_loadings(const float *X, int64_t ldx, int64_t M, int64_t N, const float *T0,
                           int64_t K, float *Q0, unsigned char *ws, hipStream_t s)
{
    const int r = first_loadings_width(K);
    float *Z = reinterpret_cast<float *>(ws);
    float *W = reinterpret_cast<float *>(ws + align256((size_t)M * r * 4));
    unsigned char *sk = ws + align256((size_t)M * r * 4) + align256((size_t)N * r * 4);
    for (int64_t c0 = 0; c0 < K; c0 += r) { // blocks of r columns, one read of X each
        const int64_t Kc = std::min<int64_t>(r, K - c0);
        hipLaunchKernelGGL(k_t0_rows, dim3(ucdiv(M * r, 256)), dim3(256), 0, s, T0, M, c0, Kc,
                           r, Z);
        launch_sketch_t(X, ldx, M, N, Z, r, W, sk, s, true);
        hipLaunchKernelGGL(k_q0_cols, dim3(ucdiv(N * Kc, 256)), dim3(256), 0, s, W, N, c0, Kc,
                           r, Q0);
    }
}

constexpr int kEig64Threads = 256;

void launch_whiten(const float *Y, int64_t M, int r, float *Z, double *g, int32_t *flag,
                   unsigned char *ws, hipStream_t s)
{
    const SketchPlan P = sketch_plan(M, 1, r);
    double *gp = reinterpret_cast<double *>(ws + P.off_gpart);
    double *qs = reinterpret_cast<double *>(ws + P.off_qs);
    if (r == 32) {
        hipLaunchKernelGGL(k_gram<32>, dim3((unsigned)P.sg), dim3(1024), 0, s, Y, M, P.rows_g,
                           gp);
        hipLaunchKernelGGL(k_gram_sum, dim3(ucdiv(32 * 32, 64)), dim3(256), 0, s, gp, (int)P.sg,
                           32 * 32);
        hipLaunchKernelGGL((k_whiten_eig<32, 256>), dim3(1), dim3(256), 0, s, gp, M, qs, g,
                           flag);
        hipLaunchKernelGGL(k_whiten_apply<32>, dim3(ucdiv(M, 64)), dim3(256), 0, s, Y, M, qs, Z);
    } else {
        hipLaunchKernelGGL(k_gram<64>, dim3((unsigned)P.sg), dim3(1024), 0, s, Y, M, P.rows_g,
                           gp);
        hipLaunchKernelGGL(k_gram_sum, dim3(ucdiv(64 * 64, 64)), dim3(256), 0, s, gp, (int)P.sg,
                           64 * 64);
        hipLaunchKernelGGL((k_whiten_eig<64, kEig64Threads>), dim3(1), dim3(kEig64Threads), 0, s,
                           gp, M, qs, g, flag);
        hipLaunchKernelGGL(k_whiten_apply<64>, dim3(ucdiv(M, 64)), dim3(256), 0, s, Y, M, qs, Z);
    }
}

} // namespace gspca

using namespace gspca;

extern "C" {

int64_t gspca_mlp_param_count(int32_t d0, int32_t d1, int32_t d2, int32_t d3)
{
    if (d0 < 1 || d1 < 1 || d2 < 1 || d3 < 1)
        return 0;
    return param_offsets(d0, d1, d2, d3).n;
}

size_t gspca_mlp_workspace_bytes(const gspca_mlp *net, int64_t rows, int32_t ninst,
                                 int64_t cols)
{
    if (!net || rows < 1 || ninst < 1 || cols < 0)
        return 0;
    // the widths the kernels accept (valid_net without the parameter pointers)
    if (net->d0 != GSPCA_WS_RANK || net->d1 < 16 || net->d1 > 1024 || net->d2 < 16 ||
        net->d2 > 1024 || net->d3 < 1 || net->d3 > net->d0)
        return 0;
    return layout(net, rows, ninst, cols).total;
}

gspca_status gspca_sketch(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Omega,
                          int32_t r, float *Y, void *stream)
{
    if (!X || !Omega || !Y || !valid_rank(r) || M < 1 || N < 1 || ldx < M)
        return GSPCA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_sketch(X, ldx, M, N, Omega, r, Y, s);
    return launched();
}

size_t gspca_sketch_workspace_bytes(int64_t M, int64_t N, int32_t r)
{
    if (M < 1 || N < 1 || !valid_rank(r))
        return 0;
    return sketch_plan(M, N, r).total;
}

gspca_status gspca_sketch_refine(const float *X, int64_t ldx, int64_t M, int64_t N,
                                 const float *Z, int32_t r, float *W, float *Y, void *ws,
                                 size_t ws_bytes, void *stream)
{
    if (!X || !Z || !W || !Y || !valid_rank(r) || M < 1 || N < 1 || ldx < M || !ws)
        return GSPCA_EINVAL;
    if (ws_bytes < sketch_plan(M, N, r).total)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_sketch_t(X, ldx, M, N, Z, r, W, static_cast<unsigned char *>(ws), s);
    launch_sketch(X, ldx, M, N, W, r, Y, s);
    return launched();
}

gspca_status gspca_whiten_sketch(const float *Y, int64_t M, int32_t r, float *Z, double *gamma,
                                 int32_t *flag, void *ws, size_t ws_bytes, void *stream)
{
    if (!Y || !Z || !valid_rank(r) || M < r || !ws)
        return GSPCA_EINVAL;
    if (ws_bytes < sketch_plan(M, 1, r).off_wpart)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    launch_whiten(Y, M, r, Z, gamma, flag, static_cast<unsigned char *>(ws), s);
    return launched();
}

gspca_status gspca_mlp_sync(const gspca_mlp *net, void *stream)
{
    if (!valid_net(net))
        return GSPCA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = param_offsets(net->d0, net->d1, net->d2, net->d3).n;
    hipLaunchKernelGGL(k_to_bf16, dim3(ucdiv(n, 256)), dim3(256), 0, s, net->theta,
                       reinterpret_cast<__bf16 *>(net->theta_bf16), n);
    return launched();
}

gspca_status gspca_mlp_forward(const gspca_mlp *net, const float *Z, int64_t rows, float *O,
                               void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_net(net) || !Z || !O || rows < 1 || !ws)
        return GSPCA_EINVAL;
    const Layout L = layout(net, rows, 1, 0);
    if (ws_bytes < L.total)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *b = static_cast<unsigned char *>(ws);
    forward(net, Z, net->d0, rows, reinterpret_cast<__bf16 *>(b + L.H1),
            reinterpret_cast<__bf16 *>(b + L.H2), O, 1, rows, s);
    return launched();
}

gspca_status gspca_mlp_loss_grad(const gspca_mlp *net, const float *Z, const float *V,
                                 int32_t ninst, int64_t rows_per_inst, double *loss, void *ws,
                                 size_t ws_bytes, void *stream)
{
    if (!valid_net(net) || !net->grad || !Z || !V || ninst < 1 || rows_per_inst < 1 || !ws)
        return GSPCA_EINVAL;
    const int64_t rows = (int64_t)ninst * rows_per_inst;
    const Layout L = layout(net, rows, ninst, 0);
    if (ws_bytes < L.total)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *b = static_cast<unsigned char *>(ws);
    __bf16 *H1 = reinterpret_cast<__bf16 *>(b + L.H1);
    __bf16 *H2 = reinterpret_cast<__bf16 *>(b + L.H2);
    float *O = reinterpret_cast<float *>(b + L.O);
    __bf16 *dO = reinterpret_cast<__bf16 *>(b + L.dO);
    __bf16 *G2 = reinterpret_cast<__bf16 *>(b + L.G2);
    __bf16 *G1 = reinterpret_cast<__bf16 *>(b + L.G1);
    double *lossp = reinterpret_cast<double *>(b + L.lossp);
    float *part = reinterpret_cast<float *>(b + L.part);
    const int d0 = net->d0, d1 = net->d1, d2 = net->d2, d3 = net->d3;
    const Offs of = param_offsets(d0, d1, d2, d3);
    const __bf16 *wb = reinterpret_cast<const __bf16 *>(net->theta_bf16);
    float *g = net->grad;

    forward(net, Z, d0, rows, H1, H2, O, d3, 1, s);
    const double inv = 1.0 / (double)ninst;
    hipLaunchKernelGGL(k_cos2, dim3(d3, ninst), dim3(256), 0, s, O, V, rows_per_inst, d3, inv, dO,
                       lossp);
    if (loss)
        hipLaunchKernelGGL(k_loss_mean, dim3(1), dim3(1), 0, s, lossp, (int64_t)ninst * d3, inv,
                           loss);
    // layer 3: dW3 = H2^T dO, db3 = colsum(dO), G2 = (dO W3^T) * [H2 > 0]
    gemm_launch<__bf16, __bf16>(H2, 1, d2, dO, d3, 1, d2, d3, rows, nullptr, 0, nullptr, 0,
                                g + of.W3, nullptr, d3, 1, part, s);
    colsum<__bf16>(dO, rows, d3, g + of.b3, part, s);
    gemm_launch<__bf16, __bf16>(dO, d3, 1, wb + of.W3, 1, d3, rows, d2, d3, nullptr, 0, H2, d2,
                                nullptr, G2, d2, 1, nullptr, s);
    // layer 2: dW2 = H1^T G2, db2 = colsum(G2), G1 = (G2 W2^T) * [H1 > 0]
    gemm_launch<__bf16, __bf16>(H1, 1, d1, G2, d2, 1, d1, d2, rows, nullptr, 0, nullptr, 0,
                                g + of.W2, nullptr, d2, 1, part, s);
    colsum<__bf16>(G2, rows, d2, g + of.b2, part, s);
    gemm_launch<__bf16, __bf16>(G2, d2, 1, wb + of.W2, 1, d2, rows, d1, d2, nullptr, 0, H1, d1,
                                nullptr, G1, d1, 1, nullptr, s);
    // layer 1: dW1 = Z^T G1 (Z rounded to bf16 as loaded), db1 = colsum(G1)
    gemm_launch<float, __bf16>(Z, 1, d0, G1, d1, 1, d0, d1, rows, nullptr, 0, nullptr, 0,
                               g + of.W1, nullptr, d1, 1, part, s);
    colsum<__bf16>(G1, rows, d1, g + of.b1, part, s);
    return launched();
}

gspca_status gspca_mlp_adam(gspca_mlp *net, float lr, float beta1, float beta2, float eps,
                            void *stream)
{
    if (!valid_net(net) || !net->grad || !net->adam_m || !net->adam_v || !(lr > 0.0f) ||
        !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
        return GSPCA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int64_t n = param_offsets(net->d0, net->d1, net->d2, net->d3).n;
    net->step += 1;
    const float c1 = (float)(1.0 - pow((double)beta1, net->step));
    const float c2 = (float)(1.0 - pow((double)beta2, net->step));
    hipLaunchKernelGGL(k_adam, dim3(ucdiv(n, 256)), dim3(256), 0, s, net->theta, net->grad,
                       net->adam_m, net->adam_v, reinterpret_cast<__bf16 *>(net->theta_bf16), n,
                       lr, beta1, beta2, eps, c1, c2);
    return launched();
}

gspca_status gspca_ws_predict(const gspca_mlp *net, const float *X, int64_t ldx, int64_t M,
                              int64_t N, const float *Omega, int32_t r, int32_t power, float *T0,
                              void *ws, size_t ws_bytes, void *stream)
{
    if (!valid_net(net) || !X || !Omega || !T0 || !valid_rank(r) || M < r || N < 1 || ldx < M ||
        !ws || power < 0 || power > 4)
        return GSPCA_EINVAL;
    const Layout L = layout(net, M, 1, N);
    if (ws_bytes < L.total)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    unsigned char *b = static_cast<unsigned char *>(ws);
    float *Y = reinterpret_cast<float *>(b + L.Y);
    float *Z = reinterpret_cast<float *>(b + L.Z);
    float *W = reinterpret_cast<float *>(b + L.W);
    unsigned char *sk = b + L.SK;
    launch_sketch(X, ldx, M, N, Omega, r, Y, s);
    launch_whiten(Y, M, r, Z, nullptr, nullptr, sk, s);
    for (int it = 0; it < power; ++it) {
        launch_sketch_t(X, ldx, M, N, Z, r, W, sk, s);
        launch_sketch(X, ldx, M, N, W, r, Y, s);
        launch_whiten(Y, M, r, Z, nullptr, nullptr, sk, s);
    }
    forward(net, Z, r, M, reinterpret_cast<__bf16 *>(b + L.H1),
            reinterpret_cast<__bf16 *>(b + L.H2), T0, 1, M, s);
    return launched();
}

} // extern "C"
