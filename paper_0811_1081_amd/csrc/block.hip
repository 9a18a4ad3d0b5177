// block.hip -- block (subspace) iteration with Rayleigh-Ritz for the K
// leading singular triplets (gspca_block.h; not in the paper, whose GS-PCA,
// Sec. 2.3, iterates one component at a time).  The products and the
// whitening are the sketch kernels of mlp.hip; this file holds the driver and
// the output kernels.
#include <math.h>

#include <utility>
#include <vector>

#include "../../include/gspca_block.h"
#include "internal.h"

namespace gspca {
namespace {

inline unsigned bcdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
inline size_t balign(size_t x) { return (x + 255) & ~(size_t)255; }

// Row slices of the vector-change sums (k_block_change_part).
constexpr int kChangeSlices = 256;

struct BlockLayout {
    size_t Y, Z, Z2, W, g, flag, norms, cpart, sk, total;
};
BlockLayout block_layout(int64_t M, int64_t N, int r)
{
    BlockLayout L{};
    size_t o = 0;
    auto put = [&](size_t &slot, size_t bytes) {
        slot = o;
        o = balign(o + bytes);
    };
    put(L.Y, (size_t)M * r * 4);
    put(L.Z, (size_t)M * r * 4);
    put(L.Z2, (size_t)M * r * 4);
    put(L.W, (size_t)N * r * 4);
    put(L.g, (size_t)2 * r * 8);
    put(L.flag, 8);
    put(L.norms, (size_t)r * 8);
    put(L.cpart, (size_t)kChangeSlices * r * 8);
    put(L.sk, sketch_plan(M, N, r).total);
    L.total = o;
    return L;
}

// sigma_i = |W[:, i]| (W row-major N x r, i = blockIdx.x) in FP64: strided
// per-thread sums, wave butterflies, then the four waves in order.
__global__ __launch_bounds__(256) void k_block_norms(const float *__restrict__ W, int64_t N,
                                                     int r, double *__restrict__ sig)
{
    __shared__ double red[4];
    const int i = blockIdx.x, tid = threadIdx.x;
    double a = 0.0;
    for (int64_t j = tid; j < N; j += 256) {
        const double w = W[j * r + i];
        a += w * w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        a += __shfl_xor(a, o, 64);
    if ((tid & 63) == 0)
        red[tid >> 6] = a;
    __syncthreads();
    if (tid == 0)
        sig[i] = sqrt(((red[0] + red[1]) + red[2]) + red[3]);
}

// Change of the unit Ritz vectors between two whitened blocks (row-major
// M x r, columns of norm sqrt(M)): d_i = |v - s u| = sqrt(2 - 2 |u . v|), s
// the sign of u . v.  The dot products are FP64 sums in a fixed order: row
// slice y = blockIdx.x of `rows` rows, thread t on column t mod r and rows
// t / r, t / r + 256 / r, ... of the slice (each wave reads whole rows), the
// 256 / r row groups added in order into part[y][c]; then the slices in
// order, four interleaved runs added at the end (k_block_change_fin).
__global__ __launch_bounds__(256) void k_block_change_part(const float *__restrict__ Zn,
                                                           const float *__restrict__ Zo,
                                                           int64_t M, int r, int64_t rows,
                                                           double *__restrict__ part)
{
    __shared__ double red[256];
    const int tid = threadIdx.x, rp = 256 / r, c = tid % r, ro = tid / r;
    const int64_t rb = (int64_t)blockIdx.x * rows;
    const int64_t re = M < rb + rows ? M : rb + rows;
    double a = 0.0;
#pragma unroll 8
    for (int64_t m = rb + ro; m < re; m += rp)
        a += (double)Zn[m * r + c] * (double)Zo[m * r + c];
    red[tid] = a;
    __syncthreads();
    if (tid < r) {
        double v = red[tid];
        for (int g = 1; g < rp; ++g)
            v += red[g * r + tid];
        part[(int64_t)blockIdx.x * r + tid] = v;
    }
}

// Wave w adds slices w, w + 4, ... in order; the four wave sums in wave order.
__global__ __launch_bounds__(256) void k_block_change_fin(const double *__restrict__ part,
                                                          int nslice, int64_t M, int r, int K,
                                                          double *__restrict__ d)
{
    __shared__ double red[3][64];
    const int i = threadIdx.x & 63, w = threadIdx.x >> 6;
    double a = 0.0;
    if (i < K) {
#pragma unroll 8
        for (int y = w; y < nslice; y += 4)
            a += part[(int64_t)y * r + i];
    }
    if (w > 0)
        red[w - 1][i] = a;
    __syncthreads();
    if (w == 0 && i < K) {
        const double c = fabs(((a + red[0][i]) + red[1][i]) + red[2][i]) / (double)M;
        d[i] = sqrt(fmax(0.0, 2.0 - 2.0 * c));
    }
}

// Outputs of component i = blockIdx.y: T[:, i] = sigma_i Z[:, i] / sqrt(M)
// (the unit score times sigma), P[:, i] = W[:, i] / sigma_i, lambda_i.
__global__ __launch_bounds__(256) void k_block_out(const float *__restrict__ Z,
                                                   const float *__restrict__ W, int64_t M,
                                                   int64_t N, int r, const double *__restrict__ sig,
                                                   float *__restrict__ T, float *__restrict__ P,
                                                   double *__restrict__ lambda,
                                                   double *__restrict__ sigma)
{
    const int i = blockIdx.y;
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const double s = sig[i];
    if (j < M)
        T[j + (int64_t)i * M] = (float)(s * (double)Z[j * r + i] / sqrt((double)M));
    if (j < N)
        P[j + (int64_t)i * N] = s > 0.0 ? (float)((double)W[j * r + i] / s) : 0.0f;
    if (j == 0) {
        lambda[i] = s * s;
        if (sigma)
            sigma[i] = s;
    }
}

} // namespace
} // namespace gspca

using namespace gspca;

extern "C" {

size_t gspca_block_workspace_bytes(int64_t M, int64_t N, int32_t r)
{
    if (M < 1 || N < 1 || !valid_rank(r) || M < r)
        return 0;
    return block_layout(M, N, r).total;
}

gspca_status gspca_fit_block(const float *X, int64_t ldx, int64_t M, int64_t N, int64_t K,
                             const gspca_block_options *opt, float *T, float *P, double *lambda,
                             double *sigma, int32_t *iters, void *ws, size_t ws_bytes,
                             void *stream)
{
    if (!X || !opt || !T || !P || !lambda || !ws)
        return GSPCA_EINVAL;
    const int r = opt->r;
    if (!valid_rank(r) || M < r || N < 1 || ldx < M || K < 1 || K > r || K > N ||
        opt->max_iter < 1 || !(opt->tol >= 0.0) || !isfinite(opt->tol) ||
        (!opt->Omega && !opt->Z0) ||
        (opt->stop != GSPCA_STOP_SIGMA_REL && opt->stop != GSPCA_STOP_LOADING))
        return GSPCA_EINVAL;
    if (((uintptr_t)ws) % 256)
        return GSPCA_EINVAL;
    const BlockLayout L = block_layout(M, N, r);
    if (ws_bytes < L.total)
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cap = stream_capturing(s);
    if (cap != 0) // reads the Ritz values back every iteration
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;
    unsigned char *base = static_cast<unsigned char *>(ws);
    float *Y = reinterpret_cast<float *>(base + L.Y);
    float *Z = reinterpret_cast<float *>(base + L.Z);
    float *Zo = reinterpret_cast<float *>(base + L.Z2); // the previous block
    float *W = reinterpret_cast<float *>(base + L.W);
    double *gd = reinterpret_cast<double *>(base + L.g);
    double *dd = gd + r; // vector changes (loading stop)
    int32_t *flag = reinterpret_cast<int32_t *>(base + L.flag);
    double *norms = reinterpret_cast<double *>(base + L.norms);
    double *cpart = reinterpret_cast<double *>(base + L.cpart);
    const int64_t crows = (M + kChangeSlices - 1) / kChangeSlices;
    const int cslices = (int)((M + crows - 1) / crows);
    unsigned char *sk = base + L.sk;

    // V_0: whitened X Omega, or whitened given start vectors
    if (opt->Z0) {
        if (hipMemcpyAsync(Y, opt->Z0, (size_t)M * r * 4, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
            return GSPCA_EDEVICE;
    } else {
        launch_sketch(X, ldx, M, N, opt->Omega, r, Y, s);
    }
    launch_whiten(Y, M, r, Z, gd, flag, sk, s);

    std::vector<double> g(2 * r), prev(K, 0.0);
    const bool vstop = opt->stop == GSPCA_STOP_LOADING;
    int32_t it = 0;
    bool conv = false;
    while (it < opt->max_iter) {
        ++it;
        // Y = X (X^T V), V = Z / sqrt(M); then V <- whitened Y (Ritz order)
        launch_sketch_t(X, ldx, M, N, Z, r, W, sk, s);
        launch_sketch(X, ldx, M, N, W, r, Y, s);
        std::swap(Z, Zo);
        launch_whiten(Y, M, r, Z, gd, flag, sk, s);
        if (vstop) {
            hipLaunchKernelGGL(k_block_change_part, dim3((unsigned)cslices), dim3(256), 0, s, Z,
                               Zo, M, r, crows, cpart);
            hipLaunchKernelGGL(k_block_change_fin, dim3(1), dim3(256), 0, s, cpart, cslices, M,
                               r, (int)K, dd);
        }
        if (hipMemcpyAsync(g.data(), gd, (size_t)(vstop ? 2 * r : r) * 8, hipMemcpyDeviceToHost,
                           s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return GSPCA_EDEVICE;
        for (int64_t i = 0; i < K; ++i)
            if (!(g[i] > 0.0) || !isfinite(g[i]))
                return GSPCA_EINVAL; // X has rank below K (or non-finite entries)
        // estimates s_i = g_i^(1/4) (g: Ritz values of (X X^T)^2), relative
        // test; or the change of the unit Ritz vectors
        bool pass = true;
        for (int64_t i = 0; i < K; ++i) {
            const double si = pow(g[i], 0.25);
            if (vstop ? !(g[r + i] < opt->tol) : !(fabs(si - prev[i]) < opt->tol * si))
                pass = false;
            prev[i] = si;
        }
        if (opt->tol > 0.0 && pass) {
            conv = true;
            break;
        }
    }
    // w_i = X^T v_i, sigma_i = |w_i|, P = w / sigma, T = sigma v
    launch_sketch_t(X, ldx, M, N, Z, r, W, sk, s);
    hipLaunchKernelGGL(k_block_norms, dim3((unsigned)K), dim3(256), 0, s, W, N, r, norms);
    hipLaunchKernelGGL(k_block_out, dim3(bcdiv(M > N ? M : N, 256), (unsigned)K), dim3(256), 0, s,
                       Z, W, M, N, r, norms, T, P, lambda, sigma);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
        return GSPCA_EDEVICE;
    if (iters)
        *iters = it;
    return (conv || opt->tol == 0.0) ? GSPCA_OK : GSPCA_NOT_CONVERGED;
}

}  // extern "C"
