// fused.hip -- single-pass form of the power iteration (one read of the data
// matrix per iteration) for GS-PCA / NIPALS-PCA (Andrecut, arXiv:0811.1081,
// Secs. 2.2-2.3), for FP64, FP32 and the reduced-precision BF16 / FP8 (OCP
// E4M3) storage of X with per-column FP32 scales.
//
// The data matrix A (the residual R for explicit deflation, X itself for
// implicit deflation, or the quantised codes Q) is held in row panels
// (panel.h); the streaming kernel that reads it once per iteration is in
// pass.hip.  This file holds the rest of the iteration: the Gram-Schmidt
// pass on t (needing all of t) is applied afterwards through W = A^T V_(k):
// A^T (t - V d) = q - W d; the re-tiling, quantisation, deflation, start and
// end-of-component kernels.
//
// Quantised storage: X~_mj = decode(Q_mj) * s_j.  The scale is folded into
// the vectors: X~ p = Q (s o p) and X~^T t = s o (Q^T t); arithmetic is FP32.
#include "panel.h"

namespace gspca {

// ---------------------------------------------------------------------------
// Re-tile X (column-major, ldx) into row panels of ldp >= N columns; rows >= M
// and columns >= N are zero.  Flags NaN/Inf.  Workgroup: a tile of 64 rows x
// 64 columns, read down the columns (256 contiguous bytes per column for
// FP32), transposed through LDS, and written as the 16-byte segments of its
// 64 / PR panels (64 consecutive segments per panel row, contiguous).
constexpr int kRetileTile = 64;
template <typename E>
__global__ __launch_bounds__(256) void k_retile(const E *__restrict__ X, int64_t ldx, int64_t M,
                                                int64_t N, int64_t NP, int64_t ldp,
                                                E *__restrict__ A, LoopState *st)
{
    constexpr int PR = 16 / sizeof(E);
    constexpr int T = kRetileTile;
    __shared__ E tile[T][T + 1]; // [column][row]
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * T, j0 = (int64_t)blockIdx.y * T;
    int bad = 0;
    const int64_t m = r0 + lane;
#pragma unroll 4
    for (int c = w; c < T; c += 4) {
        const int64_t j = j0 + c;
        const E x = (m < M && j < N) ? X[m + j * ldx] : E(0);
        bad |= !isfinite(x);
        tile[c][lane] = x;
    }
    __syncthreads();
    // segment (panel b0 + pb, column j0 + c): thread -> c = lane, pb = w, w + 4, ...
    const int64_t b0 = r0 / PR;
    for (int pb = w; pb < T / PR; pb += 4) {
        const int64_t b = b0 + pb, j = j0 + lane;
        if (b < NP && j < ldp) {
            E v[PR];
#pragma unroll
            for (int r = 0; r < PR; ++r)
                v[r] = tile[lane][pb * PR + r];
            E *dst = A + (b * ldp + j) * PR;
#pragma unroll
            for (int r = 0; r < PR; ++r)
                dst[r] = v[r];
        }
    }
    if (__any(bad) && lane == 0)
        atomicOr(&st->nonfinite, 1);
}

// Per-column scale of the quantised storage: s_j = max_m |X_mj| / Qmax
// (binary32 division; Qmax = 1 for BF16, 448 for E4M3; an all-zero column has
// s_j = 1).  One workgroup per column; flags NaN/Inf.
__global__ __launch_bounds__(256) void k_col_scale(const float *__restrict__ X, int64_t ldx,
                                                   int64_t M, float qmax,
                                                   float *__restrict__ scale, LoopState *st)
{
    __shared__ float red[4];
    const int64_t j = blockIdx.x;
    const float *col = X + j * ldx;
    float a = 0.0f;
    int bad = 0;
    for (int64_t m = threadIdx.x; m < M; m += 256) {
        const float x = col[m];
        bad |= !isfinite(x);
        a = fmaxf(a, fabsf(x));
    }
    if (__any(bad) && (threadIdx.x & 63) == 0)
        atomicOr(&st->nonfinite, 1);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        a = fmaxf(a, __shfl_xor(a, o, 64));
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = a;
    __syncthreads();
    if (threadIdx.x == 0) {
        const float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        scale[j] = amax > 0.0f ? amax / qmax : 1.0f;
    }
}

// Codes q_mj = encode(X_mj / s_j) (binary32 division, round to nearest even;
// E4M3 saturates to +-448) written into row panels.  Thread: one segment.
template <class C>
__global__ __launch_bounds__(256) void k_quantize(const float *__restrict__ X, int64_t ldx,
                                                  int64_t M, int64_t N, int64_t NP, int64_t ldp,
                                                  const float *__restrict__ scale,
                                                  unsigned char *__restrict__ Q)
{
    constexpr int PR = C::PR;
    const int64_t total = NP * ldp;
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * 256) {
        const int64_t b = s / ldp, j = s - b * ldp;
        float v[PR];
        const float sj = j < N ? scale[j] : 1.0f;
#pragma unroll
        for (int r = 0; r < PR; ++r) {
            const int64_t m = b * PR + r;
            v[r] = (m < M && j < N) ? X[m + j * ldx] / sj : 0.0f;
        }
        u32x4_t out;
        if constexpr (PR == 8) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const unsigned int lo = __bfloat16_as_ushort(__float2bfloat16(v[2 * i]));
                const unsigned int hi = __bfloat16_as_ushort(__float2bfloat16(v[2 * i + 1]));
                out[i] = lo | (hi << 16);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                float c[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    c[u] = __builtin_amdgcn_fmed3f(v[4 * i + u], 448.0f, -448.0f);
                int wd = __builtin_amdgcn_cvt_pk_fp8_f32(c[0], c[1], 0, false);
                wd = __builtin_amdgcn_cvt_pk_fp8_f32(c[2], c[3], wd, true);
                out[i] = (unsigned int)wd;
            }
        }
        *reinterpret_cast<u32x4_t *>(Q + s * 16) = out;
    }
}

// Squared column norms of the panel matrix (FP64), optionally after the
// explicit deflation A <- A - t p^T (eq. 3; Sec. 2.3 with t = lambda_k v;
// plain storage only).  Grid: (column blocks of 64) x (panel splits); each
// split writes its partial norms to cnpart[split][j].
template <class C>
__global__ __launch_bounds__(256) void k_deflate_panel(unsigned char *__restrict__ A, int64_t N,
                                                       int64_t NP, int64_t ldp,
                                                       const typename C::acc *__restrict__ t,
                                                       const typename C::acc *__restrict__ pk,
                                                       int update, const float *__restrict__ scale,
                                                       double *__restrict__ cnpart)
{
    using E = typename C::acc;
    constexpr int PR = C::PR;
    __shared__ double red[4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int64_t nsplit = gridDim.y;
    const int64_t b0 = NP * blockIdx.y / nsplit, b1 = NP * (blockIdx.y + 1) / nsplit;
    double s = 0.0;
    if (j < N) {
        const E pj = update ? pk[j] : E(0);
        double sj = 1.0;
        if constexpr (C::scaled)
            sj = (double)scale[j];
        for (int64_t b = b0 + w; b < b1; b += 4) {
            typename C::raw *ptr = reinterpret_cast<typename C::raw *>(A + (b * ldp + j) * 16);
            typename C::raw v = *ptr;
            if constexpr (!C::scaled) {
                if (update) {
#pragma unroll
                    for (int r = 0; r < PR; ++r)
                        v[r] = v[r] - t[b * PR + r] * pj;
                    *ptr = v;
                }
            }
            E e[PR];
            C::decode(v, e);
            double ss = 0.0;
#pragma unroll
            for (int r = 0; r < PR; ++r)
                ss += (double)e[r] * (double)e[r];
            s += ss * sj * sj;
        }
    }
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < N)
        cnpart[(int64_t)blockIdx.y * N + j] =
            red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane];
}

// The explicit deflation of component k fused with the first loading of
// component k + 1: A <- A - t p^T (as k_deflate_panel, same arithmetic), the
// squared column norms of the new A (partials cnpart[split][j]) and the
// loading products q_part[split][j] = sum over the split's rows of
// A'(m, j) t0(m), t0 being the next start (column c of A', formed beforehand
// from the old A by k_start_fill).  One read and one write of A instead of
// the deflation's read and write plus the first pass's read.  Grid: (column
// blocks of 64) x (panel splits = the pass's workgroup count, so that the
// loading side sums the partials as after a pass).
template <class C>
__global__ __launch_bounds__(256) void k_deflate_first(unsigned char *__restrict__ A, int64_t N,
                                                       int64_t NP, int64_t ldp,
                                                       const typename C::acc *__restrict__ t,
                                                       const typename C::acc *__restrict__ pk,
                                                       int update,
                                                       const typename C::acc *__restrict__ t0,
                                                       double *__restrict__ cnpart,
                                                       typename C::acc *__restrict__ q_part)
{
    static_assert(!C::scaled, "explicit deflation is for plain storage");
    using E = typename C::acc;
    constexpr int PR = C::PR;
    __shared__ double red[2][4][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int64_t nsplit = gridDim.y;
    const int64_t b0 = NP * blockIdx.y / nsplit, b1 = NP * (blockIdx.y + 1) / nsplit;
    double s = 0.0, qa = 0.0;
    if (j < N) {
        const E pj = update ? pk[j] : E(0);
        for (int64_t b = b0 + w; b < b1; b += 4) {
            typename C::raw *ptr = reinterpret_cast<typename C::raw *>(A + (b * ldp + j) * 16);
            typename C::raw v = *ptr;
            if (update) {
#pragma unroll
                for (int r = 0; r < PR; ++r)
                    v[r] = v[r] - t[b * PR + r] * pj;
                *ptr = v;
            }
            double ss = 0.0, sq = 0.0;
#pragma unroll
            for (int r = 0; r < PR; ++r) {
                const double e = (double)v[r];
                ss += e * e;
                sq += e * (double)t0[b * PR + r];
            }
            s += ss;
            qa += sq;
        }
    }
    red[0][w][lane] = s;
    red[1][w][lane] = qa;
    __syncthreads();
    if (w == 0 && j < N) {
        const int64_t o = (int64_t)blockIdx.y * N + j;
        cnpart[o] = red[0][0][lane] + red[0][1][lane] + red[0][2][lane] + red[0][3][lane];
        q_part[o] = (E)(red[1][0][lane] + red[1][1][lane] + red[1][2][lane] + red[1][3][lane]);
    }
}

// Column norms of A - t p_k^T predicted from those of A before that
// deflation: |A_j|^2 - 2 p_kj (A^T t)_j + p_kj^2 |t|^2, with A^T t = q' of
// the component's last pass (q' = A^T t_pass - W d = A^T (t_pass - V d)) and
// |t| = sigma.  Exact norms one deflation back plus this update choose the
// next start before the deflation is carried out (k_deflate_first).  A
// degenerate component (no deflation) keeps the norms.
template <typename E>
__global__ __launch_bounds__(256) void k_colnorm_predict(const double *__restrict__ cn,
                                                         int64_t N, const E *__restrict__ pk,
                                                         const double *__restrict__ qy,
                                                         const LoopState *st,
                                                         double *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N)
        return;
    double v = cn[j];
    if (!st->degenerate) {
        const double p = (double)pk[j], s = st->sigma;
        v += -2.0 * p * qy[j] + p * p * s * s;
        if (v < 0.0)
            v = 0.0;
    }
    out[j] = v;
}

// cn[j] = sum over splits of cnpart (fixed order); implicit mode: the norm of
// the residual column A_j - T P[j,:]^T from |A_j|^2 and the finished
// components, |A_j|^2 - 2 sum_i sigma_i P_ji (A^T v_i)_j + sum_i sigma_i^2 P_ji^2
// (scores mutually orthogonal, A^T v_i stored in W).
template <typename E>
__global__ __launch_bounds__(256) void k_colnorm_finish(const double *__restrict__ cnpart,
                                                        int nsplit, int64_t N,
                                                        double *__restrict__ cn0,
                                                        double *__restrict__ cn, int implicit,
                                                        int k, const E *__restrict__ P,
                                                        const double *__restrict__ W,
                                                        const double *__restrict__ sig)
{
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= N)
        return;
    double s;
    if (cnpart) {
        // in split order, eight loads issued before their adds
        s = 0.0;
        int i = 0;
        for (; i + 8 <= nsplit; i += 8) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                x[u] = cnpart[(int64_t)(i + u) * N + j];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                s += x[u];
        }
        for (; i < nsplit; ++i)
            s += cnpart[(int64_t)i * N + j];
        if (cn0)
            cn0[j] = s;
    } else {
        s = cn0[j];
    }
    if (implicit) {
        for (int i = 0; i < k; ++i) {
            const double pji = (double)P[j + (int64_t)i * N];
            s += -2.0 * sig[i] * pji * W[j + (int64_t)i * N] + sig[i] * sig[i] * pji * pji;
        }
        if (s < 0.0)
            s = 0.0;
    }
    cn[j] = s;
}

// Dot products of a given start vector g = T0[:, k], for the test in
// k_start_panel: part[b][0] = g . g and part[b][1 + i] = v_i . g over the
// 1024 rows of workgroup b (waves over the products, lanes over rows).
constexpr int kStartRows = 1024;
template <typename E>
__global__ __launch_bounds__(1024) void k_start_dots(const E *__restrict__ T0,
                                                     const E *__restrict__ V, int64_t M, int k,
                                                     int nd, double *__restrict__ part)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kStartRows;
    const int64_t r1 = M - r0 < kStartRows ? M : r0 + kStartRows;
    const E *g = T0 + (int64_t)k * M;
    for (int i = w - 1; i < nd; i += 16) {
        const E *v = i < 0 ? g : V + (int64_t)i * M;
        double a0 = 0.0, a1 = 0.0;
        int64_t m = r0 + lane;
        for (; m + 64 < r1; m += 128) {
            a0 += (double)v[m] * (double)g[m];
            a1 += (double)v[m + 64] * (double)g[m + 64];
        }
        if (m < r1)
            a0 += (double)v[m] * (double)g[m];
        const double sum = fwave_sum(a0 + a1);
        if (lane == 0)
            part[(int64_t)blockIdx.x * (nd + 1) + (i + 1)] = sum;
    }
}


// Start vector of component k (the pseudo-code's T^(k) <- R^(k)): explicit
// deflation takes the residual column from the panel copy; implicit forms
// A_j - sum_i sigma_i v_i P_ji.  Selection: replayed column, column k, the
// given vector, or the largest residual column norm (ties to the lowest
// index), with the fallbacks of the header.  Output t, zero-padded to NP*PR.
template <class C>
__global__ __launch_bounds__(1024) void k_start_panel(const unsigned char *__restrict__ A,
                                                      int64_t N, int64_t NP, int64_t ldp,
                                                      int64_t M, const float *__restrict__ scale,
                                                      int implicit,
                                                      const typename C::acc *__restrict__ V,
                                                      const typename C::acc *__restrict__ P,
                                                      const double *__restrict__ sig,
                                                      const double *__restrict__ cn,
                                                      const typename C::acc *__restrict__ T0,
                                                      StartArgs a, double tiny,
                                                      const double *__restrict__ part, int nb,
                                                      LoopState *st)
{
    __shared__ double sv[16];
    __shared__ double buf[1024];
    __shared__ int64_t si[16];
    __shared__ int64_t col_sel;
    __shared__ int use_given, degenerate;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        col_sel = -2;
        use_given = 0;
        degenerate = a.force_degenerate;
        if (a.replay_start && a.replay_start[a.k] >= 0 && a.replay_start[a.k] < N)
            col_sel = a.replay_start[a.k];
        else if (a.init == 1) {
            if (sqrt(cn[a.k]) >= tiny)
                col_sel = a.k;
        } else if (a.init == 2)
            use_given = 1;
    }
    __syncthreads();
    if (use_given) {
        // Norm of the given start and, for GS-PCA, of its part outside the
        // earlier normalised scores (|g|^2 - sum_i (v_i . g)^2, V orthonormal).
        // Fall back to the max-norm column if the norm is tiny or not finite,
        // or if less than a tenth of it lies outside span(V_(k)).
        // (the products come as per-row-block partials from k_start_dots,
        // added here in block order)
        const int nd = a.gs ? a.k : 0;
        double tot = 0.0, dd = 0.0;
        for (int c0 = 0; c0 < nd + 1; c0 += 1024) {
            const int j = c0 + tid;
            double r = 0.0;
            if (j < nd + 1) {
                int b = 0;
                for (; b + 8 <= nb; b += 8) { // in block order, eight loads ahead
                    double x[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        x[u] = part[(int64_t)(b + u) * (nd + 1) + j];
#pragma unroll
                    for (int u = 0; u < 8; ++u)
                        r += x[u];
                }
                for (; b < nb; ++b)
                    r += part[(int64_t)b * (nd + 1) + j];
            }
            buf[tid] = r;
            __syncthreads();
            if (tid == 0) {
                const int cnt = nd + 1 - c0 < 1024 ? nd + 1 - c0 : 1024;
                for (int q = 0; q < cnt; ++q) {
                    if (c0 + q == 0)
                        tot = buf[q];
                    else
                        dd += buf[q] * buf[q];
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            const double nrm = sqrt(tot);
            if (nrm >= tiny && isfinite(nrm) && tot - dd >= 0.01 * tot)
                col_sel = -1;
        }
        __syncthreads();
    }
    if (col_sel == -2) {
        double best = -1.0;
        int64_t bi = 0;
        for (int64_t n = tid; n < N; n += 1024) {
            const double v = cn[n];
            if (v > best) { best = v; bi = n; }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(best, o, 64);
            const int64_t oi = __shfl_xor(bi, o, 64);
            if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
        }
        if (lane == 0) { sv[w] = best; si[w] = bi; }
        __syncthreads();
        if (tid == 0) {
            double b = sv[0];
            int64_t i0 = si[0];
            for (int i = 1; i < 16; ++i)
                if (sv[i] > b || (sv[i] == b && si[i] < i0)) { b = sv[i]; i0 = si[i]; }
            col_sel = i0;
        }
        __syncthreads();
    }
    if (tid == 0 && col_sel >= 0 && !(sqrt(cn[col_sel]) >= tiny))
        degenerate = 1;
    __syncthreads();
    const int64_t c = col_sel;
    if (tid == 0) {
        st->start_col = (int32_t)c;
        st->iter = 0;
        st->mu = 0.0;
        st->sigma = 0.0;
        st->pnorm = 1.0;
        st->delta = 1.0;
        st->delta_prev = 1.0;
        st->dp = INFINITY;
        st->converged = 0;
        st->degenerate = degenerate;
        st->done = degenerate;
    }
}

// t = the chosen start (st->start_col, set by k_start_panel): the given
// vector (-1) or column c of the residual -- of A itself, or of
// X - T P^T formed from the finished components in implicit mode --
// zero-padded to NP*PR rows; one thread per row.
template <class C>
__global__ __launch_bounds__(256) void k_start_fill(const unsigned char *__restrict__ A, int64_t N,
                                                    int64_t NP, int64_t ldp, int64_t M,
                                                    const float *__restrict__ scale, int implicit,
                                                    const typename C::acc *__restrict__ V,
                                                    const typename C::acc *__restrict__ P,
                                                    const double *__restrict__ sig,
                                                    const typename C::acc *__restrict__ T0, int k,
                                                    typename C::acc *__restrict__ t,
                                                    const LoopState *st,
                                                    const typename C::acc *__restrict__ dt,
                                                    const typename C::acc *__restrict__ dp)
{
    using E = typename C::acc;
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (m >= NP * C::PR)
        return;
    const int64_t c = st->start_col;
    E v = E(0);
    if (m < M) {
        if (c < 0) {
            v = T0[m + (int64_t)k * M];
        } else if (dt) {
            // column c of A - dt dp^T before that deflation is carried out,
            // in the deflation's own arithmetic
            const E a = panel_elem<C>(A, ldp, m, c, scale);
            v = a - dt[m] * dp[c];
        } else {
            double s = (double)panel_elem<C>(A, ldp, m, c, scale);
            if (implicit)
                for (int i = 0; i < k; ++i)
                    s -= sig[i] * (double)V[m + (int64_t)i * M] * (double)P[c + (int64_t)i * N];
            v = (E)s;
        }
    }
    t[m] = v;
}

// q = sum_g q_part[g] (FP64, fixed order), q' = q - W d (the Gram-Schmidt
// correction of t carried to the loading side), then the loading's
// Gram-Schmidt coefficients c = P_(k)^T q' (Sec. 2.3), finished by the last
// workgroup.  `it` is the iteration this launch belongs to: when the
// component stopped in that iteration only q' is formed (it feeds W); when
// it stopped earlier the launch does nothing.  Workgroup: 64 columns x
// kFinGroups groups of partials (4 loads in flight per thread; the group sums
// are combined in a fixed order).
template <typename E>
__global__ __launch_bounds__(64 * kFinGroups) void k_fin_q(
    const E *__restrict__ q_part, int64_t G, int64_t N, const double *__restrict__ W, int kd,
    const double *__restrict__ d, const E *__restrict__ P, int kg, double *__restrict__ qy,
    double *__restrict__ cpart, double *__restrict__ c, LoopState *st, int it)
{
    if (st->degenerate)
        return;
    const int done = st->done;
    if (done && st->iter != it)
        return;
    constexpr int NG = kFinGroups;
    __shared__ double part[NG][64];
    __shared__ double ys[64];
    __shared__ int last;
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * 64;
    const int64_t j = r0 + lane;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (j < N) {
        int64_t g = grp;
        // sixteen loads in flight, added in the same order as the loop below
        for (; g + 15 * NG < G; g += 16 * NG) {
            E x[16];
#pragma unroll
            for (int u = 0; u < 16; ++u)
                x[u] = q_part[(g + u * NG) * N + j];
#pragma unroll
            for (int u = 0; u < 16; u += 4) {
                a0 += (double)x[u];
                a1 += (double)x[u + 1];
                a2 += (double)x[u + 2];
                a3 += (double)x[u + 3];
            }
        }
        for (; g + 3 * NG < G; g += 4 * NG) {
            a0 += (double)q_part[g * N + j];
            a1 += (double)q_part[(g + NG) * N + j];
            a2 += (double)q_part[(g + 2 * NG) * N + j];
            a3 += (double)q_part[(g + 3 * NG) * N + j];
        }
        for (; g < G; g += NG)
            a0 += (double)q_part[g * N + j];
    }
    part[grp][lane] = (a0 + a1) + (a2 + a3);
    // W d, the W columns split over the groups
    double pr = 0.0;
    if (j < N)
#pragma unroll 4
        for (int i = grp; i < kd; i += NG)
            pr += W[j + (int64_t)i * N] * d[i];
    __syncthreads();
    double v = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q)
        v += part[q][lane];
    __syncthreads();
    part[grp][lane] = pr;
    __syncthreads();
    double wd = 0.0;
#pragma unroll
    for (int q = 0; q < NG; ++q)
        wd += part[q][lane];
    const double qv = v - wd;
    if (grp == 0) {
        if (j < N)
            qy[j] = qv;
        ys[lane] = j < N ? qv : 0.0;
    }
    if (done || kg == 0)
        return;
    __syncthreads();
    int i = grp;
    // eight coefficients at a time: their loads are issued before the first
    // wave sum (many earlier components: the loads would otherwise wait one
    // after another behind each sum)
    for (; i + 7 * NG < kg; i += 8 * NG) {
        double sv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            sv[u] = (j < N) ? (double)P[j + (int64_t)(i + u * NG) * N] * ys[lane] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const double sum = fwave_sum(sv[u]);
            if (lane == 0)
                cpart[(int64_t)blockIdx.x * kg + i + u * NG] = sum;
        }
    }
    for (; i < kg; i += NG) {
        const double sv = (j < N) ? (double)P[j + (int64_t)i * N] * ys[lane] : 0.0;
        const double sum = fwave_sum(sv);
        if (lane == 0)
            cpart[(int64_t)blockIdx.x * kg + i] = sum;
    }
    if (!arrive_last(&st->counter[kCntDotN], &last))
        return;
    reduce_partials(cpart, gridDim.x, kg, c, &part[0][0]);
    if (threadIdx.x == 0)
        st->counter[kCntDotN] = 0;
}

// The loading side of an iteration in one workgroup when N <= 1024 (no
// cross-workgroup reduction, one launch instead of two): q = sum_g q_part[g]
// (fixed order), q' = q - W d, c = P_(k)^T q', p = q' - P_(k) c (Sec. 2.3),
// |p| and the loading change -- the steps and state updates of k_fin_q
// followed by k_gs_apply on the loading side.  Column j belongs to thread j;
// the partials are summed by NT / N' groups of threads (N' = N rounded up to
// whole waves), eight loads in flight, groups added in order.
constexpr int kFinApplyThreads = 1024;
static_assert(kFinApplyMaxN == kFinApplyThreads, "one column per thread");
template <typename E>
__device__ __attribute__((always_inline)) inline void fin_apply_body(const E *__restrict__ q_part, int64_t G, int64_t N,
                               const double *__restrict__ W, int kd,
                               const double *__restrict__ d, const E *__restrict__ P, int kg,
                               double *__restrict__ qy, double *__restrict__ p,
                               double *__restrict__ pprev, LoopState *st, int it, int stop,
                               double tiny)
{
    if (st->degenerate)
        return;
    const int done = st->done;
    // the state this iteration started from, read before thread 0 updates it
    const int iter0 = st->iter;
    const double pn_old = st->pnorm;
    if (done && iter0 != it)
        return;
    constexpr int NT = kFinApplyThreads, NW = NT / 64;
    __shared__ double part[NT];
    __shared__ double qs[NT];
    __shared__ double cs[NT];
    __shared__ double red[3][NW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int Np = (int)((N + 63) / 64) * 64;
    const int NGr = NT / Np;
    const int j = tid % Np, gr = tid / Np;
    const int64_t jc = j < N ? j : N - 1;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (gr < NGr) {
        for (int64_t g0 = gr; g0 < G; g0 += 8 * (int64_t)NGr) {
            E x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int64_t g = g0 + (int64_t)u * NGr;
                x[u] = q_part[(g < G ? g : G - 1) * N + jc];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                a[u] += g0 + (int64_t)u * NGr < G ? (double)x[u] : 0.0;
        }
    }
    part[tid] = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    __syncthreads();
    double qv = 0.0;
    if (tid < N) {
        double q = 0.0;
        for (int r = 0; r < NGr; ++r)
            q += part[r * Np + tid];
        double wd = 0.0;
        for (int i = 0; i < kd; ++i)
            wd += W[tid + (int64_t)i * N] * d[i];
        qv = q - wd;
        qy[tid] = qv;
        qs[tid] = qv;
    }
    if (done) // stopped in this iteration: q' only feeds W
        return;
    __syncthreads();
    for (int i = w; i < kg; i += NW) { // c = P^T q': wave per coefficient
        double sacc = 0.0;
        for (int jj = lane; jj < N; jj += 64)
            sacc += (double)P[jj + (int64_t)i * N] * qs[jj];
        sacc = fwave_sum(sacc);
        if (lane == 0)
            cs[i] = sacc;
    }
    __syncthreads();
    double v = 0.0, o = 0.0;
    if (tid < N) {
        double pr = 0.0;
        for (int i = 0; i < kg; ++i)
            pr += (double)P[tid + (int64_t)i * N] * cs[i];
        v = qv - pr;
        o = p[tid];
        pprev[tid] = o;
        p[tid] = v;
    }
    // |p|^2 and p . p_old: wave sums, then the waves in order
    double s2 = fwave_sum(v * v), dt = fwave_sum(tid < N ? v * o : 0.0);
    if (lane == 0) {
        red[0][w] = s2;
        red[1][w] = dt;
    }
    __syncthreads();
    double tot = 0.0, dtot = 0.0;
    for (int q = 0; q < NW; ++q) {
        tot += red[0][q];
        dtot += red[1][q];
    }
    const double nrm = sqrt(tot);
    double dp = INFINITY;
    if (stop == 1 && iter0 > 0 && nrm > 0.0 && pn_old > 0.0) {
        // |p/|p| - s p_old/|p_old|| (s aligning the signs), fixed order
        const double ia = 1.0 / nrm, ib = (dtot >= 0.0 ? 1.0 : -1.0) / pn_old;
        const double e = tid < N ? v * ia - o * ib : 0.0;
        const double ss = fwave_sum(e * e);
        if (lane == 0)
            red[2][w] = ss;
        __syncthreads();
        double sst = 0.0;
        for (int q = 0; q < NW; ++q)
            sst += red[2][q];
        dp = sqrt(sst);
    }
    if (tid != 0)
        return;
    st->dp = dp;
    st->pnorm = nrm;
    if (!(nrm >= tiny)) { // counts as the iteration in which it happened
        st->iter = iter0 + 1;
        st->degenerate = 1;
        st->done = 1;
    }
}

template <typename E>
__global__ __launch_bounds__(kFinApplyThreads) void k_fin_apply(
    const E *__restrict__ q_part, int64_t G, int64_t N, const double *__restrict__ W, int kd,
    const double *__restrict__ d, const E *__restrict__ P, int kg, double *__restrict__ qy,
    double *__restrict__ p, double *__restrict__ pprev, LoopState *st, int it, int stop,
    double tiny)
{
    fin_apply_body<E>(q_part, G, N, W, kd, d, P, kg, qy, p, pprev, st, it, stop, tiny);
}

// Gram-Schmidt coefficients of the score, d = V_(k)^T t (FP64), from the
// complete t of the pass: workgroup (b, y) takes `rows` consecutive rows of t
// (staged in LDS, zero past M) and columns [32y, 32y + 32) of V, two columns
// per wave; a lane issues the loads of 16 rows of both its columns before the
// first use (row and column indices clamped, their weights zero; the first
// chunk's loads are issued before the barrier that publishes the rows of t).
// Per-row-block partials are added in a fixed order by the last workgroup,
// which also finishes sigma and the stop test; a grid of one workgroup keeps
// its partials in LDS and needs no arrival counter.
constexpr int kScoreThreads = 1024;
template <typename E>
__device__ __attribute__((always_inline)) inline void score_dot_body(const double *__restrict__ t, int64_t M,
                               const E *__restrict__ V, int kd, int64_t rows,
                               const double *__restrict__ tsq, int G,
                               double *__restrict__ cpart, double *__restrict__ d,
                               LoopState *st, double tol, int32_t limit, int replay, double tiny,
                               int stop)
{
    if (st->done)
        return;
    __shared__ double ts[kScoreRows];
    __shared__ double lds[kScoreThreads];
    __shared__ double dsh[32];
    __shared__ int last;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = kScoreThreads / 64;
    const bool single = gridDim.x == 1 && gridDim.y == 1;
    const int64_t r0 = (int64_t)blockIdx.x * rows;
    const int n = (int)(M - r0 < rows ? M - r0 : rows);
    const int i0 = 32 * (int)blockIdx.y + w, i1 = i0 + nw;
    const E *c0 = V + (int64_t)(i0 < kd ? i0 : (kd > 0 ? kd - 1 : 0)) * M + r0;
    const E *c1 = V + (int64_t)(i1 < kd ? i1 : (kd > 0 ? kd - 1 : 0)) * M + r0;
    E v0[16], v1[16];
    auto load_chunk = [&](int x0) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int x = x0 + lane + 64 * u, xc = x < n ? x : n - 1;
            v0[u] = c0[xc];
            v1[u] = c1[xc];
        }
    };
    if (kd > 0)
        load_chunk(0);
    for (int x = tid; x < rows; x += kScoreThreads)
        ts[x] = x < n ? t[r0 + x] : 0.0;
    __syncthreads();
    if (kd > 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int x0 = 0; x0 < n; x0 += 16 * 64) {
            if (x0 > 0)
                load_chunk(x0);
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const double tv = ts[x0 + lane + 64 * u]; // zero past n
                a0 += (double)v0[u] * tv;
                a1 += (double)v1[u] * tv;
            }
        }
        const double s0 = fwave_sum(a0), s1 = fwave_sum(a1);
        if (lane == 0) {
            if (single) {
                if (i0 < kd)
                    dsh[i0] = s0;
                if (i1 < kd)
                    dsh[i1] = s1;
            } else {
                if (i0 < kd && i0 < 32 * (int)blockIdx.y + 32)
                    cpart[(int64_t)blockIdx.x * kd + i0] = s0;
                if (i1 < kd && i1 < 32 * (int)blockIdx.y + 32)
                    cpart[(int64_t)blockIdx.x * kd + i1] = s1;
            }
        }
    }
    if (!single && !arrive_last(&st->counter[kCntDotM], &last))
        return;
    // the |t|^2 partials and the loop state are loaded before the partials of
    // d are reduced, so that their loads overlap
    double tq = 0.0;
    for (int q = tid; q < G; q += kScoreThreads)
        tq += tsq[q];
    ScoreState ss{};
    if (tid == 0)
        ss = score_state(st);
    double ssq = 0.0;
    if (single) {
        __syncthreads();
        if (tid < kd) {
            const double dv = dsh[tid];
            d[tid] = dv;
            ssq = dv * dv;
        }
    } else if (kd > 0) {
        ssq = reduce_partials<16>(cpart, gridDim.x, kd, d, lds);
    }
    // |t|^2 and |d|^2 in a fixed order: wave sums, then the waves in order
    const double tqw = fwave_sum(tq), ssw = fwave_sum(ssq);
    __syncthreads();
    if (lane == 0) {
        lds[w] = tqw;
        lds[nw + w] = ssw;
    }
    __syncthreads();
    if (tid != 0)
        return;
    double tt = 0.0, dd = 0.0;
    for (int q = 0; q < nw; ++q) {
        tt += lds[q];
        dd += lds[nw + q];
    }
    if (!single)
        st->counter[kCntDotM] = 0;
    // sigma = |t - V d| = sqrt(|t|^2 - |d|^2) (V orthonormal; d is at rounding
    // level once t has been formed from a loading orthogonal to P_(k))
    const double s2 = tt - dd;
    score_test(st, ss, s2 > 0.0 ? sqrt(s2) : 0.0, tol, limit, replay, tiny, stop);
}

template <typename E>
__global__ __launch_bounds__(kScoreThreads) void k_score_dot(
    const double *__restrict__ t, int64_t M, const E *__restrict__ V, int kd, int64_t rows,
    const double *__restrict__ tsq, int G, double *__restrict__ cpart, double *__restrict__ d,
    LoopState *st, double tol, int32_t limit, int replay, double tiny, int stop)
{
    score_dot_body<E>(t, M, V, kd, rows, tsq, G, cpart, d, st, tol, limit, replay, tiny, stop);
}

// The score side and the loading side of an iteration in one launch when
// each fits one workgroup (the score's rows in one block, N <= 1024 and the
// q partials small): k_score_dot's steps, a barrier (d and the loop state,
// written by this workgroup, are then visible to all its threads), then
// k_fin_apply's steps -- the same arithmetic in the same order, one kernel
// boundary fewer per iteration.
static_assert(kScoreThreads == kFinApplyThreads, "one workgroup runs both steps");
template <typename E>
__global__ __launch_bounds__(kScoreThreads) void k_score_fin(
    const double *__restrict__ t, int64_t M, const E *__restrict__ V, int kd, int64_t rows,
    const double *__restrict__ tsq, int G, double *__restrict__ cpart, double *__restrict__ d,
    double tol, int32_t limit, int replay, const E *__restrict__ q_part, int64_t Gq, int64_t N,
    const double *__restrict__ W, const E *__restrict__ P, int kg, double *__restrict__ qy,
    double *__restrict__ p, double *__restrict__ pprev, LoopState *st, int it, int stop,
    double tiny)
{
    score_dot_body<E>(t, M, V, kd, rows, tsq, G, cpart, d, st, tol, limit, replay, tiny, stop);
    __syncthreads();
    fin_apply_body<E>(q_part, Gq, N, W, kd, d, P, kg, qy, p, pprev, st, it, stop, tiny);
}

// Finish component k: V[:,k] = t / sigma (GS) or T[:,k] = t (NIPALS),
// P[:,k] = p / |p|, and the new column of W = A^T V:
//   A^T v_k = q' / sigma (q' = A^T t of the last pass), minus sigma p_k when A
//   is the explicitly deflated residual (R <- R - sigma v_k p_k^T).
template <typename E>
__global__ __launch_bounds__(256) void k_comp_end(const double *__restrict__ td,
                                                  const double *__restrict__ d, int kd,
                                                  E *__restrict__ tE, int64_t M, int64_t N,
                                                  const double *__restrict__ p,
                                                  const double *__restrict__ qy, int k, int gs,
                                                  int explicit_defl, E *__restrict__ T,
                                                  E *__restrict__ P, double *__restrict__ W,
                                                  double *sigma, int32_t *iters,
                                                  int32_t *start_col, LoopState *st)
{
    const int deg = st->degenerate;
    const double s = st->sigma, pn = st->pnorm;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) {
        // the score after its Gram-Schmidt pass, t' = t - V_(k) d (Sec. 2.3)
        double v = 0.0;
        if (!deg) {
            v = td[i];
            for (int j = 0; j < kd; ++j)
                v -= (double)T[i + (int64_t)j * M] * d[j];
        }
        tE[i] = (E)v;
        T[i + (int64_t)k * M] = deg ? E(0) : (gs ? (E)(v / s) : (E)v);
    }
    if (i < N) {
        const double pk = p[i] / pn;
        P[i + (int64_t)k * N] = (E)pk;
        if (W)
            W[i + (int64_t)k * N] = deg ? 0.0 : qy[i] / s - (explicit_defl ? s * pk : 0.0);
    }
    if (i == 0) {
        sigma[k] = deg ? 0.0 : s;
        if (iters)
            iters[k] = st->iter;
        if (start_col)
            start_col[k] = st->start_col;
    }
}

// ---------------------------------------------------------------------------
// Launchers.

template <int F>
void Fused<F>::retile(const E *X, int64_t ldx, int64_t M, int64_t N, int64_t NP, int64_t ldp,
                      unsigned char *A, LoopState *st, hipStream_t s)
{
    if constexpr (F == kFmtF64 || F == kFmtF32) {
        const dim3 grid(fcdiv(NP * (16 / (int64_t)sizeof(E)), kRetileTile),
                        fcdiv(ldp, kRetileTile));
        hipLaunchKernelGGL(k_retile<E>, grid, dim3(256), 0, s, X, ldx, M, N, NP, ldp,
                           reinterpret_cast<E *>(A), st);
    }
}

template <int F>
void Fused<F>::quantize(const float *X, int64_t ldx, int64_t M, int64_t N, int64_t NP,
                        int64_t ldp, float *scale, unsigned char *Q, LoopState *st, hipStream_t s)
{
    using C = typename CodecOf<F>::type;
    if constexpr (C::scaled) {
        const float qmax = C::PR == 16 ? 448.0f : 1.0f;
        hipLaunchKernelGGL(k_col_scale, dim3((unsigned)N), dim3(256), 0, s, X, ldx, M, qmax, scale,
                           st);
        const int64_t total = NP * ldp;
        const unsigned g = (unsigned)std::min<int64_t>(fcdiv(total, 256), 8192);
        hipLaunchKernelGGL(k_quantize<C>, dim3(g), dim3(256), 0, s, X, ldx, M, N, NP, ldp, scale,
                           Q);
    }
}

template <int F>
void Fused<F>::deflate(unsigned char *A, int64_t N, int64_t NP, int64_t ldp, const E *t,
                       const E *pk, int update, const float *scale, int nsplit, double *cnpart,
                       hipStream_t s)
{
    using C = typename CodecOf<F>::type;
    hipLaunchKernelGGL(k_deflate_panel<C>, dim3(fcdiv(N, 64), nsplit), dim3(256), 0, s, A, N, NP,
                       ldp, t, pk, update, scale, cnpart);
}

template <int F>
void Fused<F>::colnorm_finish(const double *cnpart, int nsplit, int64_t N, double *cn0,
                              double *cn, int implicit, int k, const E *P, const double *W,
                              const double *sig, hipStream_t s)
{
    hipLaunchKernelGGL(k_colnorm_finish<E>, dim3(fcdiv(N, 256)), dim3(256), 0, s, cnpart, nsplit,
                       N, cn0, cn, implicit, k, P, W, sig);
}

template <int F>
void Fused<F>::start(const unsigned char *A, int64_t N, int64_t NP, int64_t ldp, int64_t M,
                     const float *scale, int implicit, const E *V, const E *P, const double *sig,
                     const double *cn, const E *T0, StartArgs a, double tiny, E *t,
                     double *part, LoopState *st, hipStream_t s, const E *defl_t,
                     const E *defl_p)
{
    using C = typename CodecOf<F>::type;
    const int nb = (int)fcdiv(M, kStartRows);
    if (a.init == 2 && T0) {
        const int nd = a.gs ? a.k : 0;
        hipLaunchKernelGGL(k_start_dots<E>, dim3((unsigned)nb), dim3(1024), 0, s, T0, V, M, a.k,
                           nd, part);
    }
    hipLaunchKernelGGL(k_start_panel<C>, dim3(1), dim3(1024), 0, s, A, N, NP, ldp, M, scale,
                       implicit, V, P, sig, cn, T0, a, tiny, part, nb, st);
    hipLaunchKernelGGL(k_start_fill<C>, dim3(fcdiv(NP * C::PR, 256)), dim3(256), 0, s, A, N, NP,
                       ldp, M, scale, implicit, V, P, sig, T0, a.k, t, st, defl_t, defl_p);
}

template <int F>
void Fused<F>::deflate_first(unsigned char *A, int64_t N, int64_t NP, int64_t ldp, const E *t,
                             const E *pk, int update, const E *t0, int nsplit, double *cnpart,
                             E *q_part, hipStream_t s)
{
    using C = typename CodecOf<F>::type;
    if constexpr (!C::scaled)
        hipLaunchKernelGGL(k_deflate_first<C>, dim3(fcdiv(N, 64), nsplit), dim3(256), 0, s, A, N,
                           NP, ldp, t, pk, update, t0, cnpart, q_part);
}

template <int F>
void Fused<F>::colnorm_predict(const double *cn, int64_t N, const E *pk, const double *qy,
                               const LoopState *st, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_colnorm_predict<E>, dim3(fcdiv(N, 256)), dim3(256), 0, s, cn, N, pk, qy,
                       st, out);
}

template <int F>
void Fused<F>::score_dot(const double *t, int64_t M, const E *V, int kd, const double *tsq,
                         int G, double *cpart, double *d, LoopState *st, double tol,
                         int32_t limit, int replay, double tiny, int stop, hipStream_t s)
{
    const int64_t rows = score_rows(M, kd);
    const unsigned cols = kd > 0 ? (unsigned)fcdiv(kd, 32) : 1u;
    hipLaunchKernelGGL(k_score_dot<E>, dim3(fcdiv(M, rows), cols), dim3(kScoreThreads), 0, s, t,
                       M, V, kd, rows, tsq, G, cpart, d, st, tol, limit, replay, tiny, stop);
}

template <int F>
void Fused<F>::fin_q(const E *q_part, int64_t G, int64_t N, const double *W, int kd,
                     const double *d, const E *P, int kg, double *qy, double *cpart, double *c,
                     LoopState *st, int it, hipStream_t s)
{
    hipLaunchKernelGGL(k_fin_q<E>, dim3(fcdiv(N, 64)), dim3(64 * kFinGroups), 0, s, q_part, G, N,
                       W, kd, d, P,
                       kg, qy, cpart, c, st, it);
}

template <int F>
bool Fused<F>::score_fin_fits(int64_t M, int kd)
{
    return fcdiv(M, score_rows(M, kd)) == 1 && (kd > 0 ? fcdiv(kd, 32) : 1) == 1;
}

template <int F>
void Fused<F>::score_fin(const double *t, int64_t M, const E *V, int kd, const double *tsq,
                         int G, double *cpart, double *d, double tol, int32_t limit, int replay,
                         const E *q_part, int64_t Gq, int64_t N, const double *W, const E *P,
                         int kg, double *qy, double *p, double *pprev, LoopState *st, int it,
                         int stop, double tiny, hipStream_t s)
{
    hipLaunchKernelGGL(k_score_fin<E>, dim3(1), dim3(kScoreThreads), 0, s, t, M, V, kd,
                       score_rows(M, kd), tsq, G, cpart, d, tol, limit, replay, q_part, Gq, N, W,
                       P, kg, qy, p, pprev, st, it, stop, tiny);
}

template <int F>
void Fused<F>::fin_apply(const E *q_part, int64_t G, int64_t N, const double *W, int kd,
                         const double *d, const E *P, int kg, double *qy, double *p,
                         double *pprev, LoopState *st, int it, int stop, double tiny,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_fin_apply<E>, dim3(1), dim3(kFinApplyThreads), 0, s, q_part, G, N, W, kd,
                       d, P, kg, qy, p, pprev, st, it, stop, tiny);
}

template <int F>
void Fused<F>::comp_end(const double *td, const double *d, int kd, E *tE, int64_t M, int64_t N,
                        const double *p, const double *qy, int k, int gs, int explicit_defl,
                        E *T, E *P, double *W, double *sigma, int32_t *iters,
                        int32_t *start_col, LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_comp_end<E>, dim3(fcdiv(M > N ? M : N, 256)), dim3(256), 0, s, td, d, kd,
                       tE, M, N, p, qy, k, gs, explicit_defl, T, P, W, sigma, iters, start_col,
                       st);
}

template struct Fused<kFmtF64>;
template struct Fused<kFmtF32>;
template struct Fused<kFmtBF16>;
template struct Fused<kFmtFP8>;

}  // namespace gspca
