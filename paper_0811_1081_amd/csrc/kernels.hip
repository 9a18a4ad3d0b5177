// kernels.hip -- gfx950 kernels of the GS-PCA / NIPALS-PCA power iteration.
//
// Each iteration of Sec. 2.3 (GS-PCA) maps to six launches:
//   gemv_t   q = R^T t              streaming R, split-row partial sums
//   gs_dot   c = P_(k)^T q          (FP64; skipped for k = 0 and for NIPALS)
//   gs_apply p = q - P_(k) c, |p|   (FP64; last workgroup finishes |p|)
//   gemv_n   t = R p / |p|          streaming R, split-column partial sums
//   gs_dot   d = V_(k)^T t          (FP64)
//   gs_apply t = t - V_(k) d, sigma = |t|, relative test (last workgroup)
// The score is kept unnormalised during the iteration: the next loading is
// normalised after the Gram-Schmidt pass, so the scale 1/sigma of Sec. 2.3's
// V <- V / lambda cancels and is applied once, when the component finishes.
//
// Reductions are deterministic: partials are written to workspace and summed
// in a fixed order; no floating-point atomics.  Every kernel of the loop
// returns at once when the current component has already stopped, so the
// host may enqueue iterations ahead of the convergence test.
#include <float.h>
#include <math.h>

#include "internal.h"

namespace gspca {

// Sum of the nsplit partials part[s * ldpart + r] in split order, eight
// loads issued before their adds.
__device__ inline double sum_parts(const double *__restrict__ part, int nsplit, int64_t ldpart,
                                   int64_t r)
{
    double v = 0.0;
    int s = 0;
    for (; s + 8 <= nsplit; s += 8) {
        double x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            x[u] = part[(int64_t)(s + u) * ldpart + r];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            v += x[u];
    }
    for (; s < nsplit; ++s)
        v += part[(int64_t)s * ldpart + r];
    return v;
}

// 16-byte native vectors (one global_load_dwordx4 per lane).
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename E> struct V16;
template <> struct V16<float> { using T = f32x4; static constexpr int n = 4; };
template <> struct V16<double> { using T = f64x2; static constexpr int n = 2; };

__device__ inline float vdot(f32x4 a, f32x4 b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3]; }
__device__ inline double vdot(f64x2 a, f64x2 b) { return a[0] * b[0] + a[1] * b[1]; }

template <typename T>
__device__ inline T wave_sum(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over a 256-thread workgroup; every thread gets the result.
template <typename T>
__device__ inline T block_sum(T v, T *lds4)
{
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0)
        lds4[w] = v;
    __syncthreads();
    T r = T(0);
    for (int i = 0; i < kBlock / 64; ++i)
        r += lds4[i];
    return r;
}


// ---------------------------------------------------------------------------
// R <- X (Sec. 2.2/2.3 first step) into the padded layout; flags NaN/Inf.

template <typename E>
__global__ __launch_bounds__(kBlock) void k_copy_pad(const E *__restrict__ X, int64_t ldx,
                                                     E *__restrict__ R, int64_t ldr, int64_t M,
                                                     int64_t N, LoopState *st)
{
    int bad = 0;
    for (int64_t n = blockIdx.y; n < N; n += gridDim.y) {
        const E *x = X + n * ldx;
        E *r = R + n * ldr;
        for (int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x; m < ldr;
             m += (int64_t)gridDim.x * kBlock) {
            const E v = m < M ? x[m] : E(0);
            bad |= !isfinite(v);
            r[m] = v;
        }
    }
    if (__any(bad) && (threadIdx.x & 63) == 0)
        atomicOr(&st->nonfinite, 1);
}

// Squared column norms in FP64: one wave per column.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_colnorm(const E *__restrict__ R, int64_t ldr,
                                                    int64_t M, int64_t N, double *cn)
{
    using VT = typename V16<E>::T;
    constexpr int VN = V16<E>::n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int64_t n = (int64_t)blockIdx.x * 4 + w; n < N; n += (int64_t)gridDim.x * 4) {
        const E *col = R + n * ldr;
        double s = 0.0;
        for (int64_t m = (int64_t)lane * VN; m < ldr; m += 64 * VN) {
            const VT v = *reinterpret_cast<const VT *>(col + m);
            const E *e = reinterpret_cast<const E *>(&v);
#pragma unroll
            for (int i = 0; i < VN; ++i)
                s += (double)e[i] * (double)e[i];
        }
        s = wave_sum(s);
        if (lane == 0)
            cn[n] = s;
    }
}

// Start vector (the pseudo-code's T^(k) <- R^(k)); one 1024-thread workgroup.
template <typename E>
__global__ __launch_bounds__(1024) void k_start(const E *__restrict__ R, int64_t ldr, int64_t M,
                                                int64_t N, const double *__restrict__ cn,
                                                const E *__restrict__ V,
                                                const E *__restrict__ T0, StartArgs a,
                                                double tiny, E *__restrict__ t, LoopState *st)
{
    __shared__ double sv[16];
    __shared__ int64_t si[16];
    __shared__ int64_t col_sel;
    __shared__ int use_given, degenerate;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;

    if (tid == 0) {
        col_sel = -2; // -2: undecided, -1: given vector
        use_given = 0;
        degenerate = a.force_degenerate;
        if (a.replay_start && a.replay_start[a.k] >= 0 && a.replay_start[a.k] < N) {
            col_sel = a.replay_start[a.k];
        } else if (a.init == 1) { // column k
            if (sqrt(cn[a.k]) >= tiny)
                col_sel = a.k;
        } else if (a.init == 2) {
            use_given = 1;
        }
    }
    __syncthreads();
    if (use_given) {
        // Norm of the given start and, for GS-PCA, of its part outside the
        // earlier normalised scores (|g|^2 - sum_i (v_i . g)^2, V orthonormal).
        // Fall back to the max-norm column if the norm is tiny or not finite,
        // or if less than a tenth of it lies outside span(V_(k)).
        const E *g = T0 + (int64_t)a.k * M;
        const int nd = a.gs ? a.k : 0;
        double tot = 0.0, dd = 0.0;
        for (int i = -1; i < nd; ++i) {
            const E *v = i < 0 ? g : V + (int64_t)i * M;
            double s = 0.0;
            for (int64_t m = tid; m < M; m += 1024)
                s += (double)v[m] * (double)g[m];
            s = wave_sum(s);
            if (lane == 0)
                sv[w] = s;
            __syncthreads();
            double r = 0.0;
            for (int j = 0; j < 16; ++j)
                r += sv[j];
            __syncthreads();
            if (i < 0)
                tot = r;
            else
                dd += r * r;
        }
        if (tid == 0) {
            const double nrm = sqrt(tot);
            if (nrm >= tiny && isfinite(nrm) && tot - dd >= 0.01 * tot)
                col_sel = -1;
        }
        __syncthreads();
    }
    if (col_sel == -2) {
        // argmax of the column norms, ties to the lowest index
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
    const E *src = c >= 0 ? R + c * ldr : T0 + (int64_t)a.k * M;
    for (int64_t m = tid; m < ldr; m += 1024)
        t[m] = m < M ? src[m] : E(0);
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

// ---------------------------------------------------------------------------
// q_part[s][n] = sum over rows of split s of R[m, n] t[m]   (p <- R^T t).
// Workgroup: CB columns x one row split; 16-byte loads along each column,
// the t chunk loaded once per row step and reused across the CB columns.

template <typename E, int CB>
__global__ __launch_bounds__(kBlock) void k_gemv_t(const E *__restrict__ R, int64_t ldr, int64_t N,
                                                   const E *__restrict__ t, int64_t rows_per_split,
                                                   double *__restrict__ qpart,
                                                   const LoopState *__restrict__ st)
{
    if (st->done)
        return;
    using VT = typename V16<E>::T;
    constexpr int VN = V16<E>::n;
    __shared__ E lds[kBlock / 64][CB];
    const int64_t n0 = (int64_t)blockIdx.x * CB;
    const int64_t r0 = (int64_t)blockIdx.y * rows_per_split;
    const int64_t r1 = min(r0 + rows_per_split, ldr);
    const E *cols[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
        cols[c] = R + min(n0 + c, N - 1) * ldr;
    E acc[CB];
#pragma unroll
    for (int c = 0; c < CB; ++c)
        acc[c] = E(0);
    for (int64_t m = r0 + (int64_t)threadIdx.x * VN; m < r1; m += kBlock * VN) {
        const VT tv = *reinterpret_cast<const VT *>(t + m);
        VT rv[CB];
#pragma unroll
        for (int c = 0; c < CB; ++c)
            rv[c] = __builtin_nontemporal_load(reinterpret_cast<const VT *>(cols[c] + m));
#pragma unroll
        for (int c = 0; c < CB; ++c)
            acc[c] += vdot(rv[c], tv);
    }
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < CB; ++c) {
        const E v = wave_sum(acc[c]);
        if (lane == 0)
            lds[w][c] = v;
    }
    __syncthreads();
    if (threadIdx.x < CB && n0 + threadIdx.x < N) {
        double s = 0.0;
        for (int i = 0; i < kBlock / 64; ++i)
            s += (double)lds[i][threadIdx.x];
        qpart[(int64_t)blockIdx.y * N + n0 + threadIdx.x] = s;
    }
}

// t_part[s][m] = sum over columns of split s of R[m, n] p[n] / |p|   (t <- R p).
// Thread: VN consecutive rows; workgroup: 256*VN rows x one column split.

template <typename E>
__global__ __launch_bounds__(kBlock) void k_gemv_n(const E *__restrict__ R, int64_t ldr, int64_t N,
                                                   const double *__restrict__ p,
                                                   int64_t cols_per_split,
                                                   double *__restrict__ tpart,
                                                   const LoopState *__restrict__ st)
{
    if (st->done)
        return;
    using VT = typename V16<E>::T;
    constexpr int VN = V16<E>::n;
    extern __shared__ unsigned char smem[];
    E *pl = reinterpret_cast<E *>(smem);
    const int64_t c0 = (int64_t)blockIdx.y * cols_per_split;
    const int64_t c1 = min(c0 + cols_per_split, N);
    const double pn = st->pnorm;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += kBlock)
        pl[c - c0] = (E)(p[c] / pn);
    __syncthreads();
    const int64_t m = ((int64_t)blockIdx.x * kBlock + threadIdx.x) * VN;
    if (m >= ldr)
        return;
    E acc[VN];
#pragma unroll
    for (int i = 0; i < VN; ++i)
        acc[i] = E(0);
    const E *base = R + m;
    int64_t c = c0;
    for (; c + 8 <= c1; c += 8) {
        VT rv[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
            rv[u] = __builtin_nontemporal_load(reinterpret_cast<const VT *>(base + (c + u) * ldr));
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const E pv = pl[c + u - c0];
            const E *e = reinterpret_cast<const E *>(&rv[u]);
#pragma unroll
            for (int i = 0; i < VN; ++i)
                acc[i] += e[i] * pv;
        }
    }
    for (; c < c1; ++c) {
        const VT rv = *reinterpret_cast<const VT *>(base + c * ldr);
        const E pv = pl[c - c0];
        const E *e = reinterpret_cast<const E *>(&rv);
#pragma unroll
        for (int i = 0; i < VN; ++i)
            acc[i] += e[i] * pv;
    }
    double *dst = tpart + (int64_t)blockIdx.y * ldr + m;
#pragma unroll
    for (int i = 0; i < VN; ++i)
        dst[i] = (double)acc[i];
}

// ---------------------------------------------------------------------------
// Gram-Schmidt, FP64.  y = sum_s part[s] (the matvec result), c = Q^T y over
// the first k columns of Q (Sec. 2.3: A <- U_(k)^T U, B <- V_(k)^T V).
// Workgroup b covers rows [256 b, 256 b + 256); its per-column partial dot
// products go to cpart[b][i]; the last workgroup sums them in block order.

template <typename E>
__global__ __launch_bounds__(kBlock) void k_gs_dot(const double *__restrict__ part, int nsplit,
                                                   int64_t ldpart, int64_t L,
                                                   const E *__restrict__ Q, int64_t ldq, int k,
                                                   double *__restrict__ y,
                                                   double *__restrict__ cpart,
                                                   double *__restrict__ c, LoopState *st,
                                                   int counter)
{
    if (st->done)
        return;
    __shared__ double ys[kBlock];
    __shared__ int last;
    const int64_t r0 = (int64_t)blockIdx.x * kBlock;
    const int64_t r = r0 + threadIdx.x;
    double v = 0.0;
    if (r < L) {
        v = sum_parts(part, nsplit, ldpart, r);
        if (y)
            y[r] = v;
    }
    ys[threadIdx.x] = v;
    __syncthreads();
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = w; i < k; i += kBlock / 64) {
        const E *q = Q + (int64_t)i * ldq;
        double s = 0.0;
        for (int j = lane; j < kBlock; j += 64)
            if (r0 + j < L)
                s += (double)q[r0 + j] * ys[j];
        s = wave_sum(s);
        if (lane == 0)
            cpart[(int64_t)blockIdx.x * k + i] = s;
    }
    if (!arrive_last(&st->counter[counter], &last))
        return;
    reduce_partials(cpart, gridDim.x, k, c, ys);
    if (threadIdx.x == 0)
        st->counter[counter] = 0;
}

// x = y - Q c (one classical Gram-Schmidt pass), squared norm; the last
// workgroup finishes the norm.  side 0 (loading): x kept in FP64 (ydst, whose
// previous content moves to yprev), |p| stored, and -- for the loading stop --
// the change of the unit loading |p_j - s p_(j-1)| (s = +-1 aligning the signs;
// infinite for the first loading of a component), summed element by element
// by the last workgroup so that it resolves changes far below sqrt(eps).
// side 1 (score): x stored
// in the element type (edst), sigma, then the stop test -- the relative sigma
// test of the host programs (Appendices 1, 3) when stop == 0, the loading
// change below tol when stop == 1, or the replayed count -- and the loop state.

template <typename E>
__global__ __launch_bounds__(kBlock) void k_gs_apply(const double *__restrict__ part, int nsplit,
                                                     int64_t ldpart, int64_t L,
                                                     const double *__restrict__ y,
                                                     const E *__restrict__ Q, int64_t ldq, int k,
                                                     const double *__restrict__ c,
                                                     double *__restrict__ ydst,
                                                     double *__restrict__ yprev,
                                                     E *__restrict__ edst,
                                                     double *__restrict__ sqpart, LoopState *st,
                                                     int side, double tol, int32_t limit,
                                                     int replay, double tiny, int stop)
{
    if (st->done)
        return;
    __shared__ double cs[1024];
    __shared__ double red[kBlock / 64];
    __shared__ int last;
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double v = 0.0;
    if (r < L) {
        if (k > 0) {
            v = y[r];
        } else {
            v = sum_parts(part, nsplit, ldpart, r);
        }
    }
    double proj = 0.0;
    for (int i0 = 0; i0 < k; i0 += 1024) {
        const int n = min(1024, k - i0);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kBlock)
            cs[i] = c[i0 + i];
        __syncthreads();
        if (r < L) {
            // eight independent sums so that the column loads overlap
            double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int i = 0;
#pragma unroll 4
            for (; i + 7 < n; i += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    a[u] += (double)Q[r + (int64_t)(i0 + i + u) * ldq] * cs[i + u];
            }
#pragma unroll 8
            for (; i < n; ++i)
                a[0] += (double)Q[r + (int64_t)(i0 + i) * ldq] * cs[i];
            proj += ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
        }
    }
    v -= proj;
    double dot_old = 0.0;
    if (r < L) {
        if (side == 0) {
            const double o = ydst[r];
            dot_old = v * o;
            yprev[r] = o;
            ydst[r] = v;
        } else {
            edst[r] = (E)v;
        }
    }
    const double sq = block_sum(r < L ? v * v : 0.0, red);
    if (threadIdx.x == 0)
        sqpart[blockIdx.x] = sq;
    if (side == 0) {
        const double dt = block_sum(dot_old, red);
        if (threadIdx.x == 0)
            sqpart[gridDim.x + blockIdx.x] = dt;
    }
    if (!arrive_last(&st->counter[side == 0 ? kCntApplyN : kCntApplyM], &last))
        return;
    double tot = 0.0, dtot = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kBlock) {
        tot += sqpart[b];
        if (side == 0)
            dtot += sqpart[gridDim.x + b];
    }
    // fixed-order final sums: per-thread strided partials, then the block tree
    tot = block_sum(tot, red);
    if (side == 0)
        dtot = block_sum(dtot, red);
    const double nrm = sqrt(tot);
    double dp = INFINITY;
    // every thread reads the state before thread 0 updates it (the barrier
    // below orders the reads of all waves before that update), so the branch
    // is taken by all threads or by none
    const int iter0 = st->iter;
    const double pn_old = st->pnorm;
    __syncthreads();
    if (side == 0 && stop == 1 && iter0 > 0 && nrm > 0.0 && pn_old > 0.0) {
        // |p/|p| - s q/|q||^2 over the whole vector (fixed order, this workgroup)
        const double a = 1.0 / nrm, bq = (dtot >= 0.0 ? 1.0 : -1.0) / pn_old;
        double ss = 0.0;
        for (int64_t i = threadIdx.x; i < L; i += kBlock) {
            const double dd = ydst[i] * a - yprev[i] * bq;
            ss += dd * dd;
        }
        dp = sqrt(block_sum(ss, red));
    }
    if (threadIdx.x != 0)
        return;
    st->counter[side == 0 ? kCntApplyN : kCntApplyM] = 0;
    if (side == 0) {
        st->dp = dp;
        st->pnorm = nrm;
        if (!(nrm >= tiny)) { // counts as the iteration in which it happened
            st->iter = st->iter + 1;
            st->degenerate = 1;
            st->done = 1;
        }
        return;
    }
    score_test(st, nrm, tol, limit, replay, tiny, stop);
}

// First pass of the doubled classical form (CGS2): y <- y - Q c in place
// (FP64), c = Q^T y from gs_dot; the second pass is gs_dot + gs_apply on y.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_gs_project(double *__restrict__ y, int64_t L,
                                                       const E *__restrict__ Q, int64_t ldq,
                                                       int k, const double *__restrict__ c,
                                                       const LoopState *st)
{
    if (st->done)
        return;
    __shared__ double cs[1024];
    const int64_t r = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double proj = 0.0;
    for (int i0 = 0; i0 < k; i0 += 1024) {
        const int n = min(1024, k - i0);
        __syncthreads();
        for (int i = threadIdx.x; i < n; i += kBlock)
            cs[i] = c[i0 + i];
        __syncthreads();
        if (r < L)
            for (int i = 0; i < n; ++i)
                proj += (double)Q[r + (int64_t)(i0 + i) * ldq] * cs[i];
    }
    if (r < L)
        y[r] -= proj;
}

// Modified Gram-Schmidt (the MGS form of the step), one workgroup: y = sum of
// the nsplit partial vectors, then for i = 0 .. k-1 in order c_i = q_i^T y
// and y <- y - c_i q_i, each coefficient from the vector already reduced by
// the earlier columns.  Every thread owns the entries r = tid + 1024 j, so y
// needs no barrier; each coefficient is a fixed-order workgroup sum (wave
// butterflies, then the 16 waves in order), and the update by column i is
// fused with the dot product for column i + 1.
constexpr int kMgsThreads = 1024;
template <typename E>
__global__ __launch_bounds__(kMgsThreads) void k_mgs(const double *__restrict__ part, int nsplit,
                                                     int64_t ldpart, int64_t L,
                                                     const E *__restrict__ Q, int64_t ldq, int k,
                                                     double *__restrict__ y, const LoopState *st)
{
    if (st->done)
        return;
    constexpr int NW = kMgsThreads / 64;
    __shared__ double red[NW];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    double acc = 0.0;
    for (int64_t r = tid; r < L; r += kMgsThreads) {
        double v = 0.0;
        v = sum_parts(part, nsplit, ldpart, r);
        y[r] = v;
        acc += (double)Q[r] * v; // column 0
    }
    for (int i = 0; i < k; ++i) {
        const double ws = wave_sum(acc);
        __syncthreads(); // the previous coefficient has been read by every thread
        if (lane == 0)
            red[w] = ws;
        __syncthreads();
        double ci = 0.0;
        for (int q = 0; q < NW; ++q)
            ci += red[q];
        const E *qi = Q + (int64_t)i * ldq;
        const E *qn = Q + (int64_t)(i + 1 < k ? i + 1 : i) * ldq;
        const bool more = i + 1 < k;
        acc = 0.0;
        for (int64_t r = tid; r < L; r += kMgsThreads) {
            const double v = y[r] - (double)qi[r] * ci;
            y[r] = v;
            if (more)
                acc += (double)qn[r] * v;
        }
    }
}

// Degenerate component: the first unit vector whose Gram-Schmidt residual
// against P_(k) has squared norm >= (N-k)/(2N), normalised, into p (FP64).
// Rare path: one workgroup, candidates tried in ascending order.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_degenerate_p(const E *__restrict__ P, int64_t N, int k,
                                                         double *__restrict__ p, LoopState *st)
{
    __shared__ double red[kBlock / 64];
    const double thresh = (double)(N - k) / (2.0 * (double)N);
    for (int64_t i = 0; i < N; ++i) {
        // r = e_i - P c with c = P^T e_i = P[i, :k]
        double sq = 0.0;
        for (int64_t n = threadIdx.x; n < N; n += kBlock) {
            double s = 0.0;
            for (int j = 0; j < k; ++j)
                s += (double)P[n + (int64_t)j * N] * (double)P[i + (int64_t)j * N];
            const double rv = (n == i ? 1.0 : 0.0) - s;
            p[n] = rv;
            sq += rv * rv;
        }
        sq = block_sum(sq, red);
        if (sq >= thresh) {
            if (threadIdx.x == 0)
                st->pnorm = sqrt(sq);
            return;
        }
    }
}

// Finish component k: V[:,k] = t / sigma (GS) or T[:,k] = t (NIPALS),
// P[:,k] = p / |p|; degenerate components get t = 0, sigma = 0.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_finalize_comp(const E *__restrict__ t, int64_t M,
                                                          int64_t N, const double *__restrict__ p,
                                                          int k, int gs, E *__restrict__ T,
                                                          E *__restrict__ P, double *sigma,
                                                          int32_t *iters, int32_t *start_col,
                                                          LoopState *st)
{
    const int deg = st->degenerate;
    const double s = st->sigma, pn = st->pnorm;
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < M)
        T[i + (int64_t)k * M] = deg ? E(0) : (gs ? (E)((double)t[i] / s) : t[i]);
    if (i < N)
        P[i + (int64_t)k * N] = (E)(p[i] / pn);
    if (i == 0) {
        sigma[k] = deg ? 0.0 : s;
        if (iters)
            iters[k] = st->iter;
        if (start_col)
            start_col[k] = st->start_col;
    }
}

// Explicit deflation R <- R - t p^T (eq. 3; Sec. 2.3 with t = lambda_k v) and the
// squared column norms of the new residual.  One wave per column.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_deflate(E *__restrict__ R, int64_t ldr, int64_t M,
                                                    int64_t N, const E *__restrict__ t,
                                                    const E *__restrict__ pk, double *cn)
{
    using VT = typename V16<E>::T;
    constexpr int VN = V16<E>::n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t n = (int64_t)blockIdx.x * 4 + w;
    if (n >= N)
        return;
    const E pn = pk[n];
    E *col = R + n * ldr;
    double s = 0.0;
    for (int64_t m = (int64_t)lane * VN; m < ldr; m += 64 * VN) {
        VT rv = *reinterpret_cast<const VT *>(col + m);
        const VT tv = *reinterpret_cast<const VT *>(t + m);
        E *re = reinterpret_cast<E *>(&rv);
        const E *te = reinterpret_cast<const E *>(&tv);
#pragma unroll
        for (int i = 0; i < VN; ++i) {
            re[i] = re[i] - te[i] * pn;
            s += (double)re[i] * (double)re[i];
        }
        *reinterpret_cast<VT *>(col + m) = rv;
    }
    s = wave_sum(s);
    if (lane == 0)
        cn[n] = s;
}

// T <- V Lambda (GS) and lambda = sigma^2.
template <typename E>
__global__ __launch_bounds__(kBlock) void k_finalize_all(E *__restrict__ T, int64_t M, int K,
                                                         const double *__restrict__ sigma,
                                                         double *lambda, double *sigma_out, int gs)
{
    for (int k = blockIdx.y; k < K; k += gridDim.y) {
        const double s = sigma[k];
        if (gs)
            for (int64_t m = (int64_t)blockIdx.x * kBlock + threadIdx.x; m < M;
                 m += (int64_t)gridDim.x * kBlock)
                T[m + (int64_t)k * M] = (E)((double)T[m + (int64_t)k * M] * s);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            lambda[k] = s * s;
            if (sigma_out)
                sigma_out[k] = s;
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers.

static inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
static inline int64_t hmin(int64_t a, int64_t b) { return a < b ? a : b; }

template <typename E>
void Launch<E>::copy_pad(const E *X, int64_t ldx, E *R, int64_t ldr, int64_t M, int64_t N,
                         LoopState *st, hipStream_t s)
{
    dim3 g(hmin(ceil_div(ldr, kBlock), 64), (unsigned)hmin(N, 4096));
    hipLaunchKernelGGL(k_copy_pad<E>, g, dim3(kBlock), 0, s, X, ldx, R, ldr, M, N, st);
}

template <typename E>
void Launch<E>::colnorm(const E *R, int64_t ldr, int64_t M, int64_t N, double *cn, hipStream_t s)
{
    hipLaunchKernelGGL(k_colnorm<E>, dim3(hmin(ceil_div(N, 4), 65535)), dim3(kBlock), 0, s,
                       R, ldr, M, N, cn);
}

template <typename E>
void Launch<E>::start(const E *R, int64_t ldr, int64_t M, int64_t N, const double *cn,
                      const E *V, const E *T0, StartArgs a, double tiny, E *t, LoopState *st,
                      hipStream_t s)
{
    hipLaunchKernelGGL(k_start<E>, dim3(1), dim3(1024), 0, s, R, ldr, M, N, cn, V, T0, a, tiny, t,
                       st);
}

template <typename E>
void Launch<E>::gemv_t(const E *R, int64_t ldr, int64_t N, const E *t, int64_t rows_per_split,
                       int nsplit, int ncolblk, double *qpart, const LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL((k_gemv_t<E, 8>), dim3(ncolblk, nsplit), dim3(kBlock), 0, s, R, ldr, N, t,
                       rows_per_split, qpart, st);
}

template <typename E>
void Launch<E>::gemv_n(const E *R, int64_t ldr, int64_t N, const double *p, int64_t cols_per_split,
                       int nsplit, double *tpart, const LoopState *st, hipStream_t s)
{
    constexpr int VN = V16<E>::n;
    dim3 g(ceil_div(ldr, (int64_t)kBlock * VN), nsplit);
    hipLaunchKernelGGL(k_gemv_n<E>, g, dim3(kBlock), cols_per_split * sizeof(E), s, R, ldr, N, p,
                       cols_per_split, tpart, st);
}

template <typename E>
void Launch<E>::gs_dot(const double *part, int nsplit, int64_t ldpart, int64_t L, const E *Q,
                       int64_t ldq, int k, double *y, double *cpart, double *c, LoopState *st,
                       int counter, hipStream_t s)
{
    hipLaunchKernelGGL(k_gs_dot<E>, dim3(ceil_div(L, kBlock)), dim3(kBlock), 0, s, part, nsplit,
                       ldpart, L, Q, ldq, k, y, cpart, c, st, counter);
}

template <typename E>
void Launch<E>::gs_apply(const double *part, int nsplit, int64_t ldpart, int64_t L,
                         const double *y, const E *Q, int64_t ldq, int k, const double *c,
                         double *ydst, double *yprev, E *edst, double *sqpart, LoopState *st,
                         int side, double tol, int32_t limit, int replay, double tiny, int stop,
                         hipStream_t s)
{
    hipLaunchKernelGGL(k_gs_apply<E>, dim3(ceil_div(L, kBlock)), dim3(kBlock), 0, s, part, nsplit,
                       ldpart, L, y, Q, ldq, k, c, ydst, yprev, edst, sqpart, st, side, tol, limit,
                       replay, tiny, stop);
}

template <typename E>
void Launch<E>::gs_project(double *y, int64_t L, const E *Q, int64_t ldq, int k, const double *c,
                           LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_gs_project<E>, dim3(ceil_div(L, kBlock)), dim3(kBlock), 0, s, y, L, Q,
                       ldq, k, c, st);
}

template <typename E>
void Launch<E>::mgs(const double *part, int nsplit, int64_t ldpart, int64_t L, const E *Q,
                    int64_t ldq, int k, double *y, LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_mgs<E>, dim3(1), dim3(kMgsThreads), 0, s, part, nsplit, ldpart, L, Q, ldq,
                       k, y, st);
}

template <typename E>
void Launch<E>::degenerate_p(const E *P, int64_t N, int k, double *p, LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_degenerate_p<E>, dim3(1), dim3(kBlock), 0, s, P, N, k, p, st);
}

template <typename E>
void Launch<E>::finalize_comp(const E *t, int64_t M, int64_t N, const double *p, int k, int gs,
                              E *T, E *P, double *sigma, int32_t *iters, int32_t *start_col,
                              LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_finalize_comp<E>, dim3(ceil_div(M > N ? M : N, kBlock)), dim3(kBlock), 0,
                       s, t, M, N, p, k, gs, T, P, sigma, iters, start_col, st);
}

template <typename E>
void Launch<E>::deflate(E *R, int64_t ldr, int64_t M, int64_t N, const E *t, const E *pk,
                        double *cn, hipStream_t s)
{
    hipLaunchKernelGGL(k_deflate<E>, dim3(ceil_div(N, 4)), dim3(kBlock), 0, s, R, ldr, M, N, t, pk,
                       cn);
}

template <typename E>
void Launch<E>::finalize_all(E *T, int64_t M, int K, const double *sigma, double *lambda,
                             double *sigma_out, int gs, hipStream_t s)
{
    dim3 g(hmin(ceil_div(M, kBlock), 256), hmin(K, 65535));
    hipLaunchKernelGGL(k_finalize_all<E>, g, dim3(kBlock), 0, s, T, M, K, sigma, lambda,
                       sigma_out, gs);
}

template struct Launch<float>;
template struct Launch<double>;

__global__ void k_state_reset(LoopState *st) { *st = LoopState{}; }

void reset_state(LoopState *st, hipStream_t s)
{
    hipLaunchKernelGGL(k_state_reset, dim3(1), dim3(1), 0, s, st);
}

int stream_capturing(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess)
        return -1;
    return cs == hipStreamCaptureStatusNone ? 0 : 1;
}

}  // namespace gspca
