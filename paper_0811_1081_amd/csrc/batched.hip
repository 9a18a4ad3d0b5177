// batched.hip -- many independent GS-PCA problems (Andrecut, arXiv:0811.1081,
// Sec. 2.3) in one persistent launch.
//
// One workgroup fits one problem at a time, from its first start vector to its
// last component, with only workgroup barriers: no grid-wide synchronisation
// and no host round-trips.  Workgroups take problems from a device-side queue
// (an atomic counter over a descriptor table the host sorted largest-first)
// until it is empty, so the launch balances uneven sizes by itself and every
// workgroup reaches the exit.  The launch contains no host synchronisation and
// can be captured in a hipGraph and replayed; the queue counter is reset by a
// one-thread kernel, not a memset.
//
// Per iteration (FP32 data, FP64 Gram-Schmidt and norms, implicit deflation
// R = X - T P^T on Gram-Schmidt-projected vectors):
//   t = X p, q = X^T t      one read of X (batch_pass): two tiles of rows
//                           are held in registers while their t is summed
//                           across the waves, then multiplied back into q
//   d = V_(k)^T t           batch_tpass over the columns of V
//   t <- t - V d, sigma = |t|, stop test (relative sigma, loading, replay)
//   q <- q - W d            W = X^T V_(k), so q = X^T (t - V d)
//   c = P_(k)^T q (batch_tpass), p = q - P c, p / |p| (and its FP32 copy)
// Per component: the first loading q = X^T t0 and W's column X^T v_k, and per
// problem the column norms, also run on batch_tpass.  t, q, p, the column
// norms and the coefficient vectors live in LDS.  A problem with more than 64
// columns per wave reads X twice instead (t = X p with threads over rows, then
// q = X^T t on batch_tpass).
#include <float.h>
#include <math.h>

#include "internal.h"
#include "panel.h"

namespace gspca {

// Workgroup sum; every thread gets the result.  `red` holds one slot per wave.
__device__ inline double bblock_sum(double v, double *red)
{
    v = fwave_sum(v);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
        red[w] = v;
    __syncthreads();
    double r = 0.0;
    for (int i = 0; i < nw; ++i)
        r += red[i];
    return r;
}

// Two workgroup sums for one pair of barriers (`red` holds two slots per wave).
__device__ inline void bblock_sum2(double a, double b, double *red, double &ra, double &rb)
{
    a = fwave_sum(a);
    b = fwave_sum(b);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        red[w] = a;
        red[16 + w] = b;
    }
    __syncthreads();
    ra = 0.0;
    rb = 0.0;
    for (int i = 0; i < nw; ++i) {
        ra += red[i];
        rb += red[16 + i];
    }
}

// LDS floats (at the start of the dynamic LDS) for the cross-wave sums of
// batch_pass: two buffers of two values per thread of a 1024-thread
// workgroup (two row tiles per step).
constexpr int kPassLdsFloats = 2 * 2 * 1024;

// Column split of the single pass: CW waves share the columns of a row tile,
// CPW (a power of two, 4..64) columns per wave, at most 32 while the
// workgroup has waves to spare; 0 when N needs more than 64 columns per wave
// or X's byte offsets do not fit 31 bits.
__device__ inline void pass_split(int N, int64_t ldx, int nw, int &CW, int &CPW)
{
    int cw = 1;
    while (cw * 32 < N && cw < nw)
        cw <<= 1;
    if (cw * 64 < N || ldx * (int64_t)N >= ((int64_t)1 << 29)) {
        CW = 0;
        CPW = 0;
        return;
    }
    const int per = (N + cw - 1) / cw;
    int c = 4;
    while (c < per)
        c <<= 1;
    CW = cw;
    CPW = c;
}

// t = X p and q = X^T t from one read of X (Sec. 2.3's two products).  The
// waves form CW column groups x RS row groups; a tile is 64 RS rows: lane l
// of row group r takes row 64 r + l and CPW consecutive columns of its column
// group (coalesced 256-byte loads down each column), forms its share of t in
// FP32, the CW shares of a row are added in FP64 through LDS (fixed order),
// and the same registers then give the row's terms of q = X^T t, summed over
// the wave's 64 rows with a reduce-scatter; each lane keeps the FP64 running
// sum of one column.  Rows past M are read clamped and weigh 0; columns past
// N are read clamped and meet p = 0 (pf is zero-padded) and are dropped.
// t and q are written to LDS.  With AHEAD the next tile's loads are issued
// before the workgroup barrier of the current one (a second set of CPW
// registers), so they are in flight while the waves wait and form their q
// terms; only the kernel built for at most 8 waves per compute unit (256
// registers) does this: under the 128-register bound of 16 waves the
// compiler spills inside the tile loop and the reload waits for the
// prefetch (121.6 vs 114.0 ms per replay of the 2048-problem batch).
template <int CPW, int TP, bool AHEAD>
__device__ void batch_pass(const float *X, int64_t ldx, int M, int N, int CW,
                           const float *pf, float *xr, double *t, double *q)
{
    const int tid = threadIdx.x, lane = tid & 63, NT = blockDim.x;
    const int nw = NT >> 6;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int cw = w % CW, rs = w / CW, RS = nw / CW;
    // a wave's columns may lie wholly past N (then it contributes zeros)
    const int cbase = cw * CPW;
    const int ld = (int)ldx;
    // buffer loads: the column's byte offset is a scalar operand, the row's
    // a per-lane one (X spans less than 2 GiB: pass_split)
    const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)X, (short)0, (int)(((int64_t)(N - 1) * ldx + M) * 4), 0x00020000);
    // the wave's p values
    float pv[CPW];
#pragma unroll
    for (int c = 0; c < CPW; ++c)
        pv[c] = pf[cbase + c];
    const int tile = 64 * RS, step = TP * tile;
    // TP tiles of 64 RS rows per step: sub-tile u of the wave is rows
    // m0 + u tile + 64 rs + [0, 64); its loads are issued together, so each
    // column is read in runs of TP * 256 bytes
    auto load = [&](float (&x)[TP][CPW], int m0) {
#pragma unroll
        for (int u = 0; u < TP; ++u) {
            const int row = m0 + u * tile + rs * 64 + lane;
            const int rowb = (row < M ? row : M - 1) * 4;
#pragma unroll
            for (int c = 0; c < CPW; ++c) {
                const int col = cbase + c < N ? cbase + c : N - 1;
                x[u][c] = __uint_as_float(
                    __builtin_amdgcn_raw_buffer_load_b32(xs, rowb, col * ld * 4, 0));
            }
        }
    };
    double qacc = 0.0;
    int slot = 0;
    int buf = 0;
    // one step: t partials of the TP tiles, the cross-wave sums (one
    // barrier), then the q terms of both tiles in one reduce-scatter
    auto body = [&](float (&x)[TP][CPW], float (&xn)[TP][CPW], int m0) {
        float *red = xr + buf * (TP * 1024);
#pragma unroll
        for (int u = 0; u < TP; ++u) {
            float ta = 0.f, tb = 0.f;
#pragma unroll
            for (int c = 0; c < CPW; c += 2) {
                ta += x[u][c] * pv[c];
                tb += x[u][c + 1] * pv[c + 1];
            }
            red[u * 1024 + cw * tile + rs * 64 + lane] = ta + tb;
        }
        if constexpr (AHEAD) {
            if (m0 + step < M)
                load(xn, m0 + step);
        }
        __syncthreads();
        float tf[TP];
#pragma unroll
        for (int u = 0; u < TP; ++u) {
            // the CW shares in order, four reads in flight at a time
            const float *rp = red + u * 1024 + rs * 64 + lane;
            double tv = 0.0;
            if (CW >= 4) {
                for (int g = 0; g < CW; g += 4) {
                    const float r0 = rp[g * tile], r1 = rp[(g + 1) * tile];
                    const float r2 = rp[(g + 2) * tile], r3 = rp[(g + 3) * tile];
                    tv += (double)r0;
                    tv += (double)r1;
                    tv += (double)r2;
                    tv += (double)r3;
                }
            } else {
                for (int g = 0; g < CW; ++g)
                    tv += (double)rp[g * tile];
            }
            const int row = m0 + u * tile + rs * 64 + lane;
            if (row >= M)
                tv = 0.0;
            else if (cw == 0)
                t[row] = tv;
            tf[u] = (float)tv;
        }
#pragma unroll
        for (int c = 0; c < CPW; ++c) {
            float y = x[0][c] * tf[0];
#pragma unroll
            for (int u = 1; u < TP; ++u)
                y += x[u][c] * tf[u];
            x[0][c] = y;
        }
        qacc += (double)wave_scatter_sum<float, CPW>(x[0], lane, slot);
        buf ^= 1;
    };
    float xa[TP][CPW];
    if constexpr (AHEAD) {
        float xb[TP][CPW];
        load(xa, 0);
        for (int m0 = 0; m0 < M; m0 += 2 * step) {
            body(xa, xb, m0);
            if (m0 + step < M)
                body(xb, xa, m0 + step);
        }
    } else {
        for (int m0 = 0; m0 < M; m0 += step) {
            load(xa, m0);
            body(xa, xa, m0);
        }
    }
    // q: the row groups' sums of each column, in order (the buffers are free
    // once every wave has passed this barrier)
    __syncthreads();
    double *qr = reinterpret_cast<double *>(xr);
    const int width = CW * CPW;
    if ((lane & (64 / CPW - 1)) == 0 && cbase + slot < N)
        qr[rs * width + cbase + slot] = qacc;
    __syncthreads();
    for (int j = tid; j < N; j += NT) {
        double v = 0.0;
        for (int r = 0; r < RS; ++r)
            v += qr[r * width + j];
        q[j] = v;
    }
}

// out_j = X_j . v for every column (v in LDS, FP64), or with SQ the squared
// column norms |X_j|^2 -- the products of the first loading (q = X^T t0), of
// W (X^T v_k) and of the column norms, and with X = V_(k) or P_(k) the
// Gram-Schmidt coefficients d = V^T t and c = P^T q.  Waves take chunks of CC = 8 columns
// with the lanes over rows (the buffer loads and 256-byte column segments of
// batch_pass), keep FP64 per-lane sums of their columns over the rows they
// visit, TI = 4 row tiles (1 KiB of each column) in flight, and finish a
// chunk with one reduce-scatter: no workgroup barrier inside, unlike
// batch_pass (whose t sums need one per tile).  With fewer chunks than
// waves, RP waves share a chunk by interleaved row tiles and their sums are
// added in LDS (scr, RP x CC x chunks doubles) in a fixed order.  Rows and
// columns out of range are read clamped; such rows weigh 0 and such columns
// are not written.
template <bool SQ>
__device__ void batch_tpass(const float *X, int64_t ldx, int M, int N, const double *v,
                            double *scr, double *out)
{
    constexpr int CC = 8, TI = 4;
    const int tid = threadIdx.x, lane = tid & 63, NT = blockDim.x;
    const int nw = NT >> 6;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nch = (N + CC - 1) / CC;
    int RP = 1;
    while (RP * 2 * nch <= nw)
        RP <<= 1;
    const int rpart = w % RP, cstep = nw / RP, rstep = 64 * RP;
    const int ld = (int)ldx;
    const __amdgpu_buffer_rsrc_t xs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)X, (short)0, (int)(((int64_t)(N - 1) * ldx + M) * 4), 0x00020000);
    for (int ch = w / RP; ch < nch; ch += cstep) {
        const int cbase = ch * CC;
        double acc[CC];
#pragma unroll
        for (int c = 0; c < CC; ++c)
            acc[c] = 0.0;
        for (int m0 = rpart * 64; m0 < M; m0 += TI * rstep) {
            float x[TI][CC];
#pragma unroll
            for (int u = 0; u < TI; ++u) {
                const int row = m0 + u * rstep + lane;
                const int rowb = (row < M ? row : M - 1) * 4;
#pragma unroll
                for (int c = 0; c < CC; ++c) {
                    const int col = cbase + c < N ? cbase + c : N - 1;
                    x[u][c] = __uint_as_float(
                        __builtin_amdgcn_raw_buffer_load_b32(xs, rowb, col * ld * 4, 0));
                }
            }
#pragma unroll
            for (int u = 0; u < TI; ++u) {
                const int row = m0 + u * rstep + lane;
                const double wt = row < M ? (SQ ? 1.0 : v[row]) : 0.0;
#pragma unroll
                for (int c = 0; c < CC; ++c) {
                    const double a = (double)x[u][c];
                    acc[c] += (SQ ? a : 1.0) * a * wt;
                }
            }
        }
        int slot;
        const double sum = wave_scatter_sum<double, CC>(acc, lane, slot);
        if ((lane & (64 / CC - 1)) == 0 && cbase + slot < N) {
            if (RP == 1)
                out[cbase + slot] = sum;
            else
                scr[rpart * nch * CC + cbase + slot] = sum;
        }
    }
    if (RP > 1) {
        __syncthreads();
        for (int j = tid; j < N; j += NT) {
            double s = 0.0;
            for (int r = 0; r < RP; ++r)
                s += scr[r * nch * CC + j];
            out[j] = s;
        }
    }
}

__global__ void k_batch_reset(uint32_t *counter) { *counter = 0u; }

// MAXT: the most threads per compute unit the build serves (1024: 128
// registers per lane; 512: 256 registers, and the single pass prefetches the
// next two tiles up to 32 columns per wave).  The single pass takes two row
// tiles per step except with 64 columns per wave in the 128-register build.
template <int MAXT>
__global__ __launch_bounds__(MAXT) void k_batched(const BatchItem *__restrict__ items, int nprob,
                                                  const int32_t *__restrict__ order,
                                                  uint32_t *__restrict__ queue, BatchArgs a)
{
    constexpr bool kAhead = MAXT <= 512;
    extern __shared__ double lds[];
    __shared__ double red[32];
    __shared__ int cur, bad;
    __shared__ int64_t sel, selmax;
    __shared__ double sred[16];
    __shared__ int64_t ired[16];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int NT = blockDim.x, nw = NT >> 6;

    for (;;) {
        if (tid == 0) {
            const uint32_t i = atomicAdd(queue, 1u);
            cur = i < (uint32_t)nprob ? order[i] : -1;
        }
        __syncthreads();
        // uniform values read from LDS go to scalar registers
        const int pi = __builtin_amdgcn_readfirstlane(cur);
        __syncthreads();
        if (pi < 0)
            return;
        const BatchItem it = items[pi];
        const int M = it.M, N = it.N, K = it.K;
        const int64_t ldx = it.ldx;
        const float *X = it.X;
        float *T = it.T, *P = it.P;
        double *W = it.W; // N x K: X^T v_i of finished components
        // LDS: pass buffers | pf[npf] (float, zero past N) | t[M] | q[N] | p[N]
        //      | pprev[N] | cn0[N] | sig[K] | dc[K]
        float *xr = reinterpret_cast<float *>(lds);
        float *pf = xr + kPassLdsFloats;
        const int npf = batched_pf_floats(N);
        double *t = reinterpret_cast<double *>(pf + npf);
        double *q = t + M;
        double *p = q + N;
        double *pprev = p + N;
        double *cn0 = pprev + N;
        double *sig = cn0 + N;
        double *dc = sig + K;

        // pf past N stays zero for the whole problem (the single pass's
        // column groups may reach past N)
        for (int j = N + tid; j < npf; j += NT)
            pf[j] = 0.f;
        // |X_j|^2: waves over columns, lanes over rows; NaN/Inf ends the problem
        if (tid == 0)
            bad = 0;
        __syncthreads();
        batch_tpass<true>(X, ldx, M, N, nullptr, reinterpret_cast<double *>(xr), cn0);
        __syncthreads();
        for (int j = tid; j < N; j += NT)
            if (!isfinite(cn0[j]))
                bad = 1;
        __syncthreads();
        if (bad) {
            if (tid == 0 && it.status)
                *it.status = -4;
            __syncthreads();
            continue;
        }
        int not_conv = 0;
        int CW = 0, CPW = 0;
        pass_split(N, ldx, nw, CW, CPW);

        for (int k = 0; k < K; ++k) {
            const int32_t limit = it.replay_iters ? it.replay_iters[k] : a.max_iter;
            // ---- start column: the largest residual column norm (ties to the
            //      lowest index), |X_j|^2 - 2 sum_i s_i P_ji (X^T v_i)_j
            //      + sum_i s_i^2 P_ji^2; replayed column or column k when asked
            double best = -1.0;
            int64_t bi = 0;
            for (int j = tid; j < N; j += NT) {
                double s = cn0[j];
                for (int i = 0; i < k; ++i) {
                    const double pji = (double)P[j + (int64_t)i * N];
                    s += -2.0 * sig[i] * pji * W[j + (int64_t)i * N] + sig[i] * sig[i] * pji * pji;
                }
                s = s < 0.0 ? 0.0 : s;
                q[j] = s;
                if (s > best) { best = s; bi = j; }
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ov = __shfl_xor(best, o, 64);
                const int64_t oi = __shfl_xor(bi, o, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if (lane == 0) { sred[w] = best; ired[w] = bi; }
            __syncthreads();
            if (tid == 0) {
                double b = sred[0];
                int64_t i0 = ired[0];
                for (int i = 1; i < nw; ++i)
                    if (sred[i] > b || (sred[i] == b && ired[i] < i0)) { b = sred[i]; i0 = ired[i]; }
                selmax = i0;
                const bool replayed =
                    it.replay_start && it.replay_start[k] >= 0 && it.replay_start[k] < N;
                if (replayed)
                    i0 = it.replay_start[k];
                else if (a.init == 1 && sqrt(q[k]) >= a.tiny)
                    i0 = k;
                else if (a.init == 2 && it.T0)
                    i0 = -1; // given vector, if it passes the test below
                sel = i0;
            }
            __syncthreads();
            if (sel < 0) {
                // Given start: keep it if its norm is at least tiny and finite
                // and more than a tenth of it lies outside span(V_(k))
                // (|g|^2 - sum_i (v_i . g)^2, V orthonormal); else the
                // largest residual column.
                const float *g0 = it.T0 + (int64_t)k * M;
                double gg = 0.0;
                for (int m = tid; m < M; m += NT)
                    gg += (double)g0[m] * (double)g0[m];
                gg = bblock_sum(gg, red);
                double dd = 0.0;
                for (int i = 0; i < k; ++i) {
                    double d = 0.0;
                    for (int m = tid; m < M; m += NT)
                        d += (double)T[m + (int64_t)i * M] * (double)g0[m];
                    d = bblock_sum(d, red);
                    dd += d * d;
                }
                if (tid == 0 && !(sqrt(gg) >= a.tiny && isfinite(gg) && gg - dd >= 0.01 * gg))
                    sel = selmax;
                __syncthreads();
            }
            const int64_t c0 = (int64_t)__builtin_amdgcn_readfirstlane((int)sel);
            // t0 = X_c - sum_i s_i v_i P_ci, or the given vector
            double ss = 0.0;
            for (int m = tid; m < M; m += NT) {
                double v;
                if (c0 >= 0) {
                    v = (double)X[m + c0 * ldx];
                    for (int i = 0; i < k; ++i)
                        v -= sig[i] * (double)T[m + (int64_t)i * M] *
                             (double)P[c0 + (int64_t)i * N];
                } else {
                    v = (double)it.T0[m + (int64_t)k * M];
                }
                t[m] = v;
                ss += v * v;
            }
            const double t0n = sqrt(bblock_sum(ss, red));
            int degenerate = !(t0n >= a.tiny) || limit < 1;
            double s_cur = 0.0, mu = 0.0, pn = 1.0, dp = INFINITY;
            int iters = 0, conv = 0;

            // loading from t: q = X^T t, one GS pass, norm (Sec. 2.3).  After
            // a single pass q holds X^T t for the t before its Gram-Schmidt
            // step, and q - W d is X^T of the projected t.
            auto loading = [&](int first, int from_pass) -> bool {
                __syncthreads();
                if (!from_pass) {
                    batch_tpass<false>(X, ldx, M, N, t, reinterpret_cast<double *>(xr), q);
                } else if (k > 0) {
                    for (int j = tid; j < N; j += NT) {
                        double wd = 0.0;
                        for (int i = 0; i < k; ++i)
                            wd += W[j + (int64_t)i * N] * dc[i];
                        q[j] -= wd;
                    }
                }
                __syncthreads();
                if (k > 0)
                    batch_tpass<false>(P, N, N, k, q, reinterpret_cast<double *>(xr), dc);
                __syncthreads();
                double s2 = 0.0, dt = 0.0;
                for (int j = tid; j < N; j += NT) {
                    double v = q[j];
                    double pr = 0.0;
                    for (int i = 0; i < k; ++i)
                        pr += (double)P[j + (int64_t)i * N] * dc[i];
                    v -= pr;
                    pprev[j] = p[j];
                    p[j] = v;
                    s2 += v * v;
                    dt += v * pprev[j];
                }
                double nrm, dot;
                bblock_sum2(s2, dt, red, nrm, dot);
                nrm = sqrt(nrm);
                if (!(nrm >= a.tiny))
                    return false;
                // FP32 copy of p / |p| for the pass (each thread its own j, as
                // written above; the barrier at the top of the iteration
                // publishes it)
                for (int j = tid; j < N; j += NT)
                    pf[j] = (float)(p[j] / nrm);
                dp = INFINITY;
                if (!first && a.stop == 1) {
                    const double ia = 1.0 / nrm, ib = (dot >= 0.0 ? 1.0 : -1.0) / pn;
                    double dd = 0.0;
                    for (int j = tid; j < N; j += NT) {
                        const double e = p[j] * ia - pprev[j] * ib;
                        dd += e * e;
                    }
                    dp = sqrt(bblock_sum(dd, red));
                }
                pn = nrm;
                return true;
            };

            if (!degenerate) {
                if (!loading(1, 0)) {
                    degenerate = 1;
                    iters = 1;
                }
            }
            while (!degenerate && iters < limit) {
                ++iters;
                // t = X p / |p| (pf, written by the loading)
                __syncthreads();
                switch (CPW) {
                case 4: batch_pass<4, 2, kAhead>(X, ldx, M, N, CW, pf, xr, t, q); break;
                case 8: batch_pass<8, 2, kAhead>(X, ldx, M, N, CW, pf, xr, t, q); break;
                case 16: batch_pass<16, 2, kAhead>(X, ldx, M, N, CW, pf, xr, t, q); break;
                case 32: batch_pass<32, 2, kAhead>(X, ldx, M, N, CW, pf, xr, t, q); break;
                case 64: batch_pass<64, kAhead ? 2 : 1, false>(X, ldx, M, N, CW, pf, xr, t, q); break;
                default: break;
                }
                for (int m = CPW ? M : tid; m < M; m += NT) {
                    // sixteen columns per step, all loads issued before use
                    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
                    const float *xr = X + m;
                    int j = 0;
                    for (; j + 16 <= N; j += 16) {
                        float x[16];
#pragma unroll
                        for (int u = 0; u < 16; ++u)
                            x[u] = xr[(int64_t)(j + u) * ldx];
#pragma unroll
                        for (int u = 0; u < 16; u += 4) {
                            a0 += x[u] * pf[j + u];
                            a1 += x[u + 1] * pf[j + u + 1];
                            a2 += x[u + 2] * pf[j + u + 2];
                            a3 += x[u + 3] * pf[j + u + 3];
                        }
                    }
                    for (; j < N; ++j)
                        a0 += xr[(int64_t)j * ldx] * pf[j];
                    t[m] = (double)((a0 + a1) + (a2 + a3));
                }
                __syncthreads();
                // d = V^T t, t <- t - V d, sigma
                if (k > 0)
                    batch_tpass<false>(T, M, M, k, t, reinterpret_cast<double *>(xr), dc);
                __syncthreads();
                double s2 = 0.0;
                for (int m = tid; m < M; m += NT) {
                    double v = t[m];
                    double pr = 0.0;
                    for (int i = 0; i < k; ++i)
                        pr += (double)T[m + (int64_t)i * M] * dc[i];
                    v -= pr;
                    t[m] = v;
                    s2 += v * v;
                }
                s_cur = sqrt(bblock_sum(s2, red));
                if (!(s_cur >= a.tiny)) {
                    degenerate = 1;
                    break;
                }
                if (!it.replay_iters) {
                    const bool pass_test = a.stop == 1 ? (dp < a.tol)
                                                       : (fabs(mu - s_cur) < a.tol * s_cur);
                    if (pass_test) {
                        conv = 1;
                        break;
                    }
                    mu = s_cur;
                }
                if (iters >= limit)
                    break;
                if (!loading(0, CPW != 0)) {
                    degenerate = 1;
                    ++iters;
                    break;
                }
            }
            if (!degenerate && !conv && !it.replay_iters)
                not_conv = 1;
            __syncthreads();
            if (degenerate) {
                // first unit vector with Gram-Schmidt residual^2 >= (N-k)/(2N)
                const double thresh = (double)(N - k) / (2.0 * (double)N);
                for (int i = 0; i < N; ++i) {
                    double sq = 0.0;
                    for (int j = tid; j < N; j += NT) {
                        double s = 0.0;
                        for (int l = 0; l < k; ++l)
                            s += (double)P[j + (int64_t)l * N] * (double)P[i + (int64_t)l * N];
                        const double rv = (j == i ? 1.0 : 0.0) - s;
                        p[j] = rv;
                        sq += rv * rv;
                    }
                    sq = bblock_sum(sq, red);
                    if (sq >= thresh) {
                        pn = sqrt(sq);
                        break;
                    }
                }
                s_cur = 0.0;
            }
            __syncthreads();
            // finish component k: V[:,k], P[:,k], then W[:,k] = X^T v_k
            for (int m = tid; m < M; m += NT) {
                const double v = degenerate ? 0.0 : t[m] / s_cur;
                t[m] = v;
                T[m + (int64_t)k * M] = (float)v;
            }
            for (int j = tid; j < N; j += NT)
                P[j + (int64_t)k * N] = (float)(p[j] / pn);
            if (tid == 0) {
                sig[k] = s_cur;
                if (it.sigma)
                    it.sigma[k] = s_cur;
                if (it.iters)
                    it.iters[k] = iters;
                if (it.start_col)
                    it.start_col[k] = (int32_t)c0;
            }
            __syncthreads();
            if (k + 1 < K) {
                // W[:, k] = X^T v_k (q is free here)
                batch_tpass<false>(X, ldx, M, N, t, reinterpret_cast<double *>(xr), q);
                __syncthreads();
                for (int j = tid; j < N; j += NT)
                    W[j + (int64_t)k * N] = degenerate ? 0.0 : q[j];
            }
            __syncthreads();
        }
        // T = V Lambda, lambda = sigma^2, status
        for (int k = 0; k < K; ++k)
            for (int m = tid; m < M; m += NT)
                T[m + (int64_t)k * M] = (float)((double)T[m + (int64_t)k * M] * sig[k]);
        if (tid < K)
            it.lambda[tid] = sig[tid] * sig[tid];
        if (tid == 0 && it.status)
            *it.status = not_conv ? 1 : 0;
        __syncthreads();
    }
}

void batched_launch(const BatchItem *items, int nprob, const int32_t *order, uint32_t *queue,
                    BatchArgs a, int grid, int threads, int per_cu, size_t lds_bytes,
                    hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(1), 0, s, queue);
    if (threads * per_cu <= 512)
        hipLaunchKernelGGL(k_batched<512>, dim3(grid), dim3(threads), lds_bytes, s, items, nprob,
                           order, queue, a);
    else
        hipLaunchKernelGGL(k_batched<1024>, dim3(grid), dim3(threads), lds_bytes, s, items,
                           nprob, order, queue, a);
}

}  // namespace gspca
