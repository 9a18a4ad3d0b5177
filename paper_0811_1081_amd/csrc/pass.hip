// pass.hip -- the streaming kernel of the single-pass power iteration
// (Andrecut, arXiv:0811.1081, Secs. 2.2-2.3: t = R p and p = R^T t of one
// iteration from one read of R): one persistent workgroup per compute unit
// walks its panels of the row-panel matrix (panel.h) and, for each panel,
// computes the PR entries of t = A p (a workgroup reduction), then
// immediately adds the panel's contribution A_b^T t_b to its private copy of
// q = A^T t, using the panel values still in registers.
#include "panel.h"

namespace gspca {

// ---------------------------------------------------------------------------
// The fused pass.  FIRST: q = A^T t_in only (the start of a component).
// Otherwise: t = A (p / |p|) (written to t_out in FP64) and q = A^T t.  q is
// left as per-workgroup partials q_part[g][j].  The pass only streams A: the
// Gram-Schmidt coefficients d = V_(k)^T t are formed by a separate coalesced
// reduction over the rows of t_out.

// Variants: PL = false keeps the loading in registers (at most 512 threads,
// 8 waves per compute unit); PL = true keeps it in LDS, freeing registers for
// 1024 threads (16 waves per compute unit).  PIPE = true prefetches the next
// panel into a second register buffer; PIPE = false holds one panel and is
// meant for two workgroups per compute unit.  `skew` != 0 interleaves the
// panel assignment (see below).

// Occupancy request of a pass variant: the single-buffer BF16 and FP8 passes
// are held to 128 registers so that two workgroups share a compute unit (at
// 65536 x 8192: BF16 206 -> 190 us, FP8 128 -> 118 us per pass, despite a few
// spilled registers outside the panel loop).
// The value `v` holds in lane r of the wave (r a compile-time constant),
// uniform across the wave.
__device__ inline float lane_value(float v, int r)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), r));
}
__device__ inline double lane_value(double v, int r)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), r);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), r);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <class C, bool PL, bool PIPE>
constexpr int pass_waves_per_eu()
{
    return (!PL && !PIPE && C::PR >= 8) ? 4 : 1;
}

template <class C, int CPT, bool FIRST, bool PL, bool PIPE>
__global__ __launch_bounds__(PL ? 1024 : 512, (pass_waves_per_eu<C, PL, PIPE>())) void k_pass(
    const unsigned char *__restrict__ A, int64_t N, int64_t NP, int64_t ldp, int64_t M,
    const float *__restrict__ scale, const double *__restrict__ p,
    const typename C::acc *__restrict__ t_in, double *__restrict__ t_out,
    double *__restrict__ tsq, typename C::acc *__restrict__ q_part, LoopState *st, int skew)
{
    if (st->done)
        return;
    using E = typename C::acc;
    using RT = typename C::raw;
    constexpr int PR = C::PR;
    __shared__ E red[2][16][PR];
    extern __shared__ unsigned char pass_smem[];
    E *pl = reinterpret_cast<E *>(pass_smem);
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int NT = blockDim.x, nw = NT >> 6;
    const int64_t G = gridDim.x, g = blockIdx.x;
    // order 0: workgroup g owns the contiguous panels [b0, b1); order 1: it
    // owns panels g, g + G, g + 2G, ... so that at any moment the grid reads
    // one contiguous stretch of the matrix.
    const bool inter = skew != 0;
    const int64_t b0 = inter ? g : NP * g / G, b1 = inter ? NP : NP * (g + 1) / G;
    const int64_t cnt = inter ? (g < NP ? (NP - 1 - g) / G + 1 : 0) : b1 - b0;
    E preg[PL ? 1 : CPT];
    E q[CPT];
    double tacc = 0.0; // |t|^2 over this workgroup's rows (threads tid < PR)
    const double inv = FIRST ? 0.0 : 1.0 / st->pnorm;
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t j = tid + (int64_t)c * NT;
        double pj = 0.0;
        if (!FIRST && j < N) {
            pj = p[j] * inv;
            if constexpr (C::scaled)
                pj *= (double)scale[j];
        }
        if constexpr (PL)
            pl[tid + c * NT] = (E)pj;
        else
            preg[c] = (E)pj;
        q[c] = E(0);
    }
    if constexpr (PL)
        __syncthreads();
    auto pval = [&](int c) -> E {
        if constexpr (PL)
            return pl[tid + c * NT];
        else
            return preg[c];
    };
    // The panel width ldp = NT * CPT covers every lane's columns (columns >= N
    // are zero), so every lane always loads: no divergent branch around the
    // loads, and the wait for one panel does not also wait for the prefetched
    // next one.  Lanes past N carry p = 0 and never store q.
    RT bufA[CPT], bufB[PIPE ? CPT : 1];
    const uint32_t lane_off = (uint32_t)tid * 16u;
    const int64_t col_step = (int64_t)NT * 16;
    // uniform (scalar) base per panel and column block + one per-lane offset
    auto load = [&](RT *buf, int64_t b) {
        const unsigned char *pb = A + b * ldp * 16;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const unsigned char *cb = pb + c * col_step;
#ifdef GSPCA_PLAIN_LOADS
            buf[c] = *reinterpret_cast<const RT *>(cb + lane_off);
#else
            buf[c] = __builtin_nontemporal_load(reinterpret_cast<const RT *>(cb + lane_off));
#endif
        }
    };
    auto process = [&](const RT *buf, int64_t b, int slot) {
        E tb[PR];
        if (FIRST) {
#pragma unroll
            for (int r = 0; r < PR; ++r)
                tb[r] = t_in[b * PR + r];
        } else {
            E tp[PR];
#pragma unroll
            for (int r = 0; r < PR; ++r)
                tp[r] = E(0);
#pragma unroll
            for (int c = 0; c < CPT; ++c) {
                E e[PR];
                C::decode(buf[c], e);
                const E pc = pval(c);
#pragma unroll
                for (int r = 0; r < PR; ++r)
                    tp[r] += e[r] * pc;
            }
            if constexpr (PR >= kScatterMinRows) {
                int row;
                const E tw = wave_scatter_sum<E, PR>(tp, lane, row);
                if ((lane & (64 / PR - 1)) == 0)
                    red[slot][w][row] = tw;
            } else {
#pragma unroll
                for (int r = 0; r < PR; ++r)
                    tp[r] = fwave_sum(tp[r]);
                if (lane == 0)
#pragma unroll
                    for (int r = 0; r < PR; ++r)
                        red[slot][w][r] = tp[r];
            }
            __syncthreads();
            // lane r < PR of every wave adds row r over the waves (in wave
            // order), then the PR totals are read from those lanes: PR LDS
            // reads per wave instead of nw * PR broadcast reads per lane
            E mine = E(0);
            if (lane < PR)
                for (int i = 0; i < nw; ++i)
                    mine += red[slot][i][lane];
#pragma unroll
            for (int r = 0; r < PR; ++r)
                tb[r] = lane_value(mine, r);
            if (tid < PR) {
                const int64_t m = b * PR + tid;
                const double tv = (double)tb[tid];
                t_out[m] = tv;
                tacc += tv * tv; // rows past M are zero
            }
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            // Decode again rather than keep the decoded values of all CPT
            // segments alive across the reduction (16 floats per segment for
            // FP8): the empty asm hides the raw value from common-subexpression
            // elimination.
            RT raw = buf[c];
            if constexpr (C::scaled) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    unsigned int x = raw[u];
                    asm volatile("" : "+v"(x));
                    raw[u] = x;
                }
            }
            E e[PR];
            C::decode(raw, e);
#pragma unroll
            for (int r = 0; r < PR; ++r)
                q[c] += e[r] * tb[r];
        }
    };

    // Software pipeline: panel i+1 is in flight while panel i is reduced.  The
    // steady-state loop issues its prefetches unconditionally; the last one or
    // two panels are peeled.  Panel i of this workgroup is b0 + (i + off) % cnt.
    auto pid = [&](int64_t i) -> int64_t { return inter ? g + i * G : b0 + i; };
    int64_t i = 0;
    if constexpr (PIPE) {
        if (i < cnt)
            load(bufA, pid(i));
        while (i + 2 < cnt) {
            load(bufB, pid(i + 1));
            process(bufA, pid(i), 0);
            load(bufA, pid(i + 2));
            process(bufB, pid(i + 1), 1);
            i += 2;
        }
        if (i + 1 < cnt) {
            load(bufB, pid(i + 1));
            process(bufA, pid(i), 0);
            process(bufB, pid(i + 1), 1);
        } else if (i < cnt) {
            process(bufA, pid(i), 0);
        }
    } else {
        // one panel in registers; latency is hidden by a second workgroup on
        // the same compute unit
        for (; i < cnt; ++i) {
            load(bufA, pid(i));
            process(bufA, pid(i), (int)(i & 1));
        }
    }
#pragma unroll
    for (int c = 0; c < CPT; ++c) {
        const int64_t j = tid + (int64_t)c * NT;
        if (j < N) {
            E v = q[c];
            if constexpr (C::scaled)
                v *= scale[j];
            q_part[g * N + j] = v;
        }
    }
    if (!FIRST && w == 0) {
        const double tt = fwave_sum(tacc); // lanes >= PR hold 0
        if (lane == 0)
            tsq[g] = tt;
    }
}

// ---------------------------------------------------------------------------
// Launcher.

template <class C, bool FIRST>
static void launch_pass(int cpt, int G, int NT, int plds, int skew, int pipe,
                        const unsigned char *A, int64_t N, int64_t NP, int64_t ldp, int64_t M,
                        const float *scale, const double *p, const typename C::acc *t_in,
                        double *t_out, double *tsq, typename C::acc *q_part, LoopState *st,
                        hipStream_t s)
{
    const size_t lds = plds ? (size_t)cpt * NT * sizeof(typename C::acc) : 0;
#define GSPCA_PASS(CP, PLV, PIV)                                                               \
    hipLaunchKernelGGL((k_pass<C, CP, FIRST, PLV, PIV>), dim3(G), dim3(NT), lds, s, A, N, NP,  \
                       ldp, M, scale, p, t_in, t_out, tsq, q_part, st, skew)
#define GSPCA_PASS_CPT(PLV, PIV)                                                               \
    switch (cpt) {                                                                             \
    case 1: GSPCA_PASS(1, PLV, PIV); break;                                                    \
    case 2: GSPCA_PASS(2, PLV, PIV); break;                                                    \
    case 4: GSPCA_PASS(4, PLV, PIV); break;                                                    \
    case 8: GSPCA_PASS(8, PLV, PIV); break;                                                    \
    default: GSPCA_PASS(16, PLV, PIV); break;                                                  \
    }
    if (plds) {
        if (pipe) { GSPCA_PASS_CPT(true, true) } else { GSPCA_PASS_CPT(true, false) }
    } else {
        if (pipe) { GSPCA_PASS_CPT(false, true) } else { GSPCA_PASS_CPT(false, false) }
    }
#undef GSPCA_PASS_CPT
#undef GSPCA_PASS
}

template <int F>
void Fused<F>::pass(int first, int cpt, int G, int NT, int plds, int skew, int pipe,
                    const unsigned char *A,
                    int64_t N, int64_t NP, int64_t ldp, int64_t M, const float *scale,
                    const double *p, const E *t_in, double *t_out, double *tsq, E *q_part,
                    LoopState *st, hipStream_t s)
{
    using C = typename CodecOf<F>::type;
    if (first)
        launch_pass<C, true>(cpt, G, NT, plds, skew, pipe, A, N, NP, ldp, M, scale, p, t_in,
                             t_out, tsq, q_part, st, s);
    else
        launch_pass<C, false>(cpt, G, NT, plds, skew, pipe, A, N, NP, ldp, M, scale, p, t_in,
                              t_out, tsq, q_part, st, s);
}

template void Fused<kFmtF64>::pass(int, int, int, int, int, int, int, const unsigned char *,
                                   int64_t, int64_t, int64_t, int64_t, const float *,
                                   const double *, const double *, double *, double *, double *,
                                   LoopState *, hipStream_t);
template void Fused<kFmtF32>::pass(int, int, int, int, int, int, int, const unsigned char *,
                                   int64_t, int64_t, int64_t, int64_t, const float *,
                                   const double *, const float *, double *, double *, float *,
                                   LoopState *, hipStream_t);
template void Fused<kFmtBF16>::pass(int, int, int, int, int, int, int, const unsigned char *,
                                    int64_t, int64_t, int64_t, int64_t, const float *,
                                    const double *, const float *, double *, double *, float *,
                                    LoopState *, hipStream_t);
template void Fused<kFmtFP8>::pass(int, int, int, int, int, int, int, const unsigned char *,
                                   int64_t, int64_t, int64_t, int64_t, const float *,
                                   const double *, const float *, double *, double *, float *,
                                   LoopState *, hipStream_t);

}  // namespace gspca
