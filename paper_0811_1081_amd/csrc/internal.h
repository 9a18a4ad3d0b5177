// internal.h -- launch interface between the host orchestration (gspca.cpp)
// and the gfx950 kernels (kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace gspca {

// Threads per workgroup of the streaming kernels (4 wave64s).
constexpr int kBlock = 256;
// Row padding of the internal residual copy: every column starts 256-byte
// aligned for FP32 (512 for FP64), so 16-byte vector loads never straddle.
constexpr int64_t kRowAlign = 64;

// Per-fit loop state, resident in device memory.  Written by the kernels that
// finish a reduction (the last workgroup to arrive), read back by the host
// once per batch of iterations.
struct LoopState {
    double sigma;      // |t| after the current iteration
    double mu;         // previous estimate (0 at the start of a component)
    double pnorm;      // |p| after the Gram-Schmidt pass of this iteration
    double delta;      // |sigma - mu| / sigma of the last iteration
    double delta_prev; // the same one iteration earlier
    double dp;         // |p_j - s p_(j-1)| of the loading in use (inf for j = 1)
    int32_t iter;      // iterations done on the current component
    int32_t done;      // the current component has stopped
    int32_t converged; // stopped by the relative test
    int32_t degenerate;
    int32_t start_col;
    int32_t nonfinite;     // X held NaN/Inf
    int32_t not_converged; // some component ran out of iterations
    int32_t pad;
    uint32_t counter[8];   // arrival counters of the last-workgroup reductions
};

enum Counter { kCntDotN = 0, kCntApplyN = 1, kCntDotM = 2, kCntApplyM = 3 };

// Last-arriving workgroup detection.  Each workgroup has written its partial
// results before calling.  The barrier orders every wave's writes before
// thread 0, whose device-scope release fence then publishes them to all XCDs
// (one L2 write-back per workgroup rather than one per wave, which costs tens
// of microseconds on wide grids); its atomic elects the final workgroup, whose
// threads acquire before reading the partials.  The winner resets the counter.
__device__ inline bool arrive_last(uint32_t *counter, int *flag_lds)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(counter, 1u);
        *flag_lds = (prev == gridDim.x * gridDim.y - 1) ? 1 : 0;
    }
    __syncthreads();
    const bool last = *flag_lds != 0;
    if (last)
        __threadfence();
    return last;
}

// The loop-state fields the stop test reads, loaded ahead of time.
struct ScoreState {
    int32_t iter;
    double mu, delta, dp;
};
__device__ inline ScoreState score_state(const LoopState *st)
{
    return ScoreState{st->iter, st->mu, st->delta, st->dp};
}

// End of an iteration on the score side, by one thread: sigma = |t| after
// the Gram-Schmidt pass, then the stop test -- the relative sigma test of the
// host programs (Appendices 1, 3) when stop == 0, the loading change below
// tol when stop == 1, or the replayed count -- and the loop state.  `ss`
// holds the state as it was before this iteration.
__device__ inline void score_test(LoopState *st, ScoreState ss, double nrm, double tol,
                                  int32_t limit, int replay, double tiny, int stop)
{
    const int it = ss.iter + 1;
    st->iter = it;
    st->sigma = nrm;
    if (!(nrm >= tiny)) {
        st->degenerate = 1;
        st->done = 1;
        return;
    }
    const double mu = ss.mu;
    st->delta_prev = ss.delta;
    st->delta = stop == 1 ? ss.dp : fabs(nrm - mu) / nrm;
    if (replay) {
        if (it >= limit)
            st->done = 1;
        return;
    }
    const bool pass_test = stop == 1 ? (ss.dp < tol) : (fabs(mu - nrm) < tol * nrm);
    if (pass_test) {
        st->converged = 1;
        st->done = 1;
        return;
    }
    st->mu = nrm;
    if (it >= limit) {
        st->done = 1;
        st->not_converged = 1;
    }
}
__device__ inline void score_test(LoopState *st, double nrm, double tol, int32_t limit,
                                  int replay, double tiny, int stop)
{
    score_test(st, score_state(st), nrm, tol, limit, replay, tiny, stop);
}

// out[i] = sum over b < nb of part[b*k + i], i < k, by one whole workgroup:
// column i gets S = blockDim / k threads (slice s sums partials b = s, s+S,
// ... with UL loads in flight), and the S slice sums are added in slice
// order, so the result is the same on every run.  `lds` holds blockDim
// doubles.  All threads must call it.  Returns, in each thread, the sum of
// squares of the outputs that thread wrote (0 in the others).
template <int UL = 8>
__device__ inline double reduce_partials(const double *__restrict__ part, int64_t nb, int k,
                                         double *__restrict__ out, double *lds)
{
    const int nt = blockDim.x, t = threadIdx.x;
    double ssq = 0.0;
    for (int c0 = 0; c0 < k; c0 += nt) {
        const int kk = k - c0 < nt ? k - c0 : nt;
        const int S = nt / kk;
        const int i = t % kk, sl = t / kk;
        double a[UL];
#pragma unroll
        for (int u = 0; u < UL; ++u)
            a[u] = 0.0;
        if (sl < S) {
            for (int64_t b = sl; b < nb; b += UL * (int64_t)S) {
                // unconditional loads (index clamped) so that all UL are in
                // flight; the ones past nb are dropped afterwards
                double x[UL];
#pragma unroll
                for (int u = 0; u < UL; ++u) {
                    const int64_t bb = b + (int64_t)u * S;
                    x[u] = part[(bb < nb ? bb : nb - 1) * k + c0 + i];
                }
#pragma unroll
                for (int u = 0; u < UL; ++u)
                    a[u] += b + (int64_t)u * S < nb ? x[u] : 0.0;
            }
        }
        // pairwise, in a fixed order
#pragma unroll
        for (int h = UL / 2; h > 0; h >>= 1)
#pragma unroll
            for (int u = 0; u < h; ++u)
                a[u] += a[u + h];
        __syncthreads();
        lds[t] = a[0];
        __syncthreads();
        if (t < kk) {
            double r = 0.0;
            for (int q = 0; q < S; ++q)
                r += lds[q * kk + t];
            out[c0 + t] = r;
            ssq += r * r;
        }
    }
    return ssq;
}

// Largest N whose loading side runs in one workgroup (k_fin_apply).
constexpr int64_t kFinApplyMaxN = 1024;

// Groups of partial sums per workgroup of the loading-side finish (64
// columns each; 64 * kFinGroups threads).
constexpr int kFinGroups = 16;

// Rows per workgroup of the score coefficient reduction: whole blocks of
// 1024, about 96 row blocks, at most kScoreRows (staged in LDS as FP64).
// A single workgroup takes everything (no arrival counter) when t fits it
// and it has at most two 1024-row chunks of V to read (kd <= 32), or none:
// FP64 sweep at M = 2000, 264 -> 237 ms per GS fit; at M = 4000 the four
// chunks in one workgroup cost more than the counter (493 -> 518 ms), while
// NIPALS (no V) still gained (331 -> 307 ms).
constexpr int64_t kScoreRows = 4096;
inline int64_t score_rows(int64_t M, int kd)
{
    if ((kd == 0 && M <= kScoreRows) || (kd <= 32 && M <= 2048))
        return (M + 1023) / 1024 * 1024;
    const int64_t r = ((M + 95) / 96 + 1023) / 1024 * 1024;
    return r > kScoreRows ? kScoreRows : r;
}

// Zero the loop state on `s` with a one-thread kernel: no memset node is
// recorded when the caller captures the stream into a graph.
void reset_state(LoopState *st, hipStream_t s);
// 1 when `s` is being captured into a graph, 0 when not, -1 when the query
// failed.  Entry points that read results back to the host refuse capture.
int stream_capturing(hipStream_t s);

struct StartArgs {
    int32_t k;
    int32_t init;           // gspca_init
    int32_t force_degenerate;
    int32_t gs;             // GS-PCA: a given start is also tested against V_(k)
    const int32_t *replay_start; // device, nullable
};

template <typename E>
struct Launch {
    static void copy_pad(const E *X, int64_t ldx, E *R, int64_t ldr, int64_t M, int64_t N,
                         LoopState *st, hipStream_t s);
    static void colnorm(const E *R, int64_t ldr, int64_t M, int64_t N, double *cn, hipStream_t s);
    static void start(const E *R, int64_t ldr, int64_t M, int64_t N, const double *cn, const E *V,
                      const E *T0, StartArgs a, double tiny, E *t, LoopState *st, hipStream_t s);
    static void gemv_t(const E *R, int64_t ldr, int64_t N, const E *t, int64_t rows_per_split,
                       int nsplit, int ncolblk, double *qpart, const LoopState *st, hipStream_t s);
    static void gemv_n(const E *R, int64_t ldr, int64_t N, const double *p, int64_t cols_per_split,
                       int nsplit, double *tpart, const LoopState *st, hipStream_t s);
    static void gs_dot(const double *part, int nsplit, int64_t ldpart, int64_t L, const E *Q,
                       int64_t ldq, int k, double *y, double *cpart, double *c, LoopState *st,
                       int counter, hipStream_t s);
    static void gs_apply(const double *part, int nsplit, int64_t ldpart, int64_t L,
                         const double *y, const E *Q, int64_t ldq, int k, const double *c,
                         double *ydst, double *yprev, E *edst, double *sqpart, LoopState *st,
                         int side, double tol, int32_t limit, int replay, double tiny, int stop,
                         hipStream_t s);
    // y <- y - Q c (FP64, in place; the first pass of CGS2)
    static void gs_project(double *y, int64_t L, const E *Q, int64_t ldq, int k, const double *c,
                           LoopState *st, hipStream_t s);
    // y <- sum of the partials, reduced by the modified Gram-Schmidt process
    // against the k columns of Q (one workgroup)
    static void mgs(const double *part, int nsplit, int64_t ldpart, int64_t L, const E *Q,
                    int64_t ldq, int k, double *y, LoopState *st, hipStream_t s);
    static void degenerate_p(const E *P, int64_t N, int k, double *p, LoopState *st, hipStream_t s);
    static void finalize_comp(const E *t, int64_t M, int64_t N, const double *p, int k, int gs,
                              E *T, E *P, double *sigma, int32_t *iters, int32_t *start_col,
                              LoopState *st, hipStream_t s);
    static void deflate(E *R, int64_t ldr, int64_t M, int64_t N, const E *t, const E *pk,
                        double *cn, hipStream_t s);
    static void finalize_all(E *T, int64_t M, int K, const double *sigma, double *lambda,
                             double *sigma_out, int gs, hipStream_t s);
};

// Single-pass path (fused.hip): the data matrix in 16-byte row panels, in one
// of four storage formats.  E is the arithmetic/output element type.
enum Fmt { kFmtF64 = 0, kFmtF32 = 1, kFmtBF16 = 2, kFmtFP8 = 3 };
template <int F> struct FmtElem { using type = float; };
template <> struct FmtElem<kFmtF64> { using type = double; };
constexpr int fmt_rows(int f) { return f == kFmtF64 ? 2 : f == kFmtF32 ? 4 : f == kFmtBF16 ? 8 : 16; }

template <int F>
struct Fused {
    using E = typename FmtElem<F>::type;
    static void retile(const E *X, int64_t ldx, int64_t M, int64_t N, int64_t NP, int64_t ldp,
                       unsigned char *A, LoopState *st, hipStream_t s);
    static void quantize(const float *X, int64_t ldx, int64_t M, int64_t N, int64_t NP,
                         int64_t ldp, float *scale, unsigned char *Q, LoopState *st,
                         hipStream_t s);
    static void deflate(unsigned char *A, int64_t N, int64_t NP, int64_t ldp, const E *t,
                        const E *pk, int update, const float *scale, int nsplit, double *cnpart,
                        hipStream_t s);
    static void colnorm_finish(const double *cnpart, int nsplit, int64_t N, double *cn0,
                               double *cn, int implicit, int k, const E *P, const double *W,
                               const double *sig, hipStream_t s);
    // defl_t, defl_p (explicit deflation pending): the start column is taken
    // from A - defl_t defl_p^T
    static void start(const unsigned char *A, int64_t N, int64_t NP, int64_t ldp, int64_t M,
                      const float *scale, int implicit, const E *V, const E *P, const double *sig,
                      const double *cn, const E *T0, StartArgs a, double tiny, E *t,
                      double *part, LoopState *st, hipStream_t s, const E *defl_t = nullptr,
                      const E *defl_p = nullptr);
    // explicit deflation and the next component's first loading in one pass
    static void deflate_first(unsigned char *A, int64_t N, int64_t NP, int64_t ldp, const E *t,
                              const E *pk, int update, const E *t0, int nsplit, double *cnpart,
                              E *q_part, hipStream_t s);
    static void colnorm_predict(const double *cn, int64_t N, const E *pk, const double *qy,
                                const LoopState *st, double *out, hipStream_t s);
    static void pass(int first, int cpt, int G, int NT, int plds, int skew, int pipe,
                     const unsigned char *A,
                     int64_t N, int64_t NP, int64_t ldp, int64_t M, const float *scale,
                     const double *p, const E *t_in, double *t_out, double *tsq, E *q_part,
                     LoopState *st, hipStream_t s);
    static void score_dot(const double *t, int64_t M, const E *V, int kd, const double *tsq,
                          int G, double *cpart, double *d, LoopState *st, double tol,
                          int32_t limit, int replay, double tiny, int stop, hipStream_t s);
    static void fin_q(const E *q_part, int64_t G, int64_t N, const double *W, int kd,
                      const double *d, const E *P, int kg, double *qy, double *cpart, double *c,
                      LoopState *st, int it, hipStream_t s);
    // score_dot and fin_apply in one launch of one workgroup, when both fit
    // one (score_fin_fits(M, kd) and the fin_apply condition)
    static bool score_fin_fits(int64_t M, int kd);
    static void score_fin(const double *t, int64_t M, const E *V, int kd, const double *tsq,
                          int G, double *cpart, double *d, double tol, int32_t limit,
                          int replay, const E *q_part, int64_t Gq, int64_t N, const double *W,
                          const E *P, int kg, double *qy, double *p, double *pprev,
                          LoopState *st, int it, int stop, double tiny, hipStream_t s);
    // fin_q and the loading-side gs_apply in one workgroup (N <= 1024)
    static void fin_apply(const E *q_part, int64_t G, int64_t N, const double *W, int kd,
                          const double *d, const E *P, int kg, double *qy, double *p,
                          double *pprev, LoopState *st, int it, int stop, double tiny,
                          hipStream_t s);
    static void comp_end(const double *td, const double *d, int kd, E *tE, int64_t M, int64_t N,
                         const double *p, const double *qy, int k, int gs, int explicit_defl,
                         E *T, E *P, double *W, double *sigma, int32_t *iters,
                         int32_t *start_col, LoopState *st, hipStream_t s);
};

// Sketch products and whitening (mlp.hip), shared by the warm start and the
// block iteration (block.hip).  Row slices of the refinement's X^T Z (about
// 2048 workgroups) and of the Gram matrix (at most 256), and the workspace
// they use (the whitening alone needs off_wpart bytes).
struct SketchPlan {
    int64_t st, rows_t, sg, rows_g;
    size_t off_gpart, off_qs, off_wpart, total;
};
SketchPlan sketch_plan(int64_t M, int64_t N, int r);
bool valid_rank(int32_t r); // sketch widths: 32 or 64
// Y = X Om (X column-major, Om row-major N x r, Y row-major M x r)
void launch_sketch(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Om, int r,
                   float *Y, hipStream_t s);
// W = X^T Z / sqrt(M) (Z row-major M x r, W row-major N x r); W = X^T Z when
// unit_scale
void launch_sketch_t(const float *X, int64_t ldx, int64_t M, int64_t N, const float *Z, int r,
                     float *W, unsigned char *ws, hipStream_t s, bool unit_scale = false);
// The first loadings X^T T0 of all given starts (FP32, implicit deflation)
// by matrix-core passes over X, one per block of r = 32 or 64 columns of T0
// (column-major M x K): the block into rows of width r (zero-padded),
// W = X^T Z, then W's first columns into Q0 (column-major N x K).  ws:
// first_loadings_bytes(M, N, K).
size_t first_loadings_bytes(int64_t M, int64_t N, int64_t K);
void launch_first_loadings(const float *X, int64_t ldx, int64_t M, int64_t N, const float *T0,
                           int64_t K, float *Q0, unsigned char *ws, hipStream_t s);
// Z = sqrt(M) Y Q diag(g)^(-1/2), g the eigenvalues of Y^T Y (decreasing)
void launch_whiten(const float *Y, int64_t M, int r, float *Z, double *g, int32_t *flag,
                   unsigned char *ws, hipStream_t s);

// Batched path (batched.hip): one workgroup per problem, persistent queue.
struct BatchItem {
    const float *X;
    int64_t ldx;
    int32_t M, N, K, pad;
    float *T, *P;
    double *lambda, *sigma;
    int32_t *iters, *start_col;
    const int32_t *replay_iters, *replay_start;
    int32_t *status;
    double *W; // N x K workspace
    const float *T0; // given start vectors (M x K), init == GIVEN
};
struct BatchArgs {
    double tol, tiny;
    int32_t max_iter, init, stop, pad;
};
void batched_launch(const BatchItem *items, int nprob, const int32_t *order, uint32_t *queue,
                    BatchArgs a, int grid, int threads, int per_cu, size_t lds_bytes,
                    hipStream_t s);
// Length of k_batched's FP32 copy of p: N values, then zeros past the last
// column any wave of the single pass reads (the column split covers at most
// 2 N + N / 8 + 30 columns), in whole 16-byte groups.
__host__ __device__ inline int batched_pf_floats(int N) { return 4 * ((3 * N + 67) / 4); }

inline size_t batched_lds_bytes(int64_t M, int64_t N, int64_t K)
{
    // 16 KiB of cross-wave sums for the single pass, p in FP32, then the vectors
    return (size_t)16384 + (size_t)batched_pf_floats((int)N) * 4 + (size_t)(M + 4 * N + 2 * K) * 8;
}

}  // namespace gspca
