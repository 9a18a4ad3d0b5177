// host.hip -- C ABI of the iterative-PCA library: validation, workspace plan and
// the stream-ordered launch sequence of NIPALS-PCA (Sec. 2.2) and GS-PCA
// (Sec. 2.3) of Andrecut, arXiv:0811.1081.
//
// Per component k:  start vector -> iterations (six kernels each, see
// kernels.hip) -> finish (V[:,k] = t / sigma, P[:,k] = p / |p|) -> explicit
// deflation R <- R - t p^T fused with the column norms used by the next start.
// The convergence test runs on the device; the host reads one small status
// record per batch of iterations and sizes the next batch from the observed
// geometric decay of the relative change (so the GPU is not idled by a
// round-trip every iteration, as in the paper's programs, which read the norm
// back twice per iteration).
#include <float.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/gspca.h"
#include "internal.h"

using namespace gspca;

namespace {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Launch geometry and workspace layout of one fit.
struct Plan {
    int64_t M, N, K, ldr;
    int ncolblk, nsplit_t, nsplit_n, nbM, nbN;
    int64_t rows_per_split, cols_per_split;
    size_t off_state, off_R, off_t, off_qpart, off_tpart, off_qy, off_ty, off_cpart, off_c,
        off_sq, off_cn, off_p, off_pprev, off_sig, total;
};

Plan make_plan(int64_t M, int64_t N, int64_t K, size_t esize)
{
    Plan pl{};
    pl.M = M;
    pl.N = N;
    pl.K = K;
    pl.ldr = cdiv(M, kRowAlign) * kRowAlign;
    const int64_t vn = 16 / (int64_t)esize;
    const int64_t row_unit = (int64_t)kBlock * vn;
    const int64_t nrow_units = cdiv(pl.ldr, row_unit);
    const int64_t target_wg = 2048; // >> 256 CUs: several resident workgroups per CU
    // gemv_t: 8 columns per workgroup, rows split so that the grid is large
    pl.ncolblk = (int)cdiv(N, 8);
    int64_t ns = std::min<int64_t>(std::max<int64_t>(cdiv(target_wg, pl.ncolblk), 1), nrow_units);
    pl.rows_per_split = cdiv(nrow_units, ns) * row_unit;
    pl.nsplit_t = (int)cdiv(pl.ldr, pl.rows_per_split);
    // gemv_n: 256*vn rows per workgroup, columns split
    const int64_t nbr = nrow_units;
    int64_t nsn = std::min<int64_t>(std::max<int64_t>(cdiv(target_wg, nbr), 1), cdiv(N, 8));
    pl.cols_per_split = std::min<int64_t>(cdiv(N, nsn), 1024);
    pl.nsplit_n = (int)cdiv(N, pl.cols_per_split);
    pl.nbM = (int)cdiv(M, kBlock);
    pl.nbN = (int)cdiv(N, kBlock);
    const int nbmax = std::max(pl.nbM, pl.nbN);

    size_t o = 0;
    pl.off_state = o; o = align_up(o + sizeof(LoopState));
    pl.off_R = o;     o = align_up(o + (size_t)pl.ldr * N * esize);
    pl.off_t = o;     o = align_up(o + (size_t)pl.ldr * esize);
    pl.off_qpart = o; o = align_up(o + (size_t)pl.nsplit_t * N * 8);
    pl.off_tpart = o; o = align_up(o + (size_t)pl.nsplit_n * pl.ldr * 8);
    pl.off_qy = o;    o = align_up(o + (size_t)N * 8);
    pl.off_ty = o;    o = align_up(o + (size_t)pl.ldr * 8);
    pl.off_cpart = o; o = align_up(o + (size_t)nbmax * (K + 1) * 8);
    pl.off_c = o;     o = align_up(o + (size_t)(K + 1) * 8);
    pl.off_sq = o;    o = align_up(o + (size_t)nbmax * 2 * 8);
    pl.off_cn = o;    o = align_up(o + (size_t)N * 8);
    pl.off_p = o;     o = align_up(o + (size_t)N * 8);
    pl.off_pprev = o; o = align_up(o + (size_t)N * 8);
    pl.off_sig = o;   o = align_up(o + (size_t)K * 8);
    pl.total = o;
    return pl;
}

size_t dtype_size(int32_t dt)
{
    return dt == GSPCA_F64 ? 8 : dt == GSPCA_F32 ? 4 : dt == GSPCA_BF16 ? 2 : dt == GSPCA_FP8_E4M3 ? 1 : 0;
}
bool is_quantised(int32_t dt) { return dt == GSPCA_BF16 || dt == GSPCA_FP8_E4M3; }

gspca_status validate(const gspca_problem *pr, const gspca_options *op)
{
    if (!pr || !op)
        return GSPCA_EINVAL;
    if (dtype_size(pr->dtype) == 0 || !pr->X)
        return GSPCA_EINVAL;
    if (pr->M < 1 || pr->N < 1 || pr->K < 1 || pr->K > pr->M || pr->K > pr->N)
        return GSPCA_EINVAL;
    if (!is_quantised(pr->dtype) && pr->ldx < pr->M)
        return GSPCA_EINVAL;
    // quantised data: codes from gspca_quantize, their scales, implicit
    // deflation (the codes are read-only), GS-PCA, N within the single-pass path
    if (is_quantised(pr->dtype) &&
        (!pr->col_scale || !op->implicit_deflation || op->algo != GSPCA_GS || pr->N > 8192))
        return GSPCA_EINVAL;
    // grid-dimension limits of the launch plan (rows: 2^30, columns: 2^25)
    if (pr->M > (int64_t(1) << 30) || pr->N > (int64_t(1) << 25))
        return GSPCA_EINVAL;
    if (op->algo != GSPCA_GS && op->algo != GSPCA_NIPALS)
        return GSPCA_EINVAL;
    if (op->init != GSPCA_INIT_MAXNORM && op->init != GSPCA_INIT_COLUMN_K &&
        op->init != GSPCA_INIT_GIVEN)
        return GSPCA_EINVAL;
    if (op->init == GSPCA_INIT_GIVEN && !op->T0)
        return GSPCA_EINVAL;
    if (!(op->tol >= 0.0) || !isfinite(op->tol) || op->max_iter < 1)
        return GSPCA_EINVAL;
    if (op->stop != GSPCA_STOP_SIGMA_REL && op->stop != GSPCA_STOP_LOADING)
        return GSPCA_EINVAL;
    if (op->implicit_deflation &&
        (op->algo != GSPCA_GS || pr->N > (pr->dtype == GSPCA_F64 ? 4096 : 8192)))
        return GSPCA_EINVAL;
    if (op->reorth != GSPCA_REORTH_CGS && op->reorth != GSPCA_REORTH_CGS2 &&
        op->reorth != GSPCA_REORTH_MGS)
        return GSPCA_EINVAL;
    // the re-orthogonalisation variants run on the two-pass path
    if (op->reorth != GSPCA_REORTH_CGS && op->algo == GSPCA_GS &&
        (op->implicit_deflation || is_quantised(pr->dtype)))
        return GSPCA_EINVAL;
    return GSPCA_OK;
}

// Next batch size from the geometric decay of the relative change:
// delta_j ~ rho^j, so the test delta < tol passes after about
// log(tol / delta) / log(rho) more iterations.
int next_batch(const LoopState &h, double tol, int cur)
{
    const double d = h.delta, dp = h.delta_prev;
    if (!(tol > 0.0) || !(d > 0.0) || !(dp > 0.0) || !(d < dp) || h.iter < 3)
        return std::min(cur * 2, 16);
    if (d < tol)
        return 1;
    const double rho = d / dp;
    const double rem = log(tol / d) / log(rho);
    if (!(rem > 0.0) || !isfinite(rem))
        return 4;
    return (int)std::min(64.0, std::max(1.0, ceil(rem)));
}

template <typename E>
gspca_status fit_two_pass(const gspca_problem *pr, const gspca_options *op, const gspca_result *rs,
                       void *ws, size_t ws_bytes, hipStream_t s)
{
    const int64_t M = pr->M, N = pr->N, K = pr->K;
    const Plan pl = make_plan(M, N, K, sizeof(E));
    if (!ws || ws_bytes < pl.total)
        return GSPCA_EWORKSPACE;
    if (((uintptr_t)ws) % kAlign)
        return GSPCA_EINVAL;
    unsigned char *base = static_cast<unsigned char *>(ws);
    LoopState *st = reinterpret_cast<LoopState *>(base + pl.off_state);
    E *R = reinterpret_cast<E *>(base + pl.off_R);
    E *t = reinterpret_cast<E *>(base + pl.off_t);
    double *qpart = reinterpret_cast<double *>(base + pl.off_qpart);
    double *tpart = reinterpret_cast<double *>(base + pl.off_tpart);
    double *qy = reinterpret_cast<double *>(base + pl.off_qy);
    double *ty = reinterpret_cast<double *>(base + pl.off_ty);
    double *cpart = reinterpret_cast<double *>(base + pl.off_cpart);
    double *c = reinterpret_cast<double *>(base + pl.off_c);
    double *sq = reinterpret_cast<double *>(base + pl.off_sq);
    double *cn = reinterpret_cast<double *>(base + pl.off_cn);
    double *p = reinterpret_cast<double *>(base + pl.off_p);
    double *pprev = reinterpret_cast<double *>(base + pl.off_pprev);
    double *sig = reinterpret_cast<double *>(base + pl.off_sig);
    E *T = static_cast<E *>(rs->T);
    E *P = static_cast<E *>(rs->P);
    const E *X = static_cast<const E *>(pr->X);
    const E *T0 = static_cast<const E *>(op->T0);
    const double tiny = sizeof(E) == 8 ? DBL_MIN : (double)FLT_MIN;
    const int gs = op->algo == GSPCA_GS;
    const double tol = op->tol;
    using L = Launch<E>;

    std::vector<int32_t> rit;
    const bool replay = op->replay_iters != nullptr;
    if (replay) {
        rit.resize(K);
        if (hipMemcpy(rit.data(), op->replay_iters, K * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return GSPCA_EDEVICE;
        for (int64_t k = 0; k < K; ++k)
            if (rit[k] < 0)
                return GSPCA_EINVAL;
    }

    // optional event timing of the streaming kernels (see gspca_profile)
    gspca_profile *prof = op->profile;
    constexpr int kMaxBatch = 64;
    std::vector<hipEvent_t> ev;
    struct EventPool {
        std::vector<hipEvent_t> *v;
        ~EventPool() { for (hipEvent_t e : *v) (void)hipEventDestroy(e); }
    } ev_guard{&ev};
    if (prof) {
        ev.resize(4 * kMaxBatch);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess)
                return GSPCA_EDEVICE;
        prof->bytes_per_pass = (int64_t)(M * N * (int64_t)sizeof(E));
        prof->single_pass = 0;
    }

    LoopState h{};
    auto read_state = [&]() -> bool {
        if (hipMemcpyAsync(&h, st, sizeof(LoopState), hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        return hipStreamSynchronize(s) == hipSuccess;
    };

    // Gram-Schmidt coefficients of one side (the vector y = sum of the
    // partials against the k columns of Q).  CGS: c = Q^T y.  CGS2: the first
    // pass y <- y - Q (Q^T y) in place, then c = Q^T y for the second pass.
    // MGS: y fully reduced in place by the modified process (the final apply
    // then runs with no columns).  The apply kernel finishes the step.
    const int reorth = gs ? op->reorth : GSPCA_REORTH_CGS;
    auto gs_side = [&](const double *part, int nsplit, int64_t ldpart, int64_t Lv, double *y,
                       const E *Q, int64_t ldq, int kq, double *cp, double *cv, int counter,
                       hipStream_t st_) {
        if (kq == 0)
            return;
        if (reorth == GSPCA_REORTH_MGS) {
            L::mgs(part, nsplit, ldpart, Lv, Q, ldq, kq, y, st, st_);
            return;
        }
        L::gs_dot(part, nsplit, ldpart, Lv, Q, ldq, kq, y, cp, cv, st, counter, st_);
        if (reorth == GSPCA_REORTH_CGS2) {
            L::gs_project(y, Lv, Q, ldq, kq, cv, st, st_);
            L::gs_dot(y, 1, Lv, Lv, Q, ldq, kq, nullptr, cp, cv, st, counter, st_);
        }
    };

    reset_state(st, s);
    L::copy_pad(X, pr->ldx, R, pl.ldr, M, N, st, s);
    if (!read_state())
        return GSPCA_EDEVICE;
    if (h.nonfinite)
        return GSPCA_ENONFINITE;
    L::colnorm(R, pl.ldr, M, N, cn, s);

    for (int64_t k = 0; k < K; ++k) {
        const int32_t limit = replay ? rit[k] : op->max_iter;
        StartArgs a{(int32_t)k, op->init, (replay && limit < 1) ? 1 : 0, gs ? 1 : 0,
                    op->replay_start_col};
        L::start(R, pl.ldr, M, N, cn, T, T0, a, tiny, t, st, s);
        const int kk = gs ? (int)k : 0;
        int32_t enq = 0;
        int batch = 4;
        bool have = false;
        int32_t iter_before = 0;
        while (enq < limit) {
            const int n = std::min<int32_t>(std::min(batch, kMaxBatch), limit - enq);
            for (int i = 0; i < n; ++i) {
                if (prof)
                    (void)hipEventRecord(ev[4 * i], s);
                L::gemv_t(R, pl.ldr, N, t, pl.rows_per_split, pl.nsplit_t, pl.ncolblk, qpart, st, s);
                if (prof)
                    (void)hipEventRecord(ev[4 * i + 1], s);
                // GS on the loading: p <- q - P_(k) c (one pass, two passes or
                // the modified process), then |p| and the loading stop
                gs_side(qpart, pl.nsplit_t, N, N, qy, P, N, kk, cpart, c, kCntDotN, s);
                if (kk > 0 && reorth != GSPCA_REORTH_CGS)
                    L::gs_apply(qy, 1, N, N, qy, P, N, reorth == GSPCA_REORTH_MGS ? 0 : kk, c, p,
                                pprev, nullptr, sq, st, 0, tol, limit, replay, tiny, op->stop, s);
                else
                    L::gs_apply(qpart, pl.nsplit_t, N, N, qy, P, N, kk, c, p, pprev, nullptr, sq,
                                st, 0, tol, limit, replay, tiny, op->stop, s);
                if (prof)
                    (void)hipEventRecord(ev[4 * i + 2], s);
                L::gemv_n(R, pl.ldr, N, p, pl.cols_per_split, pl.nsplit_n, tpart, st, s);
                if (prof)
                    (void)hipEventRecord(ev[4 * i + 3], s);
                gs_side(tpart, pl.nsplit_n, pl.ldr, M, ty, T, M, kk, cpart, c, kCntDotM, s);
                if (kk > 0 && reorth != GSPCA_REORTH_CGS)
                    L::gs_apply(ty, 1, M, M, ty, T, M, reorth == GSPCA_REORTH_MGS ? 0 : kk, c,
                                nullptr, nullptr, t, sq, st, 1, tol, limit, replay, tiny, op->stop,
                                s);
                else
                    L::gs_apply(tpart, pl.nsplit_n, pl.ldr, M, ty, T, M, kk, c, nullptr, nullptr, t,
                                sq, st, 1, tol, limit, replay, tiny, op->stop, s);
            }
            enq += n;
            if (!read_state())
                return GSPCA_EDEVICE;
            have = true;
            if (prof) {
                const int real = std::min(n, h.iter - iter_before);
                for (int i = 0; i < real; ++i) {
                    float a = 0.f, b = 0.f;
                    if (hipEventElapsedTime(&a, ev[4 * i], ev[4 * i + 1]) == hipSuccess &&
                        hipEventElapsedTime(&b, ev[4 * i + 2], ev[4 * i + 3]) == hipSuccess) {
                        prof->gemv_t_ms += a;
                        prof->gemv_n_ms += b;
                        prof->gemv_t_launches += 1;
                        prof->gemv_n_launches += 1;
                    }
                }
                prof->iterations += std::max(0, h.iter - iter_before);
                iter_before = h.iter;
            }
            if (h.done)
                break;
            batch = next_batch(h, tol, batch);
        }
        if (!have && !read_state())
            return GSPCA_EDEVICE;
        if (h.degenerate)
            L::degenerate_p(P, N, (int)k, p, st, s);
        L::finalize_comp(t, M, N, p, (int)k, gs, T, P, sig, rs->iters, rs->start_col, st, s);
        if (k + 1 < K && !h.degenerate)
            L::deflate(R, pl.ldr, M, N, t, P + k * N, cn, s);
    }
    L::finalize_all(T, M, (int)K, sig, rs->lambda, rs->sigma, gs, s);
    if (!read_state())
        return GSPCA_EDEVICE;
    if (hipGetLastError() != hipSuccess)
        return GSPCA_EDEVICE;
    return h.not_converged ? GSPCA_NOT_CONVERGED : GSPCA_OK;
}

// ---------------------------------------------------------------------------
// Single-pass path (fused.hip).

constexpr int64_t kFusedMaxN = 8192; // columns held in registers: 512 threads x 16

struct FusedPlan {
    int64_t M, N, K, PR, NP, ldp;
    int cpt, NT, G, nsplit_cn, nbM, nbN;
    int plds, skew, pipe; // pass-kernel variant: loading in LDS (1024 threads), panel-order
                          // skew, register double buffering (else two workgroups per CU)
    size_t off_state, off_A, off_tE, off_td, off_tsq, off_qpart, off_d, off_c, off_qy, off_p,
        off_pprev, off_cpart, off_sq, off_cnpart, off_cn, off_cn0, off_cnx, off_t0, off_W,
        off_sig, total;
    // the first loadings of all given starts in one pass (implicit FP32, K <= 64):
    // Q0 and its scratch after everything else; total_base excludes them
    size_t off_q0, off_flw, total_base;
};

// Given starts whose first loadings X^T t0 (t0 = the given column: the start
// takes it unmodified) can all be formed up front by matrix-core passes (one
// per 64 components): FP32 data, implicit deflation (X itself is the
// operator).
bool first_loadings_apply(const gspca_problem *pr, const gspca_options *op)
{
    return pr->dtype == GSPCA_F32 && op->implicit_deflation && op->init == GSPCA_INIT_GIVEN &&
           op->T0;
}

int device_cu_count()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1)
        cu = 256;
    return cu;
}

int fmt_of(int32_t dtype)
{
    switch (dtype) {
    case GSPCA_F64: return kFmtF64;
    case GSPCA_F32: return kFmtF32;
    case GSPCA_BF16: return kFmtBF16;
    default: return kFmtFP8;
    }
}

// Panel width: ldp = NT * cpt columns (zero beyond N), the fewest columns per
// thread with at most 512 threads.  Depends on N only, so a quantised matrix
// and the fit that reads it agree on it.
void panel_width(int64_t N, int *cpt, int *NT, int64_t *ldp)
{
    *cpt = N <= 512 ? 1 : N <= 1024 ? 2 : N <= 2048 ? 4 : N <= 4096 ? 8 : 16;
    *NT = (int)std::min<int64_t>(512, cdiv(cdiv(N, *cpt), 64) * 64);
    *ldp = (int64_t)(*NT) * (*cpt);
}

FusedPlan make_fused_plan(int64_t M, int64_t N, int64_t K, int fmt, int ncu, bool q0 = false)
{
    FusedPlan f{};
    f.M = M;
    f.N = N;
    f.K = K;
    f.PR = fmt_rows(fmt);
    const size_t esize = fmt == kFmtF64 ? 8 : 4; // arithmetic / output element
    f.NP = cdiv(M, f.PR);
    panel_width(N, &f.cpt, &f.NT, &f.ldp);
    // Variant knobs (GSPCA_PASS_LDS=1: loading in LDS with twice the threads;
    // GSPCA_PASS_SKEW=0/1: contiguous or interleaved panel order); the panel
    // width is unchanged.  Interleaved is the default: at 65536 x 8192 it
    // measured 414 vs 451 us per FP32 pass and 281 vs 287 us per FP8 pass in
    // the first form of the pass, and with the current pass 103.7 vs 107.0 us
    // (FP8) and 174.9 vs 175.7 us (BF16, which had measured 330 vs 323 us
    // in the first form).
    const char *e_lds = getenv("GSPCA_PASS_LDS");
    const char *e_skew = getenv("GSPCA_PASS_SKEW");
    const char *e_pipe = getenv("GSPCA_PASS_PIPE");
    // FP8 codes keep the loading in LDS by default: their one-buffer pass at
    // 128 registers reloads a spilled register inside the panel loop, while
    // with half the columns per thread it does not (65536 x 8192: 4.96 ->
    // 5.16 TB/s of codes; BF16 loses, 6.10 -> 5.91, and keeps registers)
    const int lds_default = fmt == kFmtFP8 ? 1 : 0;
    const int want_lds = e_lds ? (e_lds[0] == '1' ? 1 : 0) : lds_default;
    f.plds = (want_lds && f.cpt >= 2 && f.NT <= 512) ? 1 : 0;
    f.skew = e_skew ? (e_skew[0] == '1' ? 1 : 0) : 1;
    // Register double buffering pays for FP32 (318 vs 330 us per pass at 65536
    // x 8192); with decoded codes the second buffer spills (BF16 218 vs 185
    // us, FP8 210 vs 140 us with one buffer and two workgroups per CU).
    const int pipe_default = (fmt == kFmtBF16 || fmt == kFmtFP8) ? 0 : 1;
    f.pipe = e_pipe ? (e_pipe[0] == '0' ? 0 : 1) : pipe_default;
    if (f.plds) {
        f.cpt /= 2;
        f.NT *= 2;
    }
    const int64_t per_cu = std::max<int64_t>(1, (f.plds ? 1024 : 512) / f.NT) * (f.pipe ? 1 : 2);
    f.G = (int)std::max<int64_t>(1, std::min<int64_t>(ncu * per_cu, std::max<int64_t>(1, f.NP / 2)));
    f.nsplit_cn = (int)std::max<int64_t>(1, std::min<int64_t>(cdiv(2048, cdiv(N, 64)), f.NP));
    f.nbM = (int)cdiv(M, kBlock);
    f.nbN = (int)cdiv(N, kBlock);
    const int nbmax = (int)std::max<int64_t>(std::max(f.nbM, f.nbN), cdiv(N, 64));
    const size_t len = (size_t)(f.NP * f.PR);
    const bool quantised = fmt == kFmtBF16 || fmt == kFmtFP8; // Q is the caller's
    size_t o = 0;
    f.off_state = o;  o = align_up(o + sizeof(LoopState));
    f.off_A = o;      o = align_up(o + (quantised ? 0 : (size_t)f.NP * f.ldp * 16));
    f.off_tE = o;     o = align_up(o + len * esize);
    f.off_td = o;     o = align_up(o + len * 8);
    f.off_tsq = o;    o = align_up(o + (size_t)f.G * 8);
    f.off_qpart = o;  o = align_up(o + (size_t)f.G * N * esize);
    f.off_d = o;      o = align_up(o + (size_t)(K + 1) * 8);
    f.off_c = o;      o = align_up(o + (size_t)(K + 1) * 8);
    f.off_qy = o;     o = align_up(o + (size_t)N * 8);
    f.off_p = o;      o = align_up(o + (size_t)N * 8);
    f.off_pprev = o;  o = align_up(o + (size_t)N * 8);
    f.off_cpart = o;  o = align_up(o + (size_t)nbmax * (K + 1) * 8);
    f.off_sq = o;     o = align_up(o + (size_t)nbmax * 2 * 8);
    // norm partials: the deflation's splits, or the pass's workgroups when
    // the explicit deflation also forms the next first loading
    f.off_cnpart = o; o = align_up(o + (size_t)std::max(f.nsplit_cn, f.G) * N * 8);
    f.off_cn = o;     o = align_up(o + (size_t)N * 8);
    f.off_cn0 = o;    o = align_up(o + (size_t)N * 8);
    f.off_cnx = o;    o = align_up(o + (size_t)N * 8);
    f.off_t0 = o;     o = align_up(o + (quantised ? 0 : len * esize));
    f.off_W = o;      o = align_up(o + (size_t)N * K * 8);
    f.off_sig = o;    o = align_up(o + (size_t)K * 8);
    f.total_base = o;
    if (q0) {
        f.off_q0 = o;     o = align_up(o + (size_t)N * K * 4);
        f.off_flw = o;    o = align_up(o + first_loadings_bytes(M, N, K));
    }
    f.total = o;
    return f;
}

// FP64 panels hold 2 rows per 16 bytes, so twice the registers per column:
// the single-pass path takes N <= 8192 (N <= 4096 for FP64).  Quantised data
// always runs it.
bool use_fused(const gspca_problem *pr, const gspca_options *op)
{
    if (op->algo == GSPCA_GS && op->reorth != GSPCA_REORTH_CGS)
        return false; // t and p are formed explicitly on the two-pass path
    return pr->N <= (pr->dtype == GSPCA_F64 ? kFusedMaxN / 2 : kFusedMaxN);
}

template <int FM>
gspca_status fit_fused(const gspca_problem *pr, const gspca_options *op, const gspca_result *rs,
                       void *ws, size_t ws_bytes, hipStream_t s)
{
    using E = typename FmtElem<FM>::type;
    using L = Launch<E>;
    using F = Fused<FM>;
    constexpr bool quantised = FM == kFmtBF16 || FM == kFmtFP8;
    const int64_t M = pr->M, N = pr->N, K = pr->K;
    const bool want_q0 = first_loadings_apply(pr, op);
    const FusedPlan f = make_fused_plan(M, N, K, FM, device_cu_count(), want_q0);
    // the up-front first loadings need their own workspace; without it the
    // fit forms each first loading with a pass, as for any other start
    const bool use_q0 = want_q0 && ws && ws_bytes >= f.total;
    if (!ws || ws_bytes < f.total_base)
        return GSPCA_EWORKSPACE;
    if (((uintptr_t)ws) % kAlign)
        return GSPCA_EINVAL;
    unsigned char *base = static_cast<unsigned char *>(ws);
    LoopState *st = reinterpret_cast<LoopState *>(base + f.off_state);
    unsigned char *A = quantised ? const_cast<unsigned char *>(static_cast<const unsigned char *>(pr->X))
                                 : base + f.off_A;
    E *tE = reinterpret_cast<E *>(base + f.off_tE);
    double *td = reinterpret_cast<double *>(base + f.off_td);
    double *tsq = reinterpret_cast<double *>(base + f.off_tsq);
    E *qpart = reinterpret_cast<E *>(base + f.off_qpart);
    double *dvec = reinterpret_cast<double *>(base + f.off_d);
    double *cvec = reinterpret_cast<double *>(base + f.off_c);
    double *qy = reinterpret_cast<double *>(base + f.off_qy);
    double *p = reinterpret_cast<double *>(base + f.off_p);
    double *pprev = reinterpret_cast<double *>(base + f.off_pprev);
    double *cpart = reinterpret_cast<double *>(base + f.off_cpart);
    double *sq = reinterpret_cast<double *>(base + f.off_sq);
    double *cnpart = reinterpret_cast<double *>(base + f.off_cnpart);
    double *cn = reinterpret_cast<double *>(base + f.off_cn);
    double *cn0 = reinterpret_cast<double *>(base + f.off_cn0);
    double *cnx = reinterpret_cast<double *>(base + f.off_cnx);
    E *t0next = reinterpret_cast<E *>(base + f.off_t0);
    double *W = reinterpret_cast<double *>(base + f.off_W);
    double *sig = reinterpret_cast<double *>(base + f.off_sig);
    E *T = static_cast<E *>(rs->T);
    E *P = static_cast<E *>(rs->P);
    const E *T0 = static_cast<const E *>(op->T0);
    const float *scale = pr->col_scale;
    const double tiny = FM == kFmtF64 ? DBL_MIN : (double)FLT_MIN;
    const int gs = op->algo == GSPCA_GS;
    const int implicit = (op->implicit_deflation || quantised) ? 1 : 0;
    const double tol = op->tol;
    const int stop = op->stop;

    std::vector<int32_t> rit;
    const bool replay = op->replay_iters != nullptr;
    if (replay) {
        rit.resize(K);
        if (hipMemcpy(rit.data(), op->replay_iters, K * sizeof(int32_t), hipMemcpyDeviceToHost) !=
            hipSuccess)
            return GSPCA_EDEVICE;
        for (int64_t k = 0; k < K; ++k)
            if (rit[k] < 0)
                return GSPCA_EINVAL;
    }

    gspca_profile *prof = op->profile;
    constexpr int kMaxBatch = 64;
    std::vector<hipEvent_t> ev;
    struct EventPool {
        std::vector<hipEvent_t> *v;
        ~EventPool() { for (hipEvent_t e : *v) (void)hipEventDestroy(e); }
    } ev_guard{&ev};
    if (prof) {
        ev.resize(2 * kMaxBatch);
        for (auto &e : ev)
            if (hipEventCreate(&e) != hipSuccess)
                return GSPCA_EDEVICE;
        prof->bytes_per_pass = (int64_t)(M * N * (int64_t)(16 / f.PR));
        prof->single_pass = 1;
    }

    LoopState h{};
    auto read_state = [&]() -> bool {
        if (hipMemcpyAsync(&h, st, sizeof(LoopState), hipMemcpyDeviceToHost, s) != hipSuccess)
            return false;
        return hipStreamSynchronize(s) == hipSuccess;
    };

    reset_state(st, s);
    if constexpr (!quantised) {
        F::retile(static_cast<const E *>(pr->X), pr->ldx, M, N, f.NP, f.ldp, A, st, s);
        if (!read_state())
            return GSPCA_EDEVICE;
        if (h.nonfinite)
            return GSPCA_ENONFINITE;
    }
    F::deflate(A, N, f.NP, f.ldp, nullptr, nullptr, 0, scale, f.nsplit_cn, cnpart, s);
    F::colnorm_finish(cnpart, f.nsplit_cn, N, cn0, cn, 0, 0, P, W, sig, s);
    E *Q0 = use_q0 ? reinterpret_cast<E *>(base + f.off_q0) : nullptr;
    if constexpr (FM == kFmtF32) {
        if (use_q0)
            launch_first_loadings(static_cast<const float *>(pr->X), pr->ldx, M, N, T0, K, Q0,
                                  base + f.off_flw, s);
    }

    auto start_args = [&](int64_t k) {
        const int32_t lim = replay ? rit[k] : op->max_iter;
        return StartArgs{(int32_t)k, op->init, (replay && lim < 1) ? 1 : 0, gs ? 1 : 0,
                         op->replay_start_col};
    };
    // explicit deflation: the start and first loading of component k + 1 are
    // formed with the deflation that ends component k (k_deflate_first)
    bool started = false;
    for (int64_t k = 0; k < K; ++k) {
        const int32_t limit = replay ? rit[k] : op->max_iter;
        const int kg = gs ? (int)k : 0;
        // the source of the first loading's q: the pass's partials, or column
        // k of Q0 when the given start was taken (implicit: R^T t0 = X^T t0)
        const E *q_first = qpart;
        int64_t g_first = f.G;
        if (!started) {
            // the start's scratch (given-start products) shares cpart, idle here
            F::start(A, N, f.NP, f.ldp, M, scale, implicit, T, P, sig, cn, T0, start_args(k),
                     tiny, tE, cpart, st, s);
            bool from_q0 = false;
            if (use_q0) {
                if (!read_state())
                    return GSPCA_EDEVICE;
                from_q0 = h.start_col < 0 && !h.done && !h.degenerate;
            }
            if (from_q0) {
                q_first = Q0 + k * N;
                g_first = 1;
            } else {
                // first loading of the component: p = R^T t0, Gram-Schmidt, norm
                F::pass(1, f.cpt, f.G, f.NT, f.plds, f.skew, f.pipe, A, N, f.NP, f.ldp, M,
                        scale, p, tE, td, tsq, qpart, st, s);
            }
        }
        started = false;
        // the loading side: one workgroup when N and the partials are small
        // (no cross-workgroup reductions; at most 256 KiB of partials, which
        // one workgroup reads in a few microseconds -- 512 x 256 FP64: 122 ->
        // 95 ms per fit, while 2 MiB at 2000 x 1000 made it slower), else the
        // column-parallel reduction and apply kernels
        const bool one_wg =
            N <= kFinApplyMaxN && (int64_t)f.G * N * (int64_t)sizeof(E) <= (int64_t)256 * 1024;
        auto loading_side = [&](int kdv, int it, const E *qsrc, int64_t gsrc) {
            if (one_wg) {
                F::fin_apply(qsrc, gsrc, N, W, kdv, dvec, P, kg, qy, p, pprev, st, it, stop, tiny,
                             s);
            } else {
                F::fin_q(qsrc, gsrc, N, W, kdv, dvec, P, kg, qy, cpart, cvec, st, it, s);
                L::gs_apply(qy, 1, N, N, qy, P, N, kg, cvec, p, pprev, nullptr, sq, st, 0, tol,
                            limit, replay, tiny, stop, s);
            }
        };
        loading_side(0, 0, q_first, g_first);
        // both sides of an iteration in one workgroup launch when each fits
        const bool score_fin = one_wg && F::score_fin_fits(M, kg);
        int32_t enq = 0;
        int batch = 4;
        bool have = false;
        int32_t iter_before = 0;
        while (enq < limit) {
            const int n = std::min<int32_t>(std::min(batch, kMaxBatch), limit - enq);
            for (int i = 0; i < n; ++i) {
                const int it = enq + i + 1;
                if (prof)
                    (void)hipEventRecord(ev[2 * i], s);
                F::pass(0, f.cpt, f.G, f.NT, f.plds, f.skew, f.pipe, A, N, f.NP, f.ldp, M, scale, p,
                        tE, td, tsq, qpart, st, s);
                if (prof)
                    (void)hipEventRecord(ev[2 * i + 1], s);
                // score side: d = V_(k)^T t (coalesced over the rows, kept out of
                // the streaming pass), sigma = |t - V d| and the stop test; t - V d
                // itself is formed once, when the component ends
                if (score_fin) {
                    F::score_fin(td, M, T, kg, tsq, f.G, cpart, dvec, tol, limit, replay, qpart,
                                 f.G, N, W, P, kg, qy, p, pprev, st, it, stop, tiny, s);
                } else {
                    F::score_dot(td, M, T, kg, tsq, f.G, cpart, dvec, st, tol, limit, replay,
                                 tiny, stop, s);
                    loading_side(gs ? kg : 0, it, qpart, f.G);
                }
            }
            enq += n;
            if (!read_state())
                return GSPCA_EDEVICE;
            have = true;
            if (prof) {
                const int real = std::min(n, h.iter - iter_before);
                for (int i = 0; i < real; ++i) {
                    float a_ms = 0.f;
                    if (hipEventElapsedTime(&a_ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) {
                        prof->pass_ms += a_ms;
                        prof->pass_launches += 1;
                    }
                }
                prof->iterations += std::max(0, h.iter - iter_before);
                iter_before = h.iter;
            }
            if (h.done)
                break;
            batch = next_batch(h, tol, batch);
        }
        if (!have && !read_state())
            return GSPCA_EDEVICE;
        if (h.degenerate)
            L::degenerate_p(P, N, (int)k, p, st, s);
        F::comp_end(td, dvec, kg, tE, M, N, p, qy, (int)k, gs, implicit ? 0 : 1, T, P,
                    gs ? W : nullptr, sig, rs->iters, rs->start_col, st, s);
        if (k + 1 < K) {
            if (!implicit) {
                // next start on the norms this deflation leaves (predicted from
                // the exact ones before it), its column taken from R - t p_k^T;
                // then the deflation, the exact new norms and the first
                // loading R'^T t0 in one read and write of R
                F::colnorm_predict(cn, N, P + k * N, qy, st, cnx, s);
                F::start(A, N, f.NP, f.ldp, M, scale, 0, T, P, sig, cnx, T0, start_args(k + 1),
                         tiny, t0next, cpart, st, s, tE, P + k * N);
                F::deflate_first(A, N, f.NP, f.ldp, tE, P + k * N, h.degenerate ? 0 : 1, t0next,
                                 f.G, cnpart, qpart, s);
                F::colnorm_finish(cnpart, f.G, N, nullptr, cn, 0, 0, P, W, sig, s);
                started = true;
            } else {
                F::colnorm_finish(nullptr, 1, N, cn0, cn, 1, (int)k + 1, P, W, sig, s);
            }
        }
    }
    L::finalize_all(T, M, (int)K, sig, rs->lambda, rs->sigma, gs, s);
    if (!read_state())
        return GSPCA_EDEVICE;
    if (hipGetLastError() != hipSuccess)
        return GSPCA_EDEVICE;
    return h.not_converged ? GSPCA_NOT_CONVERGED : GSPCA_OK;
}

size_t workspace_for(const gspca_problem *pr, const gspca_options *op)
{
    if (use_fused(pr, op))
        return make_fused_plan(pr->M, pr->N, pr->K, fmt_of(pr->dtype), device_cu_count(),
                               first_loadings_apply(pr, op))
            .total;
    return make_plan(pr->M, pr->N, pr->K, dtype_size(pr->dtype)).total;
}

}  // namespace

extern "C" {

void gspca_default_options(gspca_options *opt)
{
    if (!opt)
        return;
    memset(opt, 0, sizeof(*opt));
    opt->algo = GSPCA_GS;
    opt->init = GSPCA_INIT_MAXNORM;
    opt->tol = 1e-7;
    opt->max_iter = 10000;
}

size_t gspca_workspace_bytes(const gspca_problem *prob, const gspca_options *opt)
{
    if (validate(prob, opt) != GSPCA_OK)
        return 0;
    return workspace_for(prob, opt);
}

gspca_status gspca_fit_ex(const gspca_problem *prob, const gspca_options *opt,
                          const gspca_result *res, void *ws, size_t ws_bytes, void *stream)
{
    gspca_status v = validate(prob, opt);
    if (v != GSPCA_OK)
        return v;
    if (!res || !res->T || !res->P || !res->lambda)
        return GSPCA_EINVAL;
    if (!ws || ws_bytes < workspace_for(prob, opt))
        return GSPCA_EWORKSPACE;
    if (((uintptr_t)ws) % kAlign)
        return GSPCA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    // the fit reads its loop state back to the host: refuse graph capture
    const int cap = stream_capturing(s);
    if (cap != 0)
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;
    if (use_fused(prob, opt)) {
        switch (prob->dtype) {
        case GSPCA_F64: return fit_fused<kFmtF64>(prob, opt, res, ws, ws_bytes, s);
        case GSPCA_F32: return fit_fused<kFmtF32>(prob, opt, res, ws, ws_bytes, s);
        case GSPCA_BF16: return fit_fused<kFmtBF16>(prob, opt, res, ws, ws_bytes, s);
        default: return fit_fused<kFmtFP8>(prob, opt, res, ws, ws_bytes, s);
        }
    }
    return prob->dtype == GSPCA_F64 ? fit_two_pass<double>(prob, opt, res, ws, ws_bytes, s)
                                    : fit_two_pass<float>(prob, opt, res, ws, ws_bytes, s);
}

static gspca_status fit_alloc(int32_t dtype, const void *X, int64_t M, int64_t N, int64_t K,
                              double tol, int32_t max_iter, void *T, void *P, double *lambda,
                              void *stream)
{
    gspca_problem pr{dtype, X, M, M, N, K, nullptr};
    gspca_options op;
    gspca_default_options(&op);
    op.tol = tol;
    op.max_iter = max_iter;
    gspca_result rs{T, P, lambda, nullptr, nullptr, nullptr};
    gspca_status v = validate(&pr, &op);
    if (v != GSPCA_OK)
        return v;
    if (!T || !P || !lambda)
        return GSPCA_EINVAL;
    const int cap = stream_capturing(static_cast<hipStream_t>(stream));
    if (cap != 0) // blocking, and allocates: never under capture
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;
    const size_t bytes = gspca_workspace_bytes(&pr, &op);
    void *ws = nullptr;
    if (hipMalloc(&ws, bytes) != hipSuccess)
        return GSPCA_ENOMEM;
    gspca_status r = gspca_fit_ex(&pr, &op, &rs, ws, bytes, stream);
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess && r >= 0)
        r = GSPCA_EDEVICE;
    if (hipFree(ws) != hipSuccess && r >= 0)
        r = GSPCA_EDEVICE;
    return r;
}

gspca_status gspca_fit(const double *X, int64_t M, int64_t N, int64_t K, double tol,
                       int32_t max_iter, double *T, double *P, double *lambda, void *stream)
{
    return fit_alloc(GSPCA_F64, X, M, N, K, tol, max_iter, T, P, lambda, stream);
}

gspca_status gspca_fit_f32(const float *X, int64_t M, int64_t N, int64_t K, double tol,
                           int32_t max_iter, float *T, float *P, double *lambda, void *stream)
{
    return fit_alloc(GSPCA_F32, X, M, N, K, tol, max_iter, T, P, lambda, stream);
}

size_t gspca_quantized_bytes(int64_t M, int64_t N, int32_t dtype)
{
    if (!is_quantised(dtype) || M < 1 || N < 1 || N > 8192 || M > (int64_t(1) << 30))
        return 0;
    int cpt = 0, NT = 0;
    int64_t ldp = 0;
    panel_width(N, &cpt, &NT, &ldp);
    return (size_t)cdiv(M, fmt_rows(fmt_of(dtype))) * (size_t)ldp * 16;
}

gspca_status gspca_quantize(const float *X, int64_t M, int64_t N, int64_t ldx, int32_t dtype,
                            void *Q, float *col_scale, void *ws, size_t ws_bytes, void *stream)
{
    if (!X || !Q || !col_scale || ldx < M || gspca_quantized_bytes(M, N, dtype) == 0)
        return GSPCA_EINVAL;
    if (!ws || ws_bytes < sizeof(LoopState))
        return GSPCA_EWORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cap = stream_capturing(s);
    if (cap != 0) // reads the non-finite flag back: blocking
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;
    LoopState *st = static_cast<LoopState *>(ws);
    int cpt = 0, NT = 0;
    int64_t ldp = 0;
    panel_width(N, &cpt, &NT, &ldp);
    const int fmt = fmt_of(dtype);
    const int64_t NP = cdiv(M, fmt_rows(fmt));
    unsigned char *q = static_cast<unsigned char *>(Q);
    reset_state(st, s);
    if (fmt == kFmtBF16)
        Fused<kFmtBF16>::quantize(X, ldx, M, N, NP, ldp, col_scale, q, st, s);
    else
        Fused<kFmtFP8>::quantize(X, ldx, M, N, NP, ldp, col_scale, q, st, s);
    int32_t bad = 0;
    if (hipMemcpyAsync(&bad, &st->nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GSPCA_EDEVICE;
    return bad ? GSPCA_ENONFINITE : GSPCA_OK;
}

const char *gspca_status_string(int status)
{
    switch (status) {
    case GSPCA_OK: return "ok";
    case GSPCA_NOT_CONVERGED: return "not converged (max_iter reached)";
    case GSPCA_EINVAL: return "invalid argument";
    case GSPCA_EWORKSPACE: return "workspace too small";
    case GSPCA_EDEVICE: return "HIP runtime error";
    case GSPCA_ENONFINITE: return "X holds NaN or Inf";
    case GSPCA_ENOMEM: return "device allocation failed";
    default: return "unknown status";
    }
}

int gspca_version(void) { return 200; }

}  // extern "C"
