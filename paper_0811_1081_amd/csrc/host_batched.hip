// host_batched.hip -- C ABI of the batched GS-PCA fits: validation, the
// descriptor table, the launch plan and its autotuner (see batched.hip).
#include <float.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/gspca.h"
#include "internal.h"

using namespace gspca;

namespace {

constexpr uint64_t kPlanMagic = 0x67737063615f6274ull; // "gspca_bt"
constexpr size_t kAlignB = 256;
inline size_t align_b(size_t x) { return (x + kAlignB - 1) / kAlignB * kAlignB; }

struct PlanImpl {
    uint64_t magic;
    BatchItem *items;
    int32_t *order;
    uint32_t *queue;
    int32_t nprob;
    int32_t threads;
    int32_t occ; // workgroups per compute unit
    int32_t ncu;
    size_t lds;
    BatchArgs args;
    int64_t sig[4]; // batch signature for the tune cache
};
static_assert(sizeof(PlanImpl) <= sizeof(gspca_batch_plan), "plan too large");

struct Layout {
    size_t off_items, off_order, off_queue, off_W, total;
};

Layout layout(const gspca_batch_problem *probs, int32_t n)
{
    Layout L{};
    size_t o = 0;
    L.off_queue = o;  o = align_b(o + 256);
    L.off_items = o;  o = align_b(o + (size_t)n * sizeof(BatchItem));
    L.off_order = o;  o = align_b(o + (size_t)n * sizeof(int32_t));
    L.off_W = o;
    for (int32_t i = 0; i < n; ++i)
        o = align_b(o + (size_t)probs[i].N * (size_t)probs[i].K * 8);
    L.total = o;
    return L;
}

bool valid_problem(const gspca_batch_problem &p)
{
    if (!p.X || !p.T || !p.P || !p.lambda)
        return false;
    if (p.M < 1 || p.N < 1 || p.K < 1 || p.K > p.M || p.K > p.N || p.K > 64 || p.ldx < p.M)
        return false;
    return p.M <= 4096 && p.N <= 1024;
}

int cu_count()
{
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cu < 1)
        cu = 256;
    return cu;
}

int max_occupancy(size_t lds)
{
    const size_t budget = 160 * 1024 - 4096; // LDS per compute unit, minus static arrays
    const int occ = (int)std::min<size_t>(4, budget / std::max<size_t>(lds, 1));
    return std::max(occ, 1);
}

void launch_plan(const PlanImpl *pl, hipStream_t s)
{
    batched_launch(pl->items, pl->nprob, pl->order, pl->queue, pl->args, pl->ncu * pl->occ,
                   pl->threads, pl->occ, pl->lds, s);
}

// ---- tune cache: one JSON object per line,
//      {"key":"n,sumMN,maxM,maxN,cus,version","threads":T,"occ":O,"ms":X}
// The key carries the compute-unit count and the library version, so an
// entry measured on another device or another build of the kernel is not
// reused.
void cache_key(const PlanImpl *pl, char *buf, size_t n)
{
    snprintf(buf, n, "%lld,%lld,%lld,%lld,%d,%d", (long long)pl->sig[0], (long long)pl->sig[1],
             (long long)pl->sig[2], (long long)pl->sig[3], pl->ncu, gspca_version());
}

// The shapes the tuner measures: whole 64-lane waves, at most 1024 threads
// (k_batched's launch bound), at most 32 waves per compute unit, and no more
// workgroups per compute unit than the problems' LDS allows.
bool valid_shape(int threads, int occ, size_t lds)
{
    const bool t_ok = threads == 256 || threads == 512 || threads == 1024;
    return t_ok && occ >= 1 && threads * occ <= 2048 && occ <= max_occupancy(lds);
}

bool cache_lookup(const PlanImpl *pl, int *threads, int *occ)
{
    const char *path = getenv("GSPCA_TUNE_CACHE");
    if (!path || !*path)
        return false;
    FILE *f = fopen(path, "r");
    if (!f)
        return false;
    char key[128], line[512];
    cache_key(pl, key, sizeof key);
    bool found = false;
    while (fgets(line, sizeof line, f)) {
        char k[128];
        int t = 0, o = 0;
        if (sscanf(line, "{\"key\":\"%127[^\"]\",\"threads\":%d,\"occ\":%d", k, &t, &o) == 3 &&
            strcmp(k, key) == 0 && valid_shape(t, o, pl->lds)) {
            *threads = t;
            *occ = o;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const PlanImpl *pl, int threads, int occ, double ms)
{
    const char *path = getenv("GSPCA_TUNE_CACHE");
    if (!path || !*path)
        return;
    FILE *f = fopen(path, "a");
    if (!f)
        return;
    char key[128];
    cache_key(pl, key, sizeof key);
    fprintf(f, "{\"key\":\"%s\",\"threads\":%d,\"occ\":%d,\"ms\":%.4f}\n", key, threads, occ, ms);
    fclose(f);
}

}  // namespace

extern "C" {

size_t gspca_batched_workspace_bytes(const gspca_batch_problem *probs, int32_t nprob)
{
    if (!probs || nprob < 1)
        return 0;
    for (int32_t i = 0; i < nprob; ++i)
        if (!valid_problem(probs[i]))
            return 0;
    return layout(probs, nprob).total;
}

gspca_status gspca_batched_prepare(const gspca_batch_problem *probs, int32_t nprob,
                                   const gspca_options *opt, void *ws, size_t ws_bytes,
                                   gspca_batch_plan *plan, void *stream)
{
    if (!probs || nprob < 1 || !opt || !plan)
        return GSPCA_EINVAL;
    if (opt->algo != GSPCA_GS || (opt->init != GSPCA_INIT_MAXNORM &&
                                  opt->init != GSPCA_INIT_COLUMN_K && opt->init != GSPCA_INIT_GIVEN))
        return GSPCA_EINVAL;
    if (opt->init == GSPCA_INIT_GIVEN)
        for (int32_t i = 0; i < nprob; ++i)
            if (!probs[i].T0)
                return GSPCA_EINVAL;
    if (!(opt->tol >= 0.0) || !isfinite(opt->tol) || opt->max_iter < 1 ||
        (opt->stop != GSPCA_STOP_SIGMA_REL && opt->stop != GSPCA_STOP_LOADING))
        return GSPCA_EINVAL;
    if (opt->reorth != GSPCA_REORTH_CGS) // one classical pass only
        return GSPCA_EINVAL;
    for (int32_t i = 0; i < nprob; ++i)
        if (!valid_problem(probs[i]))
            return GSPCA_EINVAL;
    const Layout L = layout(probs, nprob);
    if (!ws || ws_bytes < L.total)
        return GSPCA_EWORKSPACE;
    if (((uintptr_t)ws) % kAlignB)
        return GSPCA_EINVAL;
    unsigned char *base = static_cast<unsigned char *>(ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cap = stream_capturing(s);
    if (cap != 0) // uploads the table and synchronises: not capturable
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;

    std::vector<BatchItem> items(nprob);
    size_t woff = L.off_W;
    size_t lds = 0;
    int64_t sum_mn = 0, max_m = 0, max_n = 0;
    for (int32_t i = 0; i < nprob; ++i) {
        const gspca_batch_problem &p = probs[i];
        BatchItem &b = items[i];
        b.X = p.X;
        b.ldx = p.ldx;
        b.M = (int32_t)p.M;
        b.N = (int32_t)p.N;
        b.K = (int32_t)p.K;
        b.pad = 0;
        b.T = p.T;
        b.P = p.P;
        b.lambda = p.lambda;
        b.sigma = p.sigma;
        b.iters = p.iters;
        b.start_col = p.start_col;
        b.replay_iters = p.replay_iters;
        b.replay_start = p.replay_start_col;
        b.status = p.status;
        b.T0 = opt->init == GSPCA_INIT_GIVEN ? p.T0 : nullptr;
        b.W = reinterpret_cast<double *>(base + woff);
        woff = align_b(woff + (size_t)p.N * (size_t)p.K * 8);
        lds = std::max(lds, batched_lds_bytes(p.M, p.N, p.K));
        sum_mn += p.M * p.N;
        max_m = std::max<int64_t>(max_m, p.M);
        max_n = std::max<int64_t>(max_n, p.N);
    }
    {
        int dev = 0, lds_max = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                hipSuccess)
            return GSPCA_EDEVICE;
        if (lds + 1024 > (size_t)lds_max) // the problems' vectors must fit one workgroup's LDS
            return GSPCA_EINVAL;
    }
    std::vector<int32_t> order(nprob);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return probs[a].M * probs[a].N > probs[b].M * probs[b].N;
    });
    if (hipMemcpyAsync(base + L.off_items, items.data(), items.size() * sizeof(BatchItem),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(base + L.off_order, order.data(), order.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return GSPCA_EDEVICE;

    PlanImpl pl{};
    pl.magic = kPlanMagic;
    pl.items = reinterpret_cast<BatchItem *>(base + L.off_items);
    pl.order = reinterpret_cast<int32_t *>(base + L.off_order);
    pl.queue = reinterpret_cast<uint32_t *>(base + L.off_queue);
    pl.nprob = nprob;
    pl.threads = 256;
    pl.lds = lds;
    pl.occ = max_occupancy(lds);
    pl.ncu = cu_count();
    pl.args.tol = opt->tol;
    pl.args.tiny = (double)FLT_MIN;
    pl.args.max_iter = opt->max_iter;
    pl.args.init = opt->init;
    pl.args.stop = opt->stop;
    pl.sig[0] = nprob;
    pl.sig[1] = sum_mn;
    pl.sig[2] = max_m;
    pl.sig[3] = max_n;
    int t = 0, o = 0;
    if (cache_lookup(&pl, &t, &o)) {
        pl.threads = t;
        pl.occ = o;
    }
    memset(plan, 0, sizeof(*plan));
    memcpy(plan->opaque, &pl, sizeof pl);
    return GSPCA_OK;
}

gspca_status gspca_batched_launch(const gspca_batch_plan *plan, void *stream)
{
    if (!plan)
        return GSPCA_EINVAL;
    PlanImpl pl;
    memcpy(&pl, plan->opaque, sizeof pl);
    if (pl.magic != kPlanMagic)
        return GSPCA_EINVAL;
    launch_plan(&pl, static_cast<hipStream_t>(stream));
    return hipGetLastError() == hipSuccess ? GSPCA_OK : GSPCA_EDEVICE;
}

gspca_status gspca_batched_tune(gspca_batch_plan *plan, void *stream)
{
    if (!plan)
        return GSPCA_EINVAL;
    PlanImpl pl;
    memcpy(&pl, plan->opaque, sizeof pl);
    if (pl.magic != kPlanMagic)
        return GSPCA_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int cap = stream_capturing(s);
    if (cap != 0) // times launches with host-side event waits
        return cap > 0 ? GSPCA_EINVAL : GSPCA_EDEVICE;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return GSPCA_EDEVICE;
    const int occ_max = max_occupancy(pl.lds);
    double best_ms = INFINITY;
    int best_t = pl.threads, best_o = pl.occ;
    gspca_status st = GSPCA_OK;
    for (int threads : {256, 512, 1024}) {
        for (int occ = 1; occ <= occ_max; ++occ) {
            if (!valid_shape(threads, occ, pl.lds))
                continue;
            PlanImpl c = pl;
            c.threads = threads;
            c.occ = occ;
            launch_plan(&c, s); // warm-up
            float ms = 0.f;
            if (hipEventRecord(e0, s) != hipSuccess) { st = GSPCA_EDEVICE; break; }
            launch_plan(&c, s);
            if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = GSPCA_EDEVICE;
                break;
            }
            if (ms < best_ms) {
                best_ms = ms;
                best_t = threads;
                best_o = occ;
            }
        }
        if (st != GSPCA_OK)
            break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GSPCA_OK)
        return st;
    pl.threads = best_t;
    pl.occ = best_o;
    cache_store(&pl, best_t, best_o, best_ms);
    memcpy(plan->opaque, &pl, sizeof pl);
    return GSPCA_OK;
}

}  // extern "C"
