// noalloc.hip -- gspca_fit_noalloc: the fit of gspca_fit_ex with its
// workspace taken from a fixed device array of the library instead of a
// caller buffer, for callers that cannot allocate device memory.
//
// `scratch` is a file-scope device array; every GPU the library runs on holds
// its own copy until the process ends.  In host code its name is only a
// host-side stand-in, so the device address of each GPU's copy is looked up
// once per device (hipGetSymbolAddress with that device current) and kept in
// `g_scratch`; kernels receive that address as their workspace argument.
#include <mutex>

#include "../../include/gspca.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = GSPCA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (nullptr on failure).
void *scratch_ptr(int dev)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return nullptr;
        g_scratch[dev] = p;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" {

size_t gspca_noalloc_scratch_bytes(void) { return kScratchBytes; }

gspca_status gspca_fit_noalloc(const gspca_problem *prob, const gspca_options *opt,
                               const gspca_result *res, void *stream)
{
    // the variant reads nothing back beyond the loop state and creates no
    // events: replayed counts and per-kernel profiles are refused
    if (opt && (opt->replay_iters || opt->replay_start_col || opt->profile))
        return GSPCA_EINVAL;
    const size_t need = gspca_workspace_bytes(prob, opt);
    if (need == 0)
        return GSPCA_EINVAL;
    if (need > kScratchBytes)
        return GSPCA_EWORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return GSPCA_EDEVICE;
    void *ws = scratch_ptr(dev);
    if (!ws)
        return GSPCA_EDEVICE;
    return gspca_fit_ex(prob, opt, res, ws, kScratchBytes, stream);
}

}  // extern "C"
