// The one entry point for callers that cannot allocate device memory (code under HIP
// graph capture, tight serving loops, harnesses that forbid allocation): the FP64 inner
// product / squared norm of dwf_cdot / dwf_norm2, written to caller-owned device memory
// without synchronising, with the per-workgroup partial sums in a static device array
// instead of the context's reduction buffer.
//
// `scratch` below is a device symbol: in host code its name is only a stand-in, so the
// host never passes it to a kernel.  dwf_create calls noalloc_setup once per device (with
// that device current), which resolves the array's device address with
// hipGetSymbolAddress and keeps it per device; the entry point passes that address to the
// reduction kernels.  Every call on one GPU shares that GPU's array: calls that overlap on
// one GPU (different streams, or host threads) race on it.  Each call overwrites every
// partial it reads, so nothing has to start at zero.
#include <mutex>

#include "dwf_common.h"

namespace dwf {

// (re, im) partial of each workgroup of the fixed reduction grid: 16 KiB per GPU, held
// until the process ends.
constexpr int kScratchDoubles = 2 * kRedBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double *g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each GPU

int noalloc_setup(int device) {
    if (device < 0 || device >= kMaxDevices) return fail(DWF_EUNSUP, "noalloc_setup: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_dev[device]) return DWF_OK;
    int cur = -1;
    DWF_HIP(hipGetDevice(&cur));
    if (cur != device) return fail(DWF_EHIP, "noalloc_setup: the device is not current");
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (p == nullptr) return fail(DWF_EHIP, "noalloc_setup: null address for the scratch array");
    g_scratch_dev[device] = static_cast<double *>(p);
    return DWF_OK;
}

static double *scratch_of(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_dev[device];
}

}  // namespace dwf

using namespace dwf;

extern "C" int dwf_cdot_noalloc(dwf_ctx ctx, double *result, const void *x, const void *y, int full, int prec,
                                void *stream) {
    if (!ctx) return fail(DWF_EINVAL, "dwf_cdot_noalloc: null context");
    if (!result || !x) return fail(DWF_EINVAL, "dwf_cdot_noalloc: null pointer");
    if (prec < DWF_F64 || prec > DWF_BF16) return fail(DWF_EINVAL, "dwf_cdot_noalloc: bad precision");
    if (full != 0 && full != 1) return fail(DWF_EINVAL, "dwf_cdot_noalloc: full must be 0 or 1");
    // the reduction writes one (re, im) pair per workgroup of its fixed grid
    if (2 * (long)kRedBlocks > (long)kScratchDoubles)
        return fail(DWF_EINVAL, "dwf_cdot_noalloc: the reduction's partials exceed the static scratch");
    double *partials = scratch_of(ctx->device);
    if (!partials) return fail(DWF_EUNSUP, "dwf_cdot_noalloc: scratch not set up on this device");
    const long n = ctx->g.half * ctx->g.Ls * 12 * (full ? 2 : 1);  // complex elements
    return launch_reduce(partials, result, x, y, n, prec, y != nullptr, (hipStream_t)stream);
}
