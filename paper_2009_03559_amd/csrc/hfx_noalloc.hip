// Exchange build that allocates no device memory, for callers that cannot
// call hipMalloc (code under stream capture, tight serving loops, harnesses
// that forbid allocation).
//
// The only device memory a build needs beyond the caller's P and K and the
// handle's resident data is a small fixed workspace: the per-block partial
// maxima of the P symmetry check and the quartet counters.  Here it lives in
// the file-scope array `scratch` (one copy per GPU, held until the process
// ends).  Its device address is looked up once per device with
// hipGetSymbolAddress and used everywhere host code needs it; the array's
// name itself is only a host-side stand-in.
//
// Every call on one GPU shares that GPU's copy, and the array keeps the last
// call's contents: the counters are cleared by a fill kernel at the start of
// each call that asks for statistics, the check's partial maxima are written
// whole by their kernel.  Calls that overlap in time on one GPU (two host
// threads, or two streams without ordering) race on it.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "hfx.h"
#include "hfx_internal.hpp"

namespace hfx {

constexpr size_t NOALLOC_PART_BYTES = 2 * PCHECK_BLOCKS * sizeof(double);
constexpr size_t NOALLOC_COUNT_BYTES = NCOUNT * sizeof(unsigned long long);
constexpr size_t NOALLOC_SCRATCH_BYTES = (NOALLOC_PART_BYTES + NOALLOC_COUNT_BYTES + 255) / 256 * 256;
static_assert(NOALLOC_SCRATCH_BYTES == HFX_NOALLOC_SCRATCH_BYTES, "header and workspace layout disagree");

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_dev;  // device address of `scratch`, per device

// Device address of this device's `scratch` (looked up on the first call on
// each device, with that device current).
static hfx_status scratch_address(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(HFX_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(HFX_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return HFX_OK;
}

}  // namespace hfx

using namespace hfx;

extern "C" hfx_status hfx_build_K_noalloc(hfx_pairs p, const double *P_dev, double *K_dev, int64_t ld,
                                          const hfx_opts *o, void *stream, hfx_stats *st_or_null) {
    // the workspace does not grow with the system: a P check of any size
    // uses at most PCHECK_BLOCKS blocks, and there are NCOUNT counters
    if (NOALLOC_PART_BYTES + NOALLOC_COUNT_BYTES > NOALLOC_SCRATCH_BYTES)
        return fail(HFX_EUNSUPPORTED, "build workspace larger than the static scratch array");
    void *base = nullptr;
    hfx_status s = scratch_address(&base);
    if (s != HFX_OK) return s;
    const Workspace ws{(double *)base, (unsigned long long *)((char *)base + NOALLOC_PART_BYTES)};
    return build_K_impl(p, P_dev, K_dev, ld, o, 0, 1, stream, st_or_null, nullptr, &ws);
}
