// Allocation-free variant of the exclusive scan entry point, for callers that
// cannot allocate device memory (code under stream capture, tight serving
// loops, harnesses that forbid allocation). Its scratch (the per-block sums of
// the reduce-then-scan) lives in a file-scope device array instead of a
// context workspace. Each GPU holds its own copy of the array until the
// process ends; every call on that GPU shares it, so calls that overlap on one
// GPU race (the caller orders them, e.g. on one stream).
#include <hip/hip_runtime.h>

#include "kernels.h"
#include "runtime.h"

namespace swf {

// Block sums of one scan: at most one per scan block plus one (the scan grid
// is capped at 4096 blocks, so every n fits).
constexpr int kNoAllocScanSums = 4096 + 8;
static __device__ __align__(256) uint64_t scratch[kNoAllocScanSums];

// Device address of `scratch` on the context's device (the host-side name is
// only a stand-in). Called once per context at creation, with its device
// current.
swf_status noalloc_setup(Ctx* c) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return c->hip(e == hipSuccess ? hipErrorInvalidSymbol : e, "hipGetSymbolAddress(scratch)");
    c->noalloc_scratch = p;
    return SWF_OK;
}

}  // namespace swf

using namespace swf;

extern "C" swf_status swf_exclusive_scan_noalloc(swf_ctx* h, const uint32_t* counts, uint32_t* offsets,
                                                 uint64_t* total, int64_t n, void* stream) {
    Ctx* c = reinterpret_cast<Ctx*>(h);
    if (!c) return SWF_E_INVALID;
    std::lock_guard<std::recursive_mutex> lock(c->mu);
    hipSetDevice(c->device);
    if (n < 0 || !total || (n > 0 && (!counts || !offsets))) return c->fail(SWF_E_INVALID, "bad arguments");
    if (!c->noalloc_scratch) return c->fail(SWF_E_STATE, "scratch address not set up");
    if (scan_scratch_bytes(n) > sizeof(uint64_t) * kNoAllocScanSums)
        return c->fail(SWF_E_OVERFLOW, "scan needs more block sums than the static scratch holds");
    launch_exclusive_scan(counts, offsets, total, n, c->noalloc_scratch, (hipStream_t)stream);
    return c->hip(hipGetLastError(), "scan");
}
