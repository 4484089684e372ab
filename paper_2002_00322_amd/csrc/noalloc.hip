// Grouped build without any device allocation: the same launches as
// esmf_fock_build, with the build workspace (unit table, operand tiles,
// partial tiles) in a fixed static array of device memory instead of the
// handle's own allocation.  For callers that cannot allocate (code under
// stream capture, tight serving loops, harnesses that forbid hipMalloc).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>
#include <vector>

#include "internal.h"

namespace {

// The workspace of builds that allocate nothing, one copy per device (held
// from the library's load until the process ends).  In host code `scratch`
// names a host-side stand-in, not device memory: its device address comes
// from hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // device address of `scratch`, per device

hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= device) g_scratch_ptr.resize(device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

}  // namespace

extern "C" esmf_status esmf_fock_build_noalloc(esmf_eri_t eri, int32_t m, const double* d, double* j, double* k,
                                               esmf_precision prec, void* hip_stream) {
    using namespace esmf;
    clear_error();
    const Handle* h = (const Handle*)eri;
    esmf_status st = check_build_args(h, m, d, j, k, prec);
    if (st != ESMF_OK) return st;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    if (dev != h->device) return fail(ESMF_ERR_INVALID_ARG, "the handle belongs to another device than the current one");
    const int mode = build_mode(*h, prec);
    KernelVariant v = default_variant(mode);
    {
        std::lock_guard<std::mutex> lk(h->ws_mu);
        if (h->has_tuned[(int)prec]) v = h->tuned[(int)prec];
    }
    const size_t need = build_workspace_bytes(*h, m, nullptr, v);
    if (need > kScratchBytes) {
        char msg[200];
        snprintf(msg, sizeof msg, "the build needs %.1f MiB of workspace; the static scratch holds %.1f MiB",
                 need / 1048576.0, kScratchBytes / 1048576.0);
        return fail(ESMF_ERR_INVALID_ARG, msg);
    }
    void* ws = nullptr;
    e = scratch_address(dev, &ws);
    if (e != hipSuccess) return device_fail(e, "hipGetSymbolAddress(scratch)");
    // every workspace byte a build reads is written earlier in the same
    // build (operand tiles by the prep, partial slots by the contraction):
    // nothing needs clearing between calls
    return enqueue_build(*h, m, d, j, k, mode, v, (hipStream_t)hip_stream, nullptr, nullptr, nullptr, ws);
}
