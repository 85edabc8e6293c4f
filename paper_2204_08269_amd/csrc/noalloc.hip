// Forward transform for callers that cannot allocate device memory (code under
// HIP graph capture, tight serving loops, harnesses that forbid allocation): the
// workspace of jtfs_forward comes from a fixed device array of this library, one
// copy per GPU, instead of from the caller.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"
#include "timing.hpp"

namespace jtfs {
namespace {

// Every GPU the library runs on holds this array until the process ends.  Host
// code never passes its name to a kernel or a copy (on the host the name is a
// stand-in, not a device address): it uses the device address that
// hipGetSymbolAddress returns for the current device.
__device__ __align__(256) unsigned char scratch[JTFS_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

// Device address of this GPU's copy of the array (looked up once per device,
// with that device current).
int scratch_ptr(int dev, void** out) {
    if (dev < 0 || dev >= kMaxDevices) { set_error("device index beyond the scratch table"); return JTFS_EINVAL; }
    std::lock_guard<std::mutex> l(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
            return JTFS_EHIP;
        }
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return JTFS_OK;
}

}  // namespace
}  // namespace jtfs

extern "C" int jtfs_forward_noalloc(const jtfs_plan* P, const float* x, int64_t B, float* s1, float* s2,
                                    hipStream_t st) {
    if (!P) { jtfs::set_error("null plan"); return JTFS_EINVAL; }
    if (B < 1) { jtfs::set_error("B must be >= 1"); return JTFS_ESHAPE; }
    size_t need = 0;
    int rc = jtfs_forward_workspace_size(P, B, &need);
    if (rc != JTFS_OK) return rc;
    if (need > (size_t)JTFS_NOALLOC_SCRATCH_BYTES) {
        jtfs::set_error("jtfs_forward_noalloc: the forward workspace of " + std::to_string(need) +
                        " bytes exceeds the fixed scratch of " + std::to_string((size_t)JTFS_NOALLOC_SCRATCH_BYTES) +
                        " bytes (fewer signals per call, or jtfs_forward with a caller workspace)");
        return JTFS_EWORKSPACE;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) { jtfs::set_error("hipGetDevice failed"); return JTFS_EHIP; }
    if (dev != P->device) { jtfs::set_error("the current device is not the plan's device"); return JTFS_EINVAL; }
    void* ws = nullptr;
    rc = jtfs::scratch_ptr(dev, &ws);
    if (rc != JTFS_OK) return rc;
    // no stage events either: timing would create them
    jtfs::TimingSuppressed quiet;
    return jtfs_forward(P, x, B, s1, s2, ws, (size_t)JTFS_NOALLOC_SCRATCH_BYTES, st);
}
