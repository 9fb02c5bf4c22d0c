// chi0_noalloc.hip -- chi0_dynamic for callers that cannot allocate device memory.
//
// The workspace of the call (matrix elements and partial sums of a batch of q-points, the input
// scan's verdict word) lives in `scratch`, a fixed array of this library in device memory, instead
// of a caller buffer.  The array is a device symbol: in host code its name is only a stand-in, so
// its device address is looked up once per device (hipGetSymbolAddress, with that device current)
// at the first call on the device and kept; the kernels receive that address exactly as they
// receive a caller workspace.  Every call on a device shares that device's array and leaves its
// contents behind; the call writes every part of it that it reads (the verdict word is cleared by a
// kernel of the call), and calls that overlap on one device race on it.
#include "../../include/chi0.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "chi0_host.h"

namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;   // 128 MiB per device, held until process end
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

void *g_scratch_dev[kMaxDevices];     // device address of `scratch` on each device (null: not yet)
std::mutex g_scratch_lock;

hipError_t scratch_address(void **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> guard(g_scratch_lock);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_dev[dev] = ptr;
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

}  // namespace

extern "C" chi0_status chi0_dynamic_noalloc(chi0_plan_t plan, int32_t nq, const chi0_q *qs, int32_t nw,
                                            const double *omega, double *chi)
{
    if (!plan) return CHI0_E_INVALID_ARG;
    void *ws = nullptr;
    const hipError_t e = scratch_address(&ws);
    if (e != hipSuccess) return chi0::plan_device_error(plan, e, "scratch address");
    return chi0::dynamic_scratch(plan, nq, qs, nw, omega, ws, kScratchBytes, chi);
}
