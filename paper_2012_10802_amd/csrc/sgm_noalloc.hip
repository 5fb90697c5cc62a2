// sgm_match_noalloc: the whole single-pair path (census, cost, aggregation,
// selection) with its workspace in a library-owned device array, for callers
// that cannot allocate device memory (code under stream capture, tight
// serving loops).  The array is a file-scope __device__ object: every GPU
// the library runs on holds one copy of SGM_NOALLOC_SCRATCH_BYTES bytes,
// at its own address, from the code object's load until the process ends.
//
// In host code the array's name stands for a host-side shadow, not for the
// device memory: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever passed to kernels.

#include "../../include/sgm.h"

#include <stdarg.h>
#include <stdio.h>

#include <mutex>

#include "sgm_internal.h"

namespace {

constexpr size_t kScratchBytes = SGM_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;

struct DeviceScratch {
    std::once_flag once;
    hipError_t err = hipSuccess;
    void *ptr = nullptr;  // device address of `scratch` on this device
};
DeviceScratch g_dev[kMaxDevices];

sgm_status fail(sgm_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(sgm::error_buffer(), sgm::kErrorBufferSize, fmt, ap);
    va_end(ap);
    return st;
}

// Device address of `scratch` on the current device (looked up on the
// first call made with that device current).
sgm_status scratch_on_current_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(SGM_ERR_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(SGM_ERR_UNSUPPORTED, "device index %d >= %d", dev, kMaxDevices);
    DeviceScratch &d = g_dev[dev];
    std::call_once(d.once, [&d] {
        void *p = nullptr;
        d.err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (d.err == hipSuccess) d.ptr = p;
    });
    if (d.err != hipSuccess || !d.ptr)
        return fail(SGM_ERR_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                    hipGetErrorString(d.err != hipSuccess ? d.err : hipErrorInvalidSymbol));
    *out = d.ptr;
    return SGM_OK;
}

}  // namespace

extern "C" sgm_status sgm_match_noalloc(sgm_plan_t plan, const uint8_t *left, const uint8_t *right,
                                        int32_t pitch, const int32_t *d_lo, uint16_t *disp_int,
                                        float *disp_sub, void *stream)
{
    if (!plan) return fail(SGM_ERR_INVALID, "plan is NULL");
    if (!left || !right || !disp_int) return fail(SGM_ERR_INVALID, "left, right and disp_int must not be NULL");
    size_t need = 0;
    if (sgm_status s = sgm_workspace_size(plan, &need)) return s;
    if (need > kScratchBytes)
        return fail(SGM_ERR_WORKSPACE,
                    "sgm_match_noalloc: the plan needs %zu bytes of workspace, more than the %zu bytes of the "
                    "library's scratch array; use sgm_match with a caller workspace",
                    need, kScratchBytes);
    void *ws = nullptr;
    if (sgm_status s = scratch_on_current_device(&ws)) return s;
    // sgm_match only launches kernels on `stream`: no allocation, no copy,
    // no memset, and nothing in the workspace has to start at zero
    return sgm_match(plan, left, right, pitch, d_lo, disp_int, disp_sub, ws, kScratchBytes, stream);
}
