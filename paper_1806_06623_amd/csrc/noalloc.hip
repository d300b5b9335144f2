// FP64 solve that allocates nothing, for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid allocation): the workspace of spp_solve is this file's device array
// instead of a caller buffer.  Same kernels, same result as spp_solve.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.h"

namespace {

// The workspace of spp_solve_noalloc.  Each device that loads this library
// holds its own copy (zero-initialised data of the code object) until the
// process ends.  In host code this name is only a stand-in for the device
// array: kernels get the address hipGetSymbolAddress returns on the current
// device (spp_noalloc_scratch), never the name itself.
static __device__ __align__(256) unsigned char scratch[SPP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
spp_status scratch_on_current_device(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return spp_fail(SPP_EDEVICE, std::string("spp_solve_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return spp_fail(SPP_ENOTSUP, "spp_solve_noalloc: device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return spp_fail(SPP_EDEVICE, std::string("spp_solve_noalloc: hipGetSymbolAddress(scratch): ") +
                                             hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPP_OK;
}

}  // namespace

spp_status spp_noalloc_scratch_current(void** ptr) { return scratch_on_current_device(ptr); }

// Set-up hook (spp_plan_upload, with the plan's device current): resolve the
// scratch address of this device before the first no-allocation solve.  A
// failure here is not an error of the upload; the entry point reports it.
void spp_noalloc_prepare_current_device()
{
    void* ptr = nullptr;
    (void)scratch_on_current_device(&ptr);
}

extern "C" spp_status spp_solve_noalloc(spp_plan p, const double* rho_dev, double* phi_dev, double G, void* stream)
{
    if (!p) return spp_fail(SPP_EINVAL, "spp_solve_noalloc: NULL plan");
    const size_t need = spp_path_workspace_bytes(p, spp_plan_fused(p));
    if (need > SPP_NOALLOC_SCRATCH_BYTES)
        return spp_fail(SPP_ENOTSUP, "spp_solve_noalloc: this plan needs " + std::to_string(need) +
                                         " bytes of workspace on its current path, more than the " +
                                         std::to_string(SPP_NOALLOC_SCRATCH_BYTES) +
                                         " bytes of the library's scratch; use spp_solve with a workspace");
    void* ws = nullptr;
    spp_status st = scratch_on_current_device(&ws);
    if (st != SPP_OK) return st;
    st = spp_validate_solve("spp_solve_noalloc", p, rho_dev, phi_dev, G, ws);
    if (st != SPP_OK) return st;
    return spp_launch_solve_f64(p, rho_dev, phi_dev, G, ws, stream);
}
