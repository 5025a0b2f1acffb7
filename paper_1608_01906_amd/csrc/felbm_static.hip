// The library's own device workspace, for callers that cannot allocate
// device memory (fel_bind_static in include/felbm.h).
//
// `scratch` is a file-scope device array: every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  In host
// code the array's name is only a host-side stand-in, so the device address
// is looked up once per device with hipGetSymbolAddress (with that device
// current) and that address is what the context is bound to: kernel
// arguments, clears and copies all go through it.
#include "../../include/felbm.h"
#include "felbm_internal.h"

#include <mutex>

namespace {

static __device__ __align__(256) unsigned char scratch[fel::kStaticWorkspaceBytes];

std::mutex g_lookup_mu;
void* g_scratch_ptr[fel::kMaxDevices] = {};  // device address of scratch, per device

}  // namespace

extern "C" FEL_API fel_status fel_bind_static(fel_ctx* c, void* hip_stream) {
    if (!c) return FEL_EINVAL;
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fel::set_error(c, FEL_EDEVICE, hipGetErrorString(e));
    if (dev < 0 || dev >= fel::kMaxDevices) return fel::set_error(c, FEL_EDEVICE, "device index out of range");
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_lookup_mu);
        if (!g_scratch_ptr[dev]) {
            e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_scratch_ptr[dev]) {
                g_scratch_ptr[dev] = nullptr;
                return fel::set_error(c, FEL_EDEVICE, e != hipSuccess ? hipGetErrorString(e)
                                                                      : "static workspace has no device address");
            }
        }
        ptr = g_scratch_ptr[dev];
    }
    return fel::bind_static_workspace(c, ptr, fel::kStaticWorkspaceBytes, hip_stream, dev);
}
