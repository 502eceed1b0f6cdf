// pbdr_scene_create_static: a scene whose workspace is the library's own
// static device array, for callers that cannot allocate device memory.  See
// include/pbdr.h for the contract.
#include "pbdr.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "pbdr_host.h"

namespace {

using pbdr::host::fail;

// One per device: each GPU that the library runs on holds it until the
// process ends.  In host code the name is only a stand-in for the array; its
// address on each device comes from hipGetSymbolAddress (g_static_ptr), and
// only that address is handed to kernels and copies.
__device__ __align__(256) unsigned char scratch[PBDR_STATIC_WORKSPACE_BYTES];

constexpr int kStaticDevices = 64;
std::mutex g_static_mu;
void* g_static_ptr[kStaticDevices];      // device address of `scratch` on each device

}  // namespace

extern "C" pbdr_status pbdr_scene_create_static(const pbdr_params* params, const pbdr_scene_desc* desc,
                                                void* hip_stream, pbdr_scene** out)
{
    pbdr::host::clear_error();
    if (!out) return fail(PBDR_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!desc) return fail(PBDR_ERR_INVALID_ARG, "desc is NULL");
    const size_t need = pbdr_scene_bytes(params, desc->n_particles, desc->n_bodies);
    if (need == 0) return PBDR_ERR_INVALID_ARG;             // message left by pbdr_scene_bytes
    if (need > (size_t)PBDR_STATIC_WORKSPACE_BYTES)
        return fail(PBDR_ERR_WORKSPACE,
                    "the scene needs a workspace of %zu bytes, more than the %zu of the static workspace; "
                    "pbdr_scene_create takes a caller workspace of any size",
                    need, (size_t)PBDR_STATIC_WORKSPACE_BYTES);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kStaticDevices) return fail(PBDR_ERR_DEVICE, "device %d has no static workspace", dev);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {          // first call on this device, which is current
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(PBDR_ERR_DEVICE, "hipGetSymbolAddress of the static workspace failed: %s",
                        hipGetErrorString(e));
        g_static_ptr[dev] = ptr;
    }
    // the previous static scene of this device (same host record) ends its
    // work before its workspace is overwritten
    pbdr_scene* rec = pbdr::host::fixed_scene_record(dev);
    pbdr::host::release_fixed_record(rec);
    return pbdr::host::create_scene_in(params, desc, g_static_ptr[dev], PBDR_STATIC_WORKSPACE_BYTES, hip_stream,
                                       rec, out);
}
