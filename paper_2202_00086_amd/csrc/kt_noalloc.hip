// kt_noalloc.hip -- kt_render for callers that cannot allocate device
// memory: the render's workspace (ray ticket, accumulators, the device copy
// of the launch parameters, the crossing radii, the dispatch order and, for
// KT_MIXED, the fallback list) lives in a file-scope device array of fixed
// size instead of a caller's buffer.
//
// In host code the array's name is only a stand-in for a device address,
// so the address is taken once per device with hipGetSymbolAddress, with
// that device current, and only that address is ever handed to kernels.
// Every call on one GPU shares that GPU's array and leaves its contents
// behind; the render re-initialises whatever must start at zero (ticket,
// accumulators, histograms) with its own kernels, as it does for a caller's
// workspace.  Calls that overlap on one GPU (two host threads, or two
// streams without ordering between them) race on the array.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "kerrtrace.h"
#include "kt_internal.h"

namespace {

static __device__ __align__(256) unsigned char scratch[KT_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void* g_scratch[MAX_DEVICES] = {nullptr};

// Device address of this device's scratch array (taken on the first call
// on the device), or nullptr with the error left for kt_last_error().
void* scratch_address(int* rc) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        char msg[256];
        std::snprintf(msg, sizeof msg, "kt_render_noalloc: no usable current device (%s, device %d)",
                      hipGetErrorString(e), dev);
        *rc = kt::set_error(KT_EDEVICE, msg);
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            char msg[256];
            std::snprintf(msg, sizeof msg, "kt_render_noalloc: hipGetSymbolAddress of the scratch array failed: %s",
                          hipGetErrorString(e));
            *rc = kt::set_error(KT_EDEVICE, msg);
            return nullptr;
        }
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace

extern "C" int kt_render_noalloc(const kt_camera* camera, const kt_spacetime* spacetime, const kt_disk* disk,
                                 const kt_source* source, const kt_integrator* integ, const kt_outputs* out,
                                 void* hip_stream, const kt_launch* launch) {
    kt::Image im;
    int rc = kt::validate_single(camera, spacetime, disk, source, integ, out, &im);
    if (rc) return rc;
    const size_t need = kt_workspace_bytes(camera, integ);
    if (need == 0) return kt::set_error(KT_EINVAL, "kt_render_noalloc: bad camera or integrator");
    if (need > static_cast<size_t>(KT_NOALLOC_SCRATCH_BYTES)) {
        char msg[256];
        std::snprintf(msg, sizeof msg,
                      "kt_render_noalloc: this render needs %zu bytes of scratch, more than the library's %zu "
                      "(use kt_render_ex with a workspace)",
                      need, static_cast<size_t>(KT_NOALLOC_SCRATCH_BYTES));
        return kt::set_error(KT_ENOMEM, msg);
    }
    void* ptr = scratch_address(&rc);
    if (!ptr) return rc;
    return kt_render_ex(camera, spacetime, disk, source, integ, out, ptr, KT_NOALLOC_SCRATCH_BYTES, hip_stream,
                        launch);
}
