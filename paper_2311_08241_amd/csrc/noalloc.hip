// se_subcycle_noalloc: the forward subcycle with its workspace in a static device
// array instead of a caller buffer, for callers that cannot allocate device memory.
//
// The array lives in this translation unit's code object; each device the library
// runs on holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it is a host-side stand-in.  The device address
// is looked up once per device (hipGetSymbolAddress, with that device current) and
// kept; every use goes through that address.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "se_internal.h"

namespace {

constexpr size_t kScratchBytes = SE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of this device's scratch array (looked up on the first call on the
// device, with the device current).  nullptr with the error text set on failure.
void *scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) {
        sesub::set_error("se_subcycle_noalloc: device index " + std::to_string(device) +
                         " outside 0.." + std::to_string(kMaxDevices - 1));
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return g_scratch[device];
    int prev = -1;
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != device && hipSetDevice(device) != hipSuccess) {
        sesub::set_error("se_subcycle_noalloc: cannot select device " + std::to_string(device));
        return nullptr;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess || !ptr) {
        sesub::set_error(std::string("se_subcycle_noalloc: hipGetSymbolAddress of the scratch "
                                     "array: ") + hipGetErrorString(e));
        return nullptr;
    }
    g_scratch[device] = ptr;
    return ptr;
}

}  // namespace

extern "C" se_status se_subcycle_noalloc(se_mesh *mesh, const se_params *params,
                                         se_state *state, const se_forcing *forcing,
                                         int32_t nsub, double dt, void *stream) {
    if (!mesh || !params) {
        sesub::set_error("se_subcycle_noalloc: null mesh or parameters");
        return SE_ERR_ARG;
    }
    if (mesh->device < 0) {
        sesub::set_error("host-only mesh (created with device < 0) cannot run kernels");
        return SE_ERR_ARG;
    }
    size_t need = 0;
    const se_status st = se_workspace_bytes(mesh, params, nsub, 0, &need);
    if (st != SE_OK) return st;
    if (need > kScratchBytes) {
        sesub::set_error("se_subcycle_noalloc: this mesh and run need " + std::to_string(need) +
                         " bytes of workspace, above the static scratch of " +
                         std::to_string(kScratchBytes) + " bytes (use se_subcycle with a "
                         "caller workspace)");
        return SE_ERR_ARG;
    }
    void *ws = scratch_on(mesh->device);
    if (!ws) return SE_ERR_HIP;
    return sesub::subcycle_tile(mesh, params, state, forcing, nsub, dt, ws, stream, false);
}
