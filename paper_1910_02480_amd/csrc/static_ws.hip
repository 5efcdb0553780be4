// Forward pass without a caller-supplied workspace, for callers that cannot
// allocate device memory (code under HIP graph capture, serving loops that
// forbid allocation). The layer path's intermediate activations (h1, h2,
// h3, u3, u2 of the batch) live in one file-scope device array per GPU,
// `scratch`, instead of in a workspace argument.
//
// The array's host-side name is only a stand-in for the symbol: host code
// uses the device address that hipGetSymbolAddress returns for the current
// device, obtained once per device when the first handle is created there.
#include <hip/hip_runtime.h>

#include <mutex>

#include "drc_cae.h"
#include "internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)64 << 20;  // per device, held until the process ends
constexpr int kMaxDevices = 64;

__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device (null: not set up)

}  // namespace

// Called by drc_cae_create with the handle's device current.
drc_status static_scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return drc_fail(DRC_ERR_UNSUPPORTED, "create: device %d beyond the %d the library tracks", device,
                        kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_scratch[device]) return DRC_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return drc_fail(DRC_ERR_HIP, "create: hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[device] = p;
    return DRC_OK;
}

extern "C" size_t drc_cae_static_scratch_bytes(void) { return kScratchBytes; }

extern "C" drc_status drc_cae_forward_static(drc_cae* h, const float* d_x, float* d_y, int n, int H, int W,
                                             void* stream) {
    if (!h) return drc_fail(DRC_ERR_INVALID_ARG, "forward_static: handle is NULL");
    void* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (h->device >= 0 && h->device < kMaxDevices) ws = g_scratch[h->device];
    }
    if (!ws) return drc_fail(DRC_ERR_STATE, "forward_static: no scratch array on device %d", h->device);
    size_t need = 0;
    drc_status st = drc_cae_workspace_size(h, n, H, W, DRC_WS_FORWARD, &need);
    if (st != DRC_OK) return st;
    if (need > kScratchBytes)
        return drc_fail(DRC_ERR_WORKSPACE,
                        "forward_static: %d maps of %dx%d need %zu bytes of scratch; the library holds %zu per "
                        "device (split the batch, or use drc_cae_forward with a workspace)",
                        n, H, W, need, kScratchBytes);
    return drc_cae_forward(h, d_x, d_y, n, H, W, nullptr, ws, kScratchBytes, stream);
}
