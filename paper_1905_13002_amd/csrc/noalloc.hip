// noalloc.hip -- pks_filter_smooth_noalloc: pks_filter_smooth with its
// workspace in a static device array instead of caller memory, for callers
// that cannot allocate (code under HIP graph capture, serving loops, hosts
// that forbid hipMalloc).
//
// The array `scratch` below is one per GPU: the runtime places a copy on every
// device the library runs on when the code object loads, and it stays until
// the process ends.  Its host-side name is not a device address: the device
// address is taken once per device with hipGetSymbolAddress and kept in
// g_scratch[device]; only that pointer is ever handed to kernels.  Calls on
// one GPU share the array (it keeps the last call's contents), so calls that
// overlap on one GPU race; the scan kernels write every word they read before
// reading it, and the numeric flag is reset by every call.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "pks_internal.h"
#include "plan.h"

namespace pks {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;   // 32 MiB per GPU
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// device address of this device's copy of `scratch` (taken once per device,
// with that device current)
hipError_t scratch_ptr(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

}  // namespace
}  // namespace pks

extern "C" {

size_t pks_noalloc_scratch_bytes(void) { return pks::kScratchBytes; }

pks_status pks_filter_smooth_noalloc(const pks_model* model, int64_t T, const void* y, void* m, void* P, void* ms,
                                     void* Ps, pks_precision prec, void* stream) {
    if (!model) {
        pks::set_last_error("model is NULL");
        return PKS_E_ARG;
    }
    const size_t need = pks_workspace_bytes(model->nx, model->ny, T, 1, prec);
    if (need == 0) {
        pks::set_last_error("invalid nx, ny, T or precision");
        return PKS_E_ARG;
    }
    if (need > pks::kScratchBytes) {
        char buf[256];
        snprintf(buf, sizeof buf,
                 "this problem needs %zu bytes of workspace; the static scratch holds %zu bytes "
                 "(use pks_filter_smooth with a caller workspace)", need, pks::kScratchBytes);
        pks::set_last_error(buf);
        return PKS_E_UNSUPPORTED;
    }
    void* ws = nullptr;
    const hipError_t e = pks::scratch_ptr(&ws);
    if (e != hipSuccess) {
        char buf[256];
        snprintf(buf, sizeof buf, "locating the static scratch: %s", hipGetErrorString(e));
        pks::set_last_error(buf);
        return PKS_E_HIP;
    }
    return pks_filter_smooth(model, T, y, m, P, ms, Ps, prec, ws, pks::kScratchBytes, stream);
}

}  // extern "C"
