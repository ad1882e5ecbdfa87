// Allocation-free apply: the operator's time loop with the TTI gradient
// buffers (the only scratch its kernels use) in a file-scope device array of
// fixed size instead of the operator's own buffers, for callers that cannot
// allocate device memory (graph capture, tight serving loops).
//
// The array exists once per GPU for the life of the process.  Host code never
// passes its name to a kernel or a copy: the device address is taken once per
// device with hipGetSymbolAddress and kept here.
#include "fdw.h"
#include "fdw_internal.h"

#include <atomic>
#include <cstdio>

namespace {

constexpr int64_t kScratchFloats = (int64_t)16 << 20;  // 64 MiB per GPU
constexpr int kMaxDevices = 64;

static __device__ __align__(256) float scratch[kScratchFloats];

std::atomic<float *> g_scratch_ptr[kMaxDevices];

// device address of this device's scratch array (looked up on first use)
int scratch_address(float **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        char msg[160];
        std::snprintf(msg, sizeof(msg), "operator_apply_noalloc: hipGetDevice: %s", hipGetErrorString(e));
        return fdw::set_error(FDW_ERR_DEVICE, msg);
    }
    if (dev < 0 || dev >= kMaxDevices) return fdw::set_error(FDW_ERR_DEVICE, "operator_apply_noalloc: device index");
    float *p = g_scratch_ptr[dev].load();
    if (!p) {
        void *addr = nullptr;
        e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !addr) {
            char msg[160];
            std::snprintf(msg, sizeof(msg), "operator_apply_noalloc: hipGetSymbolAddress: %s",
                          hipGetErrorString(e));
            return fdw::set_error(FDW_ERR_DEVICE, msg);
        }
        p = static_cast<float *>(addr);
        g_scratch_ptr[dev].store(p);
    }
    *out = p;
    return FDW_OK;
}

}  // namespace

extern "C" int fdw_operator_apply_noalloc(fdw_op *op, int time_m, int time_M, void *stream) {
    if (!op) return fdw::set_error(FDW_ERR_ARG, "operator_apply_noalloc: NULL op");
    const int64_t need = fdw::operator_stage_floats(op);
    if (need > kScratchFloats) {
        char msg[200];
        std::snprintf(msg, sizeof(msg),
                      "operator_apply_noalloc: the operator needs %lld floats of gradient buffers, above the "
                      "%lld-float (64 MiB) allocation-free scratch",
                      (long long)need, (long long)kScratchFloats);
        return fdw::set_error(FDW_ERR_ARG, msg);
    }
    float *stage = nullptr;
    if (need > 0) {
        int st = scratch_address(&stage);
        if (st) return st;
        // the previous call's values: the gradient buffers must read zero
        // outside the domain, so the region is cleared (a fill kernel, no
        // memset node when the stream is being captured)
        hipError_t e = fdw::launch_fill_zero(stage, need, (hipStream_t)stream);
        if (e != hipSuccess) {
            char msg[160];
            std::snprintf(msg, sizeof(msg), "operator_apply_noalloc: clearing the scratch: %s", hipGetErrorString(e));
            return fdw::set_error(FDW_ERR_DEVICE, msg);
        }
    }
    return fdw::operator_apply_stage(op, time_m, time_M, stream, stage);
}
