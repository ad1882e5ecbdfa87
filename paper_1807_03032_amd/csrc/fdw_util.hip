// Bandwidth probes (gfx950): plain streaming kernels of known traffic that
// measure the HBM bandwidth the chip attains, the reference against which the
// stencil kernels' achieved bandwidth is compared (the paper's Section 7.1 takes
// the STREAM triad rate as the attainable peak of its roofline plots).
#include "fdw_internal.h"

#include <algorithm>

namespace fdw {

// Each workgroup moves a contiguous block of kProbeVec float4 per thread,
// every load of the block issued before the first store.
constexpr int kProbeThreads = 256, kProbeVec = 4;

template <int KIND>
__global__ void __launch_bounds__(kProbeThreads) bandwidth_probe(float4 *__restrict__ dst, const float4 *__restrict__ a,
                                                                 const float4 *__restrict__ b, float s, int64_t n4) {
    const int64_t base = (int64_t)blockIdx.x * (kProbeThreads * kProbeVec) + threadIdx.x;
    float4 va[kProbeVec], vb[kProbeVec];
#pragma unroll
    for (int k = 0; k < kProbeVec; ++k) {
        const int64_t i = base + (int64_t)k * kProbeThreads;
        if (i < n4) {
            va[k] = a[i];
            if (KIND == 1) vb[k] = b[i];
        }
    }
#pragma unroll
    for (int k = 0; k < kProbeVec; ++k) {
        const int64_t i = base + (int64_t)k * kProbeThreads;
        if (i < n4) {
            float4 v = va[k];
            if (KIND == 1) {
                v.x += s * vb[k].x;
                v.y += s * vb[k].y;
                v.z += s * vb[k].z;
                v.w += s * vb[k].w;
            }
            dst[i] = v;
        }
    }
}

hipError_t launch_bandwidth_probe(int kind, float *dst, const float *a, const float *b, float s, int64_t n,
                                  hipStream_t st) {
    const int64_t n4 = n / 4;
    const int64_t per = kProbeThreads * kProbeVec;
    const int64_t blocks = (n4 + per - 1) / per;
    if (blocks <= 0) return hipSuccess;
    if (kind == 0)
        hipLaunchKernelGGL(bandwidth_probe<0>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, (float4 *)dst,
                           (const float4 *)a, (const float4 *)b, s, n4);
    else
        hipLaunchKernelGGL(bandwidth_probe<1>, dim3((unsigned)blocks), dim3(kProbeThreads), 0, st, (float4 *)dst,
                           (const float4 *)a, (const float4 *)b, s, n4);
    return hipGetLastError();
}

__global__ void __launch_bounds__(256) fill_zero_kernel(float *__restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = 0.0f;
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

}  // namespace fdw
