// Persistent LDS-resident 2D isotropic kernel (gfx950): kernel templates and
// per-form launchers, included by one translation unit per LDS form.
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer, test cases).
#pragma once
#include "fdw_device.h"

namespace fdw {

// ---------------------------------------------------------------------------
// Persistent 2D isotropic kernel: one workgroup of 1024 threads runs every
// step of the apply for a grid small enough that its current level fits in
// LDS (nx * nz floats, no halo: neighbours outside the domain read as zero).
// Each thread owns the points i = tid + 1024 p and keeps, in registers, their
// previous level and (for small grids) dt^2/m and the damping factor.  Per
// step:
//   1. update the owned points from the LDS level (results in registers);
//   2. barrier; the owned points' LDS values become their previous level,
//      the results replace them in LDS;
//   3. barrier; source corners are added in LDS with LDS atomics;
//   4. barrier; receivers are interpolated from LDS (4 corners, one thread
//      each) and, in the last three steps, the level is written to its slot.
// After the apply the slots hold the same levels as with per-step launches
// (the last nslots levels, each in its slot).
// ---------------------------------------------------------------------------
template <int R, int PPT, bool HALO>
__device__ __forceinline__ void iso2d_persistent_body(const Persist2DArgs &a) {
    constexpr bool kCacheCoef = PPT <= 16;
    // LDS level: (nz + 2R) x (nx + 2R) with a zero halo when HALO, else nz x nx
    // with neighbours outside the domain read as zero
    extern __shared__ float lds_level[];
    const int nx = a.g.nx, nz = a.g.nz;
    const int n = nx * nz;
    const int lw = HALO ? nx + 2 * R : nx;
    float *cur = HALO ? lds_level + R * lw + R : lds_level;  // cur[z * lw + x]
    auto li = [&](int i) { return HALO ? (i / nx) * lw + (i % nx) : i; };
    const int tid = threadIdx.x;
    const int64_t off0 = a.g.off0, px = a.pitch_x;
    auto goff = [&](int i) { return off0 + (int64_t)(i / nx) * px + (i % nx); };
    float prev[PPT], cdt[kCacheCoef ? PPT : 1], damp[kCacheCoef ? PPT : 1];
    {
        const int S = a.nslots;
        const float *uc = a.u + (int64_t)(a.time_m % S) * a.slot;
        const float *up = a.u + (int64_t)((a.time_m + S - 1) % S) * a.slot;
        if (HALO)
            for (int i = tid; i < (nz + 2 * R) * lw; i += 1024) lds_level[i] = 0.0f;
        __syncthreads();
        for (int i = tid; i < n; i += 1024) cur[li(i)] = uc[goff(i)];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int i = tid + 1024 * p;
            prev[p] = i < n ? up[goff(i)] : 0.0f;
            if constexpr (kCacheCoef) {
                cdt[p] = i < n ? a.dt2 * fast_rcp(a.m[goff(i)]) : 0.0f;
                damp[p] = i < n ? a.eta_x[i % nx] + a.eta_z[i / nx] : 0.0f;
            }
        }
    }
    __syncthreads();
    for (int t = a.time_m; t <= a.time_M; ++t) {
        float v[PPT];
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int i = tid + 1024 * p;
            v[p] = 0.0f;
            if (i < n) {
                const int x = i % nx, z = i / nx;
                const int l = z * lw + x;
                const float uc = cur[l];
                float lap = 0.0f;
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    const float xp = (HALO || x + k < nx) ? cur[l + k] : 0.0f;
                    const float xm = (HALO || x - k >= 0) ? cur[l - k] : 0.0f;
                    const float zp = (HALO || z + k < nz) ? cur[l + k * lw] : 0.0f;
                    const float zm = (HALO || z - k >= 0) ? cur[l - k * lw] : 0.0f;
                    lap = lap_term(lap, a.c.w2[0][k], xp, xm, uc);
                    lap = lap_term(lap, a.c.w2[2][k], zp, zm, uc);
                }
                float c, dmp;
                if constexpr (kCacheCoef) {
                    c = cdt[p];
                    dmp = damp[p];
                } else {
                    c = a.dt2 * fast_rcp(a.m[goff(i)]);
                    dmp = a.eta_x[x] + a.eta_z[z];
                }
                v[p] = leapfrog(uc, prev[p], c * lap, dmp);
            }
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < PPT; ++p) {
            const int i = tid + 1024 * p;
            if (i < n) {
                prev[p] = cur[li(i)];
                cur[li(i)] = v[p];
            }
        }
        if (a.nsrc > 0) {
            __syncthreads();
            const float *q = a.src_data + (int64_t)t * a.nsrc;
            for (int e = tid; e < a.nsrc * 4; e += 1024) {
                const int s = e >> 2, c = e & 3;
                const int64_t rel = a.src_base[s] - off0;
                const int x = (int)(rel % px) + (c & 1), z = (int)(rel / px) + (c >> 1);
                const int64_t gi = off0 + (int64_t)z * px + x;
                atomicAdd(&cur[z * lw + x], a.src_w[s * 4 + c] * q[s] * fast_rcp(a.m[gi]));
            }
        }
        __syncthreads();
        if (t >= a.time_M - (a.nslots - 1)) {
            float *un = a.u + (int64_t)((t + 1) % a.nslots) * a.slot;
            for (int i = tid; i < n; i += 1024) un[goff(i)] = cur[li(i)];
        }
        if (a.nrec > 0) {
            float *rr = a.rec_data + (int64_t)t * a.nrec;
            for (int e = tid; e < a.nrec * 4; e += 1024) {
                const int r = e >> 2, c = e & 3;
                const int64_t rel = a.rec_base[r] - off0;
                const int x = (int)(rel % px) + (c & 1), z = (int)(rel / px) + (c >> 1);
                float val = a.rec_w[r * 4 + c] * cur[z * lw + x];
                // groups of 4 lanes are aligned in the wavefront
                val += __shfl_xor(val, 1);
                val += __shfl_xor(val, 2);
                if (c == 0) rr[r] = val;
            }
        }
        // LDS is only read from here to the first barrier of the next step
    }
}

template <int R, int PPT, bool HALO>
__global__ void __launch_bounds__(1024) iso2d_persistent(Persist2DArgs a) {
    iso2d_persistent_body<R, PPT, HALO>(a);
}

// Shots of one geometry, one workgroup each (blockIdx.x selects the shot's
// arguments); each runs its own step range.
template <int R, int PPT, bool HALO>
__global__ void __launch_bounds__(1024) iso2d_persistent_multi(const Persist2DArgs *__restrict__ shots) {
    iso2d_persistent_body<R, PPT, HALO>(shots[blockIdx.x]);
}

template <int R, bool HALO>
static hipError_t launch_iso2d_persistent_h(const Persist2DArgs &a, size_t lds, hipStream_t s, const LaunchEvents &ev) {
    const int ppt = (a.g.nx * a.g.nz + 1023) / 1024;
#define P2D(PPT_)                                                                                       \
    {                                                                                                   \
        hipError_t e = hipFuncSetAttribute((const void *)iso2d_persistent<R, PPT_, HALO>,              \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);       \
        if (e != hipSuccess) return e;                                                                  \
        hipExtLaunchKernelGGL((iso2d_persistent<R, PPT_, HALO>), dim3(1), dim3(1024), lds, s, ev.start, \
                              ev.stop, 0, a);                                                           \
        return hipGetLastError();                                                                       \
    }
    if (ppt <= 8) P2D(8)
    if (ppt <= 16) P2D(16)
    if (ppt <= 24) P2D(24)
    if (ppt <= 40) P2D(40)
#undef P2D
    return hipErrorInvalidValue;
}

template <int R, bool HALO>
static hipError_t launch_iso2d_persistent_multi_h(const Geom &g, const Persist2DArgs *shots, int n, size_t lds,
                                                  hipStream_t s) {
    const int ppt = (g.nx * g.nz + 1023) / 1024;
#define P2M(PPT_)                                                                                         \
    {                                                                                                     \
        hipError_t e = hipFuncSetAttribute((const void *)iso2d_persistent_multi<R, PPT_, HALO>,          \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);         \
        if (e != hipSuccess) return e;                                                                    \
        hipLaunchKernelGGL((iso2d_persistent_multi<R, PPT_, HALO>), dim3((unsigned)n), dim3(1024), lds, s, \
                           shots);                                                                        \
        return hipGetLastError();                                                                         \
    }
    if (ppt <= 8) P2M(8)
    if (ppt <= 16) P2M(16)
    if (ppt <= 24) P2M(24)
    if (ppt <= 40) P2M(40)
#undef P2M
    return hipErrorInvalidValue;
}

// Launchers of one LDS form (HALO) for every radius: one translation unit
// per form (fdw_iso2d_halo.hip, fdw_iso2d_nohalo.hip) keeps the build parallel.
template <bool HALO>
static hipError_t p2d_form_launch(int R, const Persist2DArgs *one, const Geom &g, const Persist2DArgs *shots, int n,
                                  size_t lds, hipStream_t s, const LaunchEvents &ev) {
#define P2F(r) (one ? launch_iso2d_persistent_h<r, HALO>(*one, lds, s, ev) \
                    : launch_iso2d_persistent_multi_h<r, HALO>(g, shots, n, lds, s))
    FDW_DISPATCH_R(R, P2F)
#undef P2F
}
}  // namespace fdw
