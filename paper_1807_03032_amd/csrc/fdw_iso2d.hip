// Isotropic acoustic 2D kernels (gfx950): dispatch of the LDS-resident
// persistent kernel that runs a whole apply of a small grid in one launch
// (one workgroup per shot; kernels in fdw_iso2d_persist.h), and 2D temporal
// blocking (several steps per launch on overlapped LDS patches).
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer, test cases), Section 8
// (time tiling).
#include "fdw_device.h"

namespace fdw {

// LDS form: a zero halo around the level when it fits, else the level alone
static hipError_t launch_iso2d_persistent_any(int R, const Persist2DArgs *one, const Geom &g,
                                              const Persist2DArgs *shots, int n, hipStream_t s,
                                              const LaunchEvents &ev) {
    if ((size_t)g.nx * g.nz * sizeof(float) > (size_t)kPersist2DMaxLds || R < 1 || R > kMaxR)
        return hipErrorInvalidValue;
    const size_t halo = sizeof(float) * (size_t)(g.nx + 2 * R) * (size_t)(g.nz + 2 * R);
    if (halo <= (size_t)kPersist2DMaxLds) return launch_iso2d_persistent_halo(R, one, g, shots, n, halo, s, ev);
    return launch_iso2d_persistent_nohalo(R, one, g, shots, n, sizeof(float) * (size_t)g.nx * g.nz, s, ev);
}

hipError_t launch_iso2d_persistent_multi(int R, const Geom &g, const Persist2DArgs *shots, int n, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    return launch_iso2d_persistent_any(R, nullptr, g, shots, n, s, LaunchEvents{});
}

hipError_t launch_iso2d_persistent(int R, const Persist2DArgs &a, hipStream_t s, const LaunchEvents &ev) {
    return launch_iso2d_persistent_any(R, &a, a.g, nullptr, 1, s, ev);
}

// ---------------------------------------------------------------------------
// 2D temporal blocking (time tiling): one workgroup of 1024 threads per inner
// tile IX x IZ.  The workgroup loads the patch (tile plus a halo of
// H = K R + 1 points, clipped to nothing outside the domain: those points stay
// zero) of levels t0 - 1 and t0 into LDS, with an R-wide zero margin so every
// neighbour read stays inside the array, and advances it K steps:
//   1. every thread updates its patch points from the LDS levels (the same
//      Laplacian, leapfrog and fused injection as the per-step kernels, so the
//      results are the per-step results bit for bit) and writes each result
//      over the point's older level (read by no other point);
//   2. barrier; receivers whose base node lies in the inner tile are sampled
//      from the new level in LDS (same summation order as the lane reduction
//      of the per-step sampling kernel).
// After j steps the values at distance >= j R from the patch edge are exact;
// the inner tile plus one ring (receiver corners) stays exact for j <= K.  The
// inner tile's last two levels are written to the output buffers.
// HBM bytes per inner point per pass: reads of two levels and m over the
// patch (H-halo overhead), writes of two levels: (3 P / I + 2) x 4 B for K
// steps, against 16 B per step for the per-step kernel.
// ---------------------------------------------------------------------------
template <int R>
struct TB2DCfg {
    static constexpr int K = R <= 4 ? 4 : 2;
    static constexpr int IX = R <= 6 ? 128 : 112, IZ = 64;
    static constexpr int H = K * R + 1;
    static constexpr int PX = IX + 2 * H, PZ = IZ + 2 * H;  // patch
    static constexpr int LX = PX + 2 * R, LZ = PZ + 2 * R;  // LDS rows with the zero margin
    static constexpr int NT = 1024;
    static constexpr int PPT = (PX * PZ + NT - 1) / NT;
    static constexpr size_t lds = 2 * sizeof(float) * (size_t)LX * LZ;
};

template <int R>
__global__ void __launch_bounds__(1024) iso2d_tb(TB2DArgs a) {
    using C = TB2DCfg<R>;
    extern __shared__ float lds_tb[];
    float *bufA = lds_tb, *bufB = lds_tb + C::LX * C::LZ;
    const int tid = threadIdx.x;
    const int tiles_x = (a.g.nx + C::IX - 1) / C::IX;
    const int tx = blockIdx.x % tiles_x, tz = blockIdx.x / tiles_x;
    const int ix0 = tx * C::IX, iz0 = tz * C::IZ;  // inner tile origin
    const int px0 = ix0 - C::H, pz0 = iz0 - C::H;  // patch origin
    for (int i = tid; i < C::LX * C::LZ; i += C::NT) {
        bufA[i] = 0.0f;
        bufB[i] = 0.0f;
    }
    __syncthreads();
    // LDS view of the patch as a 2D grid (x stride 1, z stride LX)
    Geom gl{};
    gl.sz = C::LX;
    // LDS index of patch point i (the zero margin is R wide)
    auto lidx = [&](int i) { return (i / C::PX + R) * C::LX + (i % C::PX + R); };
    uint32_t inmask = 0, outmask = 0;  // bit p: point p in the domain / in the inner tile
#pragma unroll
    for (int p = 0; p < C::PPT; ++p) {
        const int i = tid + C::NT * p;
        const int lx = i % C::PX, lz = i / C::PX;
        const int x = px0 + lx, z = pz0 + lz;
        if (i < C::PX * C::PZ && x >= 0 && x < a.g.nx && z >= 0 && z < a.g.nz) {
            inmask |= 1u << p;
            if (x >= ix0 && x < ix0 + C::IX && z >= iz0 && z < iz0 + C::IZ) outmask |= 1u << p;
            const int64_t gi = a.g.off0 + (int64_t)z * a.g.sz + x;
            bufA[lidx(i)] = a.in_prev[gi];
            bufB[lidx(i)] = a.in_cur[gi];
        }
    }
    __syncthreads();
    float *cur = bufB, *prv = bufA;
    for (int j = 0; j < a.nsteps; ++j) {
        const float *q = a.src.n ? a.src.q + (int64_t)j * a.src_stride : nullptr;
        // the new level overwrites the older one in place: prv at a point is
        // read only by that point's own update, cur is not written this step
        // (two points in flight per thread keep the loads within registers)
#pragma unroll 2
        for (int p = 0; p < C::PPT; ++p) {
            if (inmask & (1u << p)) {
                const int i = tid + C::NT * p;
                const int l = lidx(i);
                const int x = px0 + i % C::PX, z = pz0 + i / C::PX;
                // 1/m and the damping factor are re-read each step (cache hits)
                const float rm = fast_rcp(a.m[a.g.off0 + (int64_t)z * a.g.sz + x]);
                const float damp = a.eta_x[x] + a.eta_z[z];
                const float lap = laplacian_at<2, R>(cur, l, gl, a.c);
                float un = leapfrog(cur[l], prv[l], a.dt2 * rm * lap, damp);
                if (a.src.n) un = fused_inject(a.src, q, 2, x, 0, z, rm, un, 1.0f);
                prv[l] = un;
            }
        }
        lds_barrier();
        float *t = cur;
        cur = prv;
        prv = t;
        // receivers of this step whose base node lies in the inner tile (they
        // read the new level, which the next step only reads)
        for (int r = tid; r < a.nrec; r += C::NT) {
            const int bx = a.rec_idx[3 * r], bz = a.rec_idx[3 * r + 2];
            if (bx < ix0 || bx >= ix0 + C::IX || bz < iz0 || bz >= iz0 + C::IZ) continue;
            {  // products rounded before the sums, as in the lane reduction
#pragma clang fp contract(off)
                const int l0 = (bz - pz0 + R) * C::LX + (bx - px0 + R);
                const float *w = a.rec_w + 4 * r;
                const float v0 = w[0] * cur[l0], v1 = w[1] * cur[l0 + 1];
                const float v2 = w[2] * cur[l0 + C::LX], v3 = w[3] * cur[l0 + C::LX + 1];
                a.rec_rows[(int64_t)j * a.nrec + r] = (v0 + v1) + (v2 + v3);
            }
        }
    }
    // the inner tile's last two levels
#pragma unroll
    for (int p = 0; p < C::PPT; ++p) {
        if (!(outmask & (1u << p))) continue;
        const int i = tid + C::NT * p;
        const int64_t gi = a.g.off0 + (int64_t)(pz0 + i / C::PX) * a.g.sz + (px0 + i % C::PX);
        a.out_cur[gi] = cur[lidx(i)];
        a.out_prev[gi] = prv[lidx(i)];
    }
}

template <int R>
static hipError_t launch_iso2d_tb_r(const TB2DArgs &a, hipStream_t s, const LaunchEvents &ev) {
    using C = TB2DCfg<R>;
    static_assert(C::PPT <= 32, "point mask holds 32 points per thread");
    static_assert(C::lds <= (size_t)kPersist2DMaxLds, "patch does not fit in LDS");
    if (a.nsteps < 1 || a.nsteps > C::K) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute((const void *)iso2d_tb<R>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)C::lds);
    if (e != hipSuccess) return e;
    const int tiles = ((a.g.nx + C::IX - 1) / C::IX) * ((a.g.nz + C::IZ - 1) / C::IZ);
    hipExtLaunchKernelGGL((iso2d_tb<R>), dim3((unsigned)tiles), dim3(C::NT), C::lds, s, ev.start, ev.stop, 0, a);
    return hipGetLastError();
}

TB2DShape tb2d_shape(int R) {
#define TBS(r) \
    case r: return TB2DShape{TB2DCfg<r>::K, TB2DCfg<r>::IX, TB2DCfg<r>::IZ};
    switch (R) { TBS(1) TBS(2) TBS(3) TBS(4) TBS(5) TBS(6) TBS(7) TBS(8) default: return TB2DShape{0, 0, 0}; }
#undef TBS
}

size_t tb2d_lds_bytes(int R) {
#define TBL(r) \
    case r: return TB2DCfg<r>::lds;
    switch (R) { TBL(1) TBL(2) TBL(3) TBL(4) TBL(5) TBL(6) TBL(7) TBL(8) default: return 0; }
#undef TBL
}

hipError_t launch_iso2d_tb(int R, const TB2DArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define TBR(r) launch_iso2d_tb_r<r>(a, s, ev)
    FDW_DISPATCH_R(R, TBR)
#undef TBR
}

}  // namespace fdw
