// Isotropic acoustic step kernels (gfx950): 3D z-streaming operator, the
// one-thread-per-point schedule, and the LDS-resident persistent 2D kernel.
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer, test cases).
#include "fdw_device.h"

namespace fdw {

// ---------------------------------------------------------------------------
// Naive kernels: one thread per grid point, every neighbour loaded from
// global memory (cache-served).  Kept as the simplest correct schedule and as
// the fallback for shapes the streaming kernels do not cover.
// ---------------------------------------------------------------------------

template <int NDIM, int R>
__device__ __forceinline__ void iso_naive_point(const IsoArgs &a, int x, int y, int z) {
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    const float *u = a.u_cur;
    const float uc = u[i];
    const float lap = laplacian_at<NDIM, R>(u, i, a.g, a.c);
    const float rm = fast_rcp(a.m[i]);
    const float d = damp_at(a.eta_x, a.eta_y, a.eta_z, NDIM, x, y, z);
    float un = leapfrog(uc, a.u_prev[i], a.dt2 * rm * lap, d);
    if (a.src.n) un = fused_inject(a.src, NDIM, x, y, z, rm, un, a.adjoint ? 1.0f / (1.0f + d) : 1.0f);
    a.u_next[i] = un;
    if (a.save) a.save[i] = un;
}

template <int NDIM, int R>
__global__ void __launch_bounds__(256) iso_naive(IsoArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    iso_naive_point<NDIM, R>(a, x, y, z);
}

// 2D shots of one geometry in one launch: blockIdx.z selects the shot.
template <int R>
__global__ void __launch_bounds__(256) iso2d_naive_multi(const NaiveShot<IsoArgs> *__restrict__ shots) {
    const NaiveShot<IsoArgs> &S = shots[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y * blockDim.y + threadIdx.y;
    if (!S.live || x >= S.a.g.nx || z >= S.a.g.nz) return;
    iso_naive_point<2, R>(S.a, x, 0, z);
}

// ---- isotropic step: stencil field u(t); pointwise u(t-1), m ----------------
struct IsoOp {
    static constexpr bool kBufferAccess = false;  // raw buffer (true) or global accesses
    Coefs c;
    DampTables eta;
    float dt2;
    FusedSrc src;
    float *u_next;
    float *save;   // optional second destination of the new level
    int adjoint;   // injected terms divided by (1 + a)
    // does a fused source touch this tile and chunk?
    __device__ __forceinline__ bool begin_tile(int x0, int tx, int y0, int ty, int z0, int z1) const {
        return src_in_tile(src, x0, tx, y0, ty, z0, z1);
    }
    // damping: eta_x + eta_y per column, + eta_z per plane
    __device__ __forceinline__ float begin_column(int x, int y) const { return eta.column(x, y); }
    __device__ __forceinline__ float begin_plane(int z) const { return eta.plane(z); }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool src_here, float a, bool live) const {
        const float uc = pt.qz(0, 0);
        const float u2 = 2.0f * uc;
        // Laplacian as sum_k w_k ((u+k + u-k) - 2u): no centre weight, so
        // rounding the weights cannot add a spurious mass term
        float lap = 0.0f;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lap += c.w2[2][k] * ((pt.qz(0, k) + pt.qz(0, -k)) - u2);
            lap += c.w2[0][k] * ((pt.qx(0, k) + pt.qx(0, -k)) - u2);
            lap += c.w2[1][k] * ((pt.qy(0, k) + pt.qy(0, -k)) - u2);
        }
        const float rm = fast_rcp(pt.p(1));
        float v = leapfrog(uc, pt.p(0), dt2 * rm * lap, a);
        if (src_here) v = fused_inject(src, 3, pt.x, pt.y, pt.z, rm, v, adjoint ? 1.0f / (1.0f + a) : 1.0f);
        if (live) {
            pt.store(u_next, v);
            if (save) pt.store(save, v);
        }
    }
};

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
                const float u2 = 2.0f * uc;
                float lap = 0.0f;
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    const float xp = (HALO || x + k < nx) ? cur[l + k] : 0.0f;
                    const float xm = (HALO || x - k >= 0) ? cur[l - k] : 0.0f;
                    const float zp = (HALO || z + k < nz) ? cur[l + k * lw] : 0.0f;
                    const float zm = (HALO || z - k >= 0) ? cur[l - k * lw] : 0.0f;
                    lap += a.c.w2[0][k] * ((xp + xm) - u2);
                    lap += a.c.w2[2][k] * ((zp + zm) - u2);
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

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int NDIM, int R>
static hipError_t launch_iso_naive(const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
    dim3 blk(64, 4, 1);
    dim3 grd = NDIM == 3 ? dim3((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz)
                         : dim3((a.g.nx + 63) / 64, (a.g.nz + 3) / 4, 1);
    hipExtLaunchKernelGGL((iso_naive<NDIM, R>), grd, blk, 0, s, ev.start, ev.stop, 0, a);
    return hipGetLastError();
}

// Tile shapes are (NY y-columns per thread, BY wavefronts per workgroup, z-chunk
// ZC, prefetch PF); tile = 64 x (NY * BY).  Environment overrides for tuning:
//   FDW_ISO_TILE="NY,ZC,PF,BY"   FDW_TTI_TILE="NY1,BY1,NY2,BY2,ZC"
struct IsoShape {
    int ny, zc, pf, by;
};

// default shape 64 x 8 tile, 4 waves, prefetch 2; z-chunk 32 for large grids,
// shorter when the grid has too few tile columns to occupy the chip
static int iso_default_zchunk(const Geom &g) {
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    return adaptive_zchunk(cols, g.nz, 32, 1024, 2048);
}

static IsoShape iso_stream_shape(const Geom &g) {
    IsoShape sh{2, iso_default_zchunk(g), 2, 4};
    if (const char *e = std::getenv("FDW_ISO_TILE")) {
        int a = 0, b = 0, c = 1, d = 4;
        const int n = std::sscanf(e, "%d,%d,%d,%d", &a, &b, &c, &d);
        if (n >= 2 && (a == 1 || a == 2 || a == 4) && b > 0 && (c == 1 || c == 2) && (d == 4 || d == 8))
            sh = IsoShape{a, b, c, d};
    }
    if (sh.zc > g.nz) sh.zc = g.nz;
    return sh;
}

static IsoOp make_iso_op(const IsoArgs &a);

// Fields of 4 GiB or more are beyond the global accesses' 32-bit byte
// offsets: they take the raw buffer form (offsets within one plane).
struct IsoOpWide : IsoOp {
    static constexpr bool kBufferAccess = true;
};
// (FDW_ISO_WIDE=1 takes the wide form on any grid: checks of that path)
static bool iso_wide_form(const Geom &g) {
    const char *e = std::getenv("FDW_ISO_WIDE");
    return (e && e[0] == '1') || iso_wide_fields(g);
}
static StreamFields<1, 2> iso_fields(const IsoArgs &a);

template <int R, int NY, int PF, int BY>
static hipError_t launch_iso3d_stream_cfg(const IsoArgs &a, int zc, hipStream_t s, const LaunchEvents &ev) {
    return launch_stream3d<R, NY, PF, BY>(make_iso_op(a), iso_fields(a), a.g, zc, s, ev.start, ev.stop, a.rec);
}

template <int R, int NY, int PF>
static hipError_t launch_iso3d_stream_by(const IsoArgs &a, const IsoShape &sh, hipStream_t s, const LaunchEvents &ev) {
    if (sh.by == 8) return launch_iso3d_stream_cfg<R, NY, PF, 8>(a, sh.zc, s, ev);
    return launch_iso3d_stream_cfg<R, NY, PF, 4>(a, sh.zc, s, ev);
}

template <int R, int NY>
static hipError_t launch_iso3d_stream_ny(const IsoArgs &a, const IsoShape &sh, hipStream_t s, const LaunchEvents &ev) {
    if (sh.pf == 2) return launch_iso3d_stream_by<R, NY, 2>(a, sh, s, ev);
    return launch_iso3d_stream_by<R, NY, 1>(a, sh, s, ev);
}

// Tuning variants are instantiated for R = 4 (space order 8) only; other
// orders use the default shape.
template <int R>
static hipError_t launch_iso3d_stream(const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
    const IsoShape sh = iso_stream_shape(a.g);
    // FDW_ISO_WIDE=1 takes the wide form on any grid (checks of that path)
    if (iso_wide_form(a.g))
        return launch_stream3d<R, 2, 2, 4>(IsoOpWide{make_iso_op(a)}, iso_fields(a), a.g, sh.zc, s, ev.start, ev.stop,
                                           a.rec);
    if constexpr (R == 4) {
        if (sh.ny == 1) return launch_iso3d_stream_ny<R, 1>(a, sh, s, ev);
        if (sh.ny == 2) return launch_iso3d_stream_ny<R, 2>(a, sh, s, ev);
        return launch_iso3d_stream_ny<R, 4>(a, sh, s, ev);
    } else {
        return launch_iso3d_stream_cfg<R, 2, 2, 4>(a, sh.zc, s, ev);
    }
}

hipError_t launch_iso(int ndim, int R, IsoVariant v, const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define ISO_S3(r) launch_iso3d_stream<r>(a, s, ev)
    if (ndim == 3 && v == IsoVariant::Stream) { FDW_DISPATCH_R(R, ISO_S3) }
#undef ISO_S3
#define ISO_N3(r) launch_iso_naive<3, r>(a, s, ev)
#define ISO_N2(r) launch_iso_naive<2, r>(a, s, ev)
    if (ndim == 3) { FDW_DISPATCH_R(R, ISO_N3) }
    FDW_DISPATCH_R(R, ISO_N2)
#undef ISO_N3
#undef ISO_N2
}

// ---------------------------------------------------------------------------
// Fused multi-shot steps (same geometry and space order)
// ---------------------------------------------------------------------------
static IsoOp make_iso_op(const IsoArgs &a) {
    IsoOp op;
    op.c = a.c;
    op.eta = DampTables{a.eta_x, a.eta_y, a.eta_z};
    op.dt2 = a.dt2;
    op.src = a.src;
    op.u_next = a.u_next;
    op.save = a.save;
    op.adjoint = a.adjoint;
    return op;
}

static StreamFields<1, 2> iso_fields(const IsoArgs &a) {
    StreamFields<1, 2> F;
    F.q[0] = a.u_cur;
    F.p[0] = a.u_prev;
    F.p[1] = a.m;
    return F;
}

using IsoShot3 = StreamShot<IsoOp, 1, 2>;

size_t iso_multi_record_bytes(int ndim) { return ndim == 3 ? sizeof(IsoShot3) : sizeof(NaiveShot<IsoArgs>); }

void multi_pack_iso(int ndim, const IsoArgs &a, bool live, const SparseArgs &rec, void *dst) {
    if (ndim == 3) {
        IsoShot3 r;
        std::memset(&r, 0, sizeof(r));
        r.op = make_iso_op(a);
        r.F = iso_fields(a);
        r.rec = rec;
        r.live = live ? 1 : 0;
        std::memcpy(dst, &r, sizeof(r));
    } else {
        NaiveShot<IsoArgs> r;
        std::memset(&r, 0, sizeof(r));
        r.a = a;
        r.a.rec = nullptr;  // host pointer: never read on the device
        r.live = live ? 1 : 0;
        std::memcpy(dst, &r, sizeof(r));
    }
}

template <int R>
static hipError_t launch_iso_multi_r(int ndim, const Geom &g, const void *recs, int n, int64_t rec_lanes,
                                     hipStream_t s) {
    if (ndim == 3) {
        return launch_stream3d_multi<R, 2, 2, 4>(static_cast<const IsoShot3 *>(recs), n, rec_lanes, g,
                                                 iso_default_zchunk(g), s);
    }
    dim3 blk(64, 4, 1), grd((g.nx + 63) / 64, (g.nz + 3) / 4, n);
    hipLaunchKernelGGL((iso2d_naive_multi<R>), grd, blk, 0, s, static_cast<const NaiveShot<IsoArgs> *>(recs));
    return hipGetLastError();
}

hipError_t launch_iso_multi(int ndim, int R, const Geom &g, const void *recs, int n, int64_t rec_lanes,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define ISO_M(r) launch_iso_multi_r<r>(ndim, g, recs, n, rec_lanes, s)
    FDW_DISPATCH_R(R, ISO_M)
#undef ISO_M
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

template <int R>
static hipError_t launch_iso2d_persistent_r(const Persist2DArgs &a, hipStream_t s, const LaunchEvents &ev) {
    const size_t halo = sizeof(float) * (size_t)(a.g.nx + 2 * R) * (size_t)(a.g.nz + 2 * R);
    if (halo <= (size_t)kPersist2DMaxLds) return launch_iso2d_persistent_h<R, true>(a, halo, s, ev);
    return launch_iso2d_persistent_h<R, false>(a, sizeof(float) * (size_t)a.g.nx * a.g.nz, s, ev);
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

template <int R>
static hipError_t launch_iso2d_persistent_multi_r(const Geom &g, const Persist2DArgs *shots, int n, hipStream_t s) {
    const size_t halo = sizeof(float) * (size_t)(g.nx + 2 * R) * (size_t)(g.nz + 2 * R);
    if (halo <= (size_t)kPersist2DMaxLds) return launch_iso2d_persistent_multi_h<R, true>(g, shots, n, halo, s);
    return launch_iso2d_persistent_multi_h<R, false>(g, shots, n, sizeof(float) * (size_t)g.nx * g.nz, s);
}

hipError_t launch_iso2d_persistent_multi(int R, const Geom &g, const Persist2DArgs *shots, int n, hipStream_t s) {
    if ((size_t)g.nx * g.nz * sizeof(float) > (size_t)kPersist2DMaxLds || n <= 0) return hipErrorInvalidValue;
#define P2MR(r) launch_iso2d_persistent_multi_r<r>(g, shots, n, s)
    FDW_DISPATCH_R(R, P2MR)
#undef P2MR
}

hipError_t launch_iso2d_persistent(int R, const Persist2DArgs &a, hipStream_t s, const LaunchEvents &ev) {
    if ((size_t)a.g.nx * a.g.nz * sizeof(float) > (size_t)kPersist2DMaxLds) return hipErrorInvalidValue;
#define P2R(r) launch_iso2d_persistent_r<r>(a, s, ev)
    FDW_DISPATCH_R(R, P2R)
#undef P2R
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

const char *iso_kernel_name(int ndim, IsoVariant v, const Geom &g) {
    if (ndim == 3 && v == IsoVariant::Stream) {
        static thread_local char buf[96];
        const IsoShape sh = iso_stream_shape(g);
        if (iso_wide_form(g))
            std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x8 (4 waves) zchunk=%d prefetch=2 wide", sh.zc);
        else
            std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x%d (%d waves) zchunk=%d prefetch=%d", sh.by * sh.ny,
                          sh.by, sh.zc, sh.pf);
        return buf;
    }
    return ndim == 3 ? "iso_naive<3>" : "iso_naive<2>";
}

}  // namespace fdw
