// Isotropic acoustic step kernels (gfx950): 3D z-streaming operator, the
// one-thread-per-point schedule, and the LDS-resident persistent 2D kernel.
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer, test cases).
#include "fdw_device.h"
#include "fdw_iso_op.h"
#include "fdw_stream2.h"

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

// sampling: receivers are sampled by extra workgroups of the launch, which
// the hardware dispatches after the stencil workgroups; chunks that give two
// rounds of stencil workgroups (2048 rather than 1024) let them overlap the
// second round (256^3 with 65,536 receivers: 49.0-50.0 vs 50.7 us per step;
// without receivers the 1024-workgroup chunks are faster)
static IsoShape iso_stream_shape(const Geom &g, bool sampling) {
    IsoShape sh{2, iso_default_zchunk(g), 2, 4};
    if (sampling) {
        const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
        sh.zc = adaptive_zchunk(cols, g.nz, 32, 2048, 2048);
    }
    // grids with 2048 or more 64 x 16 tile chunks of 64 planes (512^3 and up)
    // take that shape (8 waves): half the y-halo rows and warm-up planes per
    // point of the 64 x 8 x 32 default (512^3: 451 vs 470 us per step)
    const int64_t cols16 = (int64_t)((g.nx + 63) / 64) * ((g.ny + 15) / 16);
    const int64_t chunks16 = cols16 * ((g.nz + 63) / 64);
    // (or one round of them fills nine tenths of the 512 eight-wavefront
    // workgroup slots: 320^3, 500 chunks, 129.5 vs 132.8 us per step with
    // the imaging factor stored)
    if (chunks16 >= 2048 || (chunks16 >= 461 && chunks16 <= 512)) sh = IsoShape{2, 64, 2, 8};
    // the chunks a walk needs, evened out (400 planes: 13 of 31 rather than
    // 12 of 32 and one of 16; grids that are multiples of the chunk keep it)
    if (sh.zc < g.nz) {
        const int n = (g.nz + sh.zc - 1) / sh.zc;
        sh.zc = (g.nz + n - 1) / n;
    }
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

// engine of the 3D isotropic step: the ring-buffer engine at orders up to 8
// (FDW_ENGINE=1 forces the shifting-queue engine), the shifting-queue engine
// above (there the ring kernel copies its operator record to scratch memory)
static bool iso_ring_engine(int R) {
    static const bool ring = [] {
        const char *e = std::getenv("FDW_ENGINE");
        return !(e && e[0] == '1');
    }();
    return ring && R <= 4;
}

// Fields of 4 GiB or more are beyond the global accesses' 32-bit byte
// offsets: the shifting-queue engine takes its raw buffer form for them (the
// ring engine is buffer-addressed at any size).
struct IsoOpWide : IsoOp {
    static constexpr bool kBufferAccess = true;
};
// (FDW_ISO_WIDE=1 takes the wide form on any grid: checks of that path)
static bool iso_wide_form(const Geom &g, int R) {
    const char *e = std::getenv("FDW_ISO_WIDE");
    return (e && e[0] == '1') || (iso_wide_fields(g) && !iso_ring_engine(R));
}
static StreamFields<1, 2> iso_fields(const IsoArgs &a);

// Pointwise fields read with the non-temporal hint, so that the L2 keeps more
// of the stencil field's re-read halo rows and warm-up planes:
//   2: all of them (u(t-1), m; the imaging step's S and gradient too) on
//      grids whose step working set (two levels and m) exceeds the 256 MB
//      last-level cache (512^3: counted traffic 1.18 -> 1.09x, 449.7 ->
//      438.5 us per step);
//   1: u(t-1) only on smaller grids, which keep m in the last-level cache
//      from step to step (256^3: 48.8 -> 48.3 us; with m too, 53.5 us);
//   0: none.
// FDW_ISO_NT=0/u/1 overrides the choice (0, 1, 2).
static int iso_streaming_mode(const Geom &g, int R) {
    if (const char *e = std::getenv("FDW_ISO_NT")) return e[0] == '1' ? 2 : e[0] == 'u' ? 1 : 0;
    const double field = (double)g.sz * (double)(g.nz + 2 * R) * 4.0;
    return 3.0 * field > 256.0 * 1024.0 * 1024.0 ? 2 : 1;
}
struct IsoOpNT : IsoOp {  // u(t + 1) written with the hint too (512^3: 439.4 -> 431 us)
    static constexpr bool kStreamingPointwise = true;
    static constexpr bool kStreamingStores = true;
};
struct IsoOpNTu : IsoOp {  // u(t-1) only
    static constexpr bool kStreamingPointwise = true;
    static constexpr unsigned kStreamingMask = 1u;
};
struct IsoImgOpNT : IsoImgOp {
    static constexpr bool kStreamingPointwise = true;
};

template <int R, int NY, int PF, int BY>
static hipError_t launch_iso3d_stream_cfg(const IsoArgs &a, int zc, hipStream_t s, const LaunchEvents &ev) {
    if constexpr (R <= 4) {
        if (iso_ring_engine(R)) {
            const int mode = iso_streaming_mode(a.g, R);
            if (mode == 2)
                return launch_stream3d_ring<R, NY, PF, BY>(IsoOpNT{make_iso_op(a)}, iso_fields(a), a.g, zc, s,
                                                           ev.start, ev.stop, a.rec);
            if (mode == 1)
                return launch_stream3d_ring<R, NY, PF, BY>(IsoOpNTu{make_iso_op(a)}, iso_fields(a), a.g, zc, s,
                                                           ev.start, ev.stop, a.rec);
            return launch_stream3d_ring<R, NY, PF, BY>(make_iso_op(a), iso_fields(a), a.g, zc, s, ev.start, ev.stop,
                                                       a.rec);
        }
    }
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

// Adjoint step fused with the imaging condition of its centre level (IsoImgOp:
// pointwise u(t-1), m, imaging factor, gradient), in one tile shape per order:
// 64 x 8, four wavefronts; loads one plane ahead in the ring engine (two
// would exceed its 128 registers at order 8; one column per thread in eight
// wavefronts with two planes ahead fits in 80 but ran 17 % slower), two in
// the shifting-queue one (10 % slower than the ring at 320^3).
struct IsoImgOpWide : IsoImgOp {
    static constexpr bool kBufferAccess = true;
};
// Its z-chunk: the longest of 64, 32, 16 ... planes whose 64 x 8 tile chunks
// still fill nine tenths of the chip's 1024 four-wavefront workgroup slots
// (it moves 28 bytes per point, 4 of them re-read at chunk ends: 320^3 with
// 64-plane chunks, 1000 workgroups, 0.32 s per 1500-step gradient against
// 0.35 s with the forward step's 32; 64 x 16 tiles of eight wavefronts
// measured no faster).
static int image_zchunk(const Geom &g) {
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    int zc = 64;
    while (zc > 4 && cols * ((g.nz + zc - 1) / zc) < 920) zc /= 2;
    return std::min(zc, g.nz);
}

template <int R>
static hipError_t launch_iso3d_image(const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
    IsoImgOp op;
    static_cast<IsoOp &>(op) = make_iso_op(a);
    op.grad = a.grad;
    op.inv_dt2 = a.inv_dt2;
    StreamFields<1, 4> F;
    F.q[0] = a.u_cur;
    F.p[0] = a.u_prev;
    F.p[1] = a.m;
    F.p[2] = a.img_s;
    F.p[3] = a.grad;
    const int zc = image_zchunk(a.g);
    if constexpr (R <= 4) {
        if (iso_ring_engine(R)) {
            if (iso_streaming_mode(a.g, R) == 2) {
                IsoImgOpNT w;
                static_cast<IsoImgOp &>(w) = op;
                return launch_stream3d_ring<R, 2, 1, 4>(w, F, a.g, zc, s, ev.start, ev.stop, a.rec);
            }
            return launch_stream3d_ring<R, 2, 1, 4>(op, F, a.g, zc, s, ev.start, ev.stop, a.rec);
        }
    }
    if (iso_wide_form(a.g, R)) {
        IsoImgOpWide w;
        static_cast<IsoImgOp &>(w) = op;
        return launch_stream3d<R, 2, 2, 4>(w, F, a.g, zc, s, ev.start, ev.stop, a.rec);
    }
    return launch_stream3d<R, 2, 2, 4>(op, F, a.g, zc, s, ev.start, ev.stop, a.rec);
}

// Tuning variants are instantiated for R = 4 (space order 8) only; other
// orders use the default shape.
template <int R>
static hipError_t launch_iso3d_stream(const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
    const IsoShape sh = iso_stream_shape(a.g, a.sampling != 0);
    if (a.img_s) return launch_iso3d_image<R>(a, s, ev);
    // FDW_ISO_WIDE=1 takes the wide form on any grid (checks of that path)
    if (iso_wide_form(a.g, R))
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
    // (order 16 stays one thread per point: there the ring kernel would copy
    // its operator record to scratch memory)
    if (ndim == 2 && v == IsoVariant::Stream && R < 8) return launch_iso2d_stream(R, a, s, ev);
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
    op.isave = a.isave;
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
static hipError_t launch_iso_multi_r(int ndim, const Geom &g, const void *recs, int n, int64_t max_rec,
                                     hipStream_t s) {
    if (ndim == 3) {
        return launch_stream3d_multi<R, 2, 2, 4>(static_cast<const IsoShot3 *>(recs), n, max_rec, g,
                                                 iso_default_zchunk(g), s);
    }
    dim3 blk(64, 4, 1), grd((g.nx + 63) / 64, (g.nz + 3) / 4, n);
    hipLaunchKernelGGL((iso2d_naive_multi<R>), grd, blk, 0, s, static_cast<const NaiveShot<IsoArgs> *>(recs));
    return hipGetLastError();
}

hipError_t launch_iso_multi(int ndim, int R, const Geom &g, const void *recs, int n, int64_t max_rec,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define ISO_M(r) launch_iso_multi_r<r>(ndim, g, recs, n, max_rec, s)
    FDW_DISPATCH_R(R, ISO_M)
#undef ISO_M
}

const char *iso_kernel_name(int ndim, int R, IsoVariant v, const Geom &g, bool sampling) {
    if (ndim == 3 && v == IsoVariant::Stream) {
        static thread_local char buf[96];
        const IsoShape sh = iso_stream_shape(g, sampling);
        if (iso_wide_form(g, R))
            std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x8 (4 waves) zchunk=%d prefetch=2 wide", sh.zc);
        else
            std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x%d (%d waves) zchunk=%d prefetch=%d%s",
                          sh.by * sh.ny, sh.by, sh.zc, sh.pf,
                          !iso_ring_engine(R)                 ? ""
                          : iso_streaming_mode(g, R) == 2 ? " pointwise=nt"
                          : iso_streaming_mode(g, R) == 1 ? " pointwise=nt(u(t-1))"
                                                          : "");
        return buf;
    }
    if (ndim == 2 && v == IsoVariant::Stream && R < 8) {
        static thread_local char buf2[64];
        std::snprintf(buf2, sizeof(buf2), "iso2d_stream 64-column wavefronts zchunk=%d prefetch=2",
                      iso2d_stream_zchunk(g));
        return buf2;
    }
    return ndim == 3 ? "iso_naive<3>" : "iso_naive<2>";
}

}  // namespace fdw
