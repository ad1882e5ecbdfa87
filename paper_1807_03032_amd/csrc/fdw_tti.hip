// TTI pseudo-acoustic step kernels (gfx950): stage 1 (rotated gradients)
// and stage 2 (rotated second derivatives, Laplacian, coupled update) on the
// z-streaming engine, plus the one-thread-per-point schedule.
// Paper: arXiv 1807.03032, Section 7.2 (two coupled acoustic equations with
// Laplacians built from rotated first derivatives) and Section 6 (the
// producer/consumer temporaries that the two-stage split corresponds to).
#include "fdw_device.h"

namespace fdw {

constexpr int kTti2DStreamMaxR = 8;

// Unit normal of the TTI symmetry axis: (sin th cos ph, sin th sin ph, cos th)
// in 3D, (sin th, cos th) over (x, z) in 2D.
template <int NDIM>
__device__ __forceinline__ void tti_normal(const TtiArgs &a, int64_t i, float &nx, float &ny, float &nz) {
    float st, ct;
    sincosf(a.theta[i], &st, &ct);
    if (NDIM == 3) {
        float sp, cp;
        sincosf(a.phi[i], &sp, &cp);
        nx = st * cp;
        ny = st * sp;
        nz = ct;
    } else {
        nx = st;
        ny = 0.0f;
        nz = ct;
    }
}

// n . grad f at element i (centred first derivatives of order 2R).
template <int NDIM, int R>
__device__ __forceinline__ float rot_grad(const float *f, int64_t i, const Geom &g, const Coefs &c, float nx,
                                          float ny, float nz) {
#pragma clang fp contract(off)
    float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        dx = d1_term(dx, c.w1[0][k], f[i + k], f[i - k]);
        dz = d1_term(dz, c.w1[2][k], f[i + k * g.sz], f[i - k * g.sz]);
        if (NDIM == 3) dy = d1_term(dy, c.w1[1][k], f[i + k * g.sy], f[i - k * g.sy]);
    }
    return dot3(nx, dx, ny, NDIM == 3 ? dy : 0.0f, nz, dz);
}

// TTI stage 1: gp = n . grad p, gr = n . grad r on every domain point.
template <int NDIM, int R>
__device__ __forceinline__ void tti_stage1_point(const TtiArgs &a, int x, int y, int z) {
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    float nx, ny, nz;
    tti_normal<NDIM>(a, i, nx, ny, nz);
    a.gp[i] = rot_grad<NDIM, R>(a.p_cur, i, a.g, a.c, nx, ny, nz);
    a.gr[i] = rot_grad<NDIM, R>(a.r_cur, i, a.g, a.c, nx, ny, nz);
}

template <int NDIM, int R>
__global__ void __launch_bounds__(256) tti_naive_stage1(TtiArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    tti_stage1_point<NDIM, R>(a, x, y, z);
}

// TTI stage 2: H p = n . grad gp, H r = n . grad gr, L p, coupled update.
template <int NDIM, int R>
__device__ __forceinline__ void tti_stage2_point(const TtiArgs &a, int x, int y, int z) {
#pragma clang fp contract(off)
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    float nx, ny, nz;
    tti_normal<NDIM>(a, i, nx, ny, nz);
    const float hp = rot_grad<NDIM, R>(a.gp, i, a.g, a.c, nx, ny, nz);
    const float hr = rot_grad<NDIM, R>(a.gr, i, a.g, a.c, nx, ny, nz);
    const float pc = a.p_cur[i];
    const float lap = laplacian_at<NDIM, R>(a.p_cur, i, a.g, a.c);
    const float d = damp_at(a.eta_x, a.eta_y, a.eta_z, NDIM, x, y, z);
    float pn, rn;
    tti_update(pc, a.p_prev[i], a.r_cur[i], a.r_prev[i], lap - hp, hr, a.m[i], a.eps[i], a.delta[i], a.dt2, d, pn,
               rn);
    const float rm = fast_rcp(a.m[i]);
    if (a.src.n) {  // the same injected sum into p and r
        const float inj = fused_inject(a.src, NDIM, x, y, z, rm, 0.0f);
        pn += inj;
        rn += inj;
    }
    a.p_next[i] = pn;
    a.r_next[i] = rn;
    if (a.save_p) {
        a.save_p[i] = pn;
        a.save_r[i] = rn;
    }
}

template <int NDIM, int R>
__global__ void __launch_bounds__(256) tti_naive_stage2(TtiArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    tti_stage2_point<NDIM, R>(a, x, y, z);
}

// 2D shots of one geometry in one launch: blockIdx.z selects the shot.
template <int R, int STAGE>
__global__ void __launch_bounds__(256) tti2d_naive_multi(const NaiveShot<TtiArgs> *__restrict__ shots) {
    const NaiveShot<TtiArgs> &S = shots[blockIdx.z];
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int z = blockIdx.y * blockDim.y + threadIdx.y;
    if (!S.live || x >= S.a.g.nx || z >= S.a.g.nz) return;
    if (STAGE == 1)
        tti_stage1_point<2, R>(S.a, x, 0, z);
    else
        tti_stage2_point<2, R>(S.a, x, 0, z);
}

// n = (sin th cos ph, sin th sin ph, cos th) with the hardware sin/cos
// (arguments in [0, 2 pi) after range reduction by the builtin).
__device__ __forceinline__ void tti_normal3(float th, float ph, float &nx, float &ny, float &nz) {
    const float st = __sinf(th), ct = __cosf(th), sp = __sinf(ph), cp = __cosf(ph);
    nx = st * cp;
    ny = st * sp;
    nz = ct;
}

// ---- TTI stage 1: stencil fields p, r; pointwise theta, phi ------------------
//   gp = n . grad p,  gr = n . grad r   (order-2R centred first derivatives)
struct TtiS1Op {
    static constexpr bool kBufferAccess = true;  // raw buffer (true) or global accesses
    Coefs c;
    float *gp, *gr;
    __device__ __forceinline__ bool begin_tile(int, int, int, int, int, int) const { return false; }
    __device__ __forceinline__ float begin_column(int, int) const { return 0.0f; }
    __device__ __forceinline__ float begin_plane(int) const { return 0.0f; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool, float, bool live) const {
#pragma clang fp contract(off)
        float nx, ny, nz;
        tti_normal3(pt.p(0), pt.p(1), nx, ny, nz);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx = d1_term(dx, c.w1[0][k], pt.qx(f, k), pt.qx(f, -k));
                dy = d1_term(dy, c.w1[1][k], pt.qy(f, k), pt.qy(f, -k));
                dz = d1_term(dz, c.w1[2][k], pt.qz(f, k), pt.qz(f, -k));
            }
            const float gv = dot3(nx, dx, ny, dy, nz, dz);
            if (live) pt.store(f == 0 ? gp : gr, gv);
        }
    }
};

// ---- TTI stage 2: stencil fields gp, gr, p; pointwise p(t-1), r(t), r(t-1),
// m, eps, delta, theta, phi --------------------------------------------------
//   Hp = n . grad gp, Hr = n . grad gr, A = L p - Hp, B = Hr
//   p+ from (1 + 2 eps) A + sqrt(1 + 2 delta) B, r+ from sqrt(1 + 2 delta) A + B
struct TtiS2Op {
    static constexpr bool kBufferAccess = true;  // raw buffer (true) or global accesses
    Coefs c;
    DampTables eta;
    float dt2;
    FusedSrc src;
    float *p_next, *r_next;
    float *save_p, *save_r;  // optional second destination of the new levels
    __device__ __forceinline__ bool begin_tile(int x0, int tx, int y0, int ty, int z0, int z1) const {
        return src_in_tile(src, x0, tx, y0, ty, z0, z1);
    }
    __device__ __forceinline__ float begin_column(int x, int y) const { return eta.column(x, y); }
    __device__ __forceinline__ float begin_plane(int z) const { return eta.plane(z); }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool src_here, float a, bool live) const {
#pragma clang fp contract(off)
        float nx, ny, nz;
        tti_normal3(pt.p(6), pt.p(7), nx, ny, nz);
        float h[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx = d1_term(dx, c.w1[0][k], pt.qx(f, k), pt.qx(f, -k));
                dy = d1_term(dy, c.w1[1][k], pt.qy(f, k), pt.qy(f, -k));
                dz = d1_term(dz, c.w1[2][k], pt.qz(f, k), pt.qz(f, -k));
            }
            h[f] = dot3(nx, dx, ny, dy, nz, dz);
        }
        const float pc = pt.qz(2, 0);
        float lap = 0.0f;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lap = lap_term(lap, c.w2[2][k], pt.qz(2, k), pt.qz(2, -k), pc);
            lap = lap_term(lap, c.w2[0][k], pt.qx(2, k), pt.qx(2, -k), pc);
            lap = lap_term(lap, c.w2[1][k], pt.qy(2, k), pt.qy(2, -k), pc);
        }
        float pn, rn;
        tti_update(pc, pt.p(0), pt.p(1), pt.p(2), lap - h[0], h[1], pt.p(3), pt.p(4), pt.p(5), dt2, a, pn, rn);
        const float rm = fast_rcp(pt.p(3));
        if (src_here) {
            const float inj = fused_inject(src, 3, pt.x, pt.y, pt.z, rm, 0.0f);
            pn += inj;
            rn += inj;
        }
        if (live) {
            pt.store(p_next, pn);
            pt.store(r_next, rn);
            if (save_p) {
                pt.store(save_p, pn);
                pt.store(save_r, rn);
            }
        }
    }
};

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int NDIM, int R>
static hipError_t launch_tti_naive(const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
    dim3 blk(64, 4, 1);
    dim3 grd = NDIM == 3 ? dim3((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz)
                         : dim3((a.g.nx + 63) / 64, (a.g.nz + 3) / 4, 1);
    hipExtLaunchKernelGGL((tti_naive_stage1<NDIM, R>), grd, blk, 0, s, ev.start, nullptr, 0, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipExtLaunchKernelGGL((tti_naive_stage2<NDIM, R>), grd, blk, 0, s, nullptr, ev.stop, 0, a);
    return hipGetLastError();
}

struct TtiShape {
    int ny1, by1, ny2, by2, zc;
};

// z-chunk of both stages: 64 for large grids, shorter when stage 2's 64 x 8
// tile columns are too few to occupy the chip, down to the longest chunk
// that still gives 1792 workgroups (three and a half rounds of the 512
// eight-wavefront slots; shorter chunks re-read 2R warm-up planes each:
// 300^3 order 12, 32 planes, 588 vs 615 us per step with 16; 200^3 keeps 8
// planes, 222 vs 229 us with 16); then evened out over the chunks the walk
// needs (400 planes: 7 chunks of 58 instead of six of 64 and one of 16,
// whose workgroups ran alone at the end: 1348 -> 1289 us per step at space
// order 12)
static int tti_default_zchunk(const Geom &g) {
    const int64_t cols = (int64_t)((g.nx + 63) / 64) * ((g.ny + 7) / 8);
    const int zc = adaptive_zchunk(cols, g.nz, 64, 2048, 1792);
    const int n = (g.nz + zc - 1) / zc;
    return (g.nz + n - 1) / n;
}

// Stage 1 64 x 16 (two columns per thread), stage 2 64 x 8; at space order 16
// on grids long enough for 32-plane chunks stage 2 takes 64 x 16 too (fewer
// halo rows per point: 400^3 1705 -> 1601 us per step, 512^3 3041 -> 2826;
// equal at 300^3, slower at order 12 and on small grids).
static TtiShape tti_stream_shape(const Geom &g, int R) {
    TtiShape sh{2, 8, 1, 8, tti_default_zchunk(g)};
    if (R == 8 && sh.zc >= 32) sh.ny2 = 2;
    if (const char *e = std::getenv("FDW_TTI_TILE")) {
        int a = 0, b = 0, c = 0, d = 0, z = 0;
        if (std::sscanf(e, "%d,%d,%d,%d,%d", &a, &b, &c, &d, &z) == 5 && (a == 1 || a == 2) && (b == 4 || b == 8) &&
            (c == 1 || c == 2) && (d == 4 || d == 8) && z >= 0)
            sh = TtiShape{a, b, c, d, z > 0 ? z : sh.zc};  // z = 0: the default z-chunk
    }
    if (sh.zc > g.nz) sh.zc = g.nz;
    return sh;
}

// Planes of loads in flight: two for stage 1 (two stencil fields) in its
// default 64 x 16 shape at space order 12 (2.42 -> 2.38 ms per 512^3 step),
// one elsewhere (stage 2 with two: 2.95 ms, its registers drop occupancy).
constexpr int tti_prefetch(int R, int NQ, int NY, int BY) { return R == 6 && NQ == 2 && NY == 2 && BY == 8 ? 2 : 1; }

template <int R, int NY, int BY, class Op, int NQ, int NP>
static hipError_t launch_tti_stage(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc, hipStream_t s,
                                   hipEvent_t e0, hipEvent_t e1, const SparseArgs *sp) {
    return launch_stream3d<R, NY, tti_prefetch(R, NQ, NY, BY), BY>(op, F, g, zc, s, e0, e1, sp);
}

// Tuning variants are instantiated for R = 6 and 8 (space orders 12 and 16);
// other orders use (NY, BY) = (2, 8) for stage 1 and (1, 8) for stage 2.
template <int R, class Op, int NQ, int NP>
static hipError_t launch_tti_stage_shape(int ny, int by, const Op &op, const StreamFields<NQ, NP> &F, const Geom &g,
                                         int zc, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                                         const SparseArgs *sp = nullptr) {
    if constexpr (R == 6 || R == 8) {
        if (ny == 2)
            return by == 8 ? launch_tti_stage<R, 2, 8>(op, F, g, zc, s, e0, e1, sp)
                           : launch_tti_stage<R, 2, 4>(op, F, g, zc, s, e0, e1, sp);
        return by == 8 ? launch_tti_stage<R, 1, 8>(op, F, g, zc, s, e0, e1, sp)
                       : launch_tti_stage<R, 1, 4>(op, F, g, zc, s, e0, e1, sp);
    } else {
        if (NQ == 2) return launch_tti_stage<R, 2, 8>(op, F, g, zc, s, e0, e1, sp);
        return launch_tti_stage<R, 1, 8>(op, F, g, zc, s, e0, e1, sp);
    }
}

static void tti_stage1_parts(const TtiArgs &a, TtiS1Op &o1, StreamFields<2, 2> &F1) {
    o1.c = a.c;
    o1.gp = a.gp;
    o1.gr = a.gr;
    F1.q[0] = a.p_cur;
    F1.q[1] = a.r_cur;
    F1.p[0] = a.theta;
    F1.p[1] = a.phi;
}

static void tti_stage2_parts(const TtiArgs &a, TtiS2Op &o2, StreamFields<3, 8> &F2) {
    o2.c = a.c;
    o2.eta = DampTables{a.eta_x, a.eta_y, a.eta_z};
    o2.dt2 = a.dt2;
    o2.src = a.src;
    o2.p_next = a.p_next;
    o2.r_next = a.r_next;
    o2.save_p = a.save_p;
    o2.save_r = a.save_r;
    F2.q[0] = a.gp;
    F2.q[1] = a.gr;
    F2.q[2] = a.p_cur;
    const float *pw[8] = {a.p_prev, a.r_cur, a.r_prev, a.m, a.eps, a.delta, a.theta, a.phi};
    for (int i = 0; i < 8; ++i) F2.p[i] = pw[i];
}

// Grids whose step working set exceeds the 256 MB last-level cache read the
// stages' once-read pointwise fields and write their outputs with the
// non-temporal hint, leaving L2 to the stencil fields' re-read halo rows and
// warm-up planes (512^3 order 12: 2.42 ms per step with plain accesses, 2.32
// with hinted loads, 2.28 with hinted stores too).  FDW_TTI_NT=0/1 overrides
// the choice.
static bool tti_streaming_hint(const Geom &g, int R) {
    if (const char *e = std::getenv("FDW_TTI_NT")) return e[0] == '1';
    const double field = (double)g.sz * (double)(g.nz + 2 * R) * 4.0;
    return 11.0 * field > 256.0 * 1024.0 * 1024.0;
}
struct TtiS1OpNT : TtiS1Op {
    static constexpr bool kStreamingPointwise = true;
    static constexpr bool kStreamingStores = true;
};
struct TtiS2OpNT : TtiS2Op {
    static constexpr bool kStreamingPointwise = true;
    static constexpr bool kStreamingStores = true;
};

template <int R, class Op1, class Op2>
static hipError_t launch_tti3d_stream_ops(const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
    const TtiShape sh = tti_stream_shape(a.g, R);
    Op1 o1;
    StreamFields<2, 2> F1;
    tti_stage1_parts(a, static_cast<TtiS1Op &>(o1), F1);
    hipError_t e = launch_tti_stage_shape<R>(sh.ny1, sh.by1, o1, F1, a.g, sh.zc, s, ev.start, nullptr, a.rec);
    if (e != hipSuccess) return e;
    Op2 o2;
    StreamFields<3, 8> F2;
    tti_stage2_parts(a, static_cast<TtiS2Op &>(o2), F2);
    return launch_tti_stage_shape<R>(sh.ny2, sh.by2, o2, F2, a.g, sh.zc, s, nullptr, ev.stop);
}

template <int R>
static hipError_t launch_tti3d_stream(const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
    if (tti_streaming_hint(a.g, R)) return launch_tti3d_stream_ops<R, TtiS1OpNT, TtiS2OpNT>(a, s, ev);
    return launch_tti3d_stream_ops<R, TtiS1Op, TtiS2Op>(a, s, ev);
}

// ---------------------------------------------------------------------------
// Fused multi-shot steps (same geometry and space order)
// ---------------------------------------------------------------------------
using TtiShot1 = StreamShot<TtiS1Op, 2, 2>;
using TtiShot2 = StreamShot<TtiS2Op, 3, 8>;

size_t tti_multi_record_bytes(int ndim, int stage) {
    if (ndim != 3) return sizeof(NaiveShot<TtiArgs>);
    return stage == 1 ? sizeof(TtiShot1) : sizeof(TtiShot2);
}

void multi_pack_tti(int ndim, const TtiArgs &a, bool live, const SparseArgs &rec, void *dst1, void *dst2) {
    if (ndim == 3) {
        TtiShot1 r1;
        TtiShot2 r2;
        std::memset(&r1, 0, sizeof(r1));
        std::memset(&r2, 0, sizeof(r2));
        tti_stage1_parts(a, r1.op, r1.F);
        tti_stage2_parts(a, r2.op, r2.F);
        r1.rec = rec;  // sampled by stage 1, which only reads p(t)
        r1.live = r2.live = live ? 1 : 0;
        std::memcpy(dst1, &r1, sizeof(r1));
        std::memcpy(dst2, &r2, sizeof(r2));
    } else {
        NaiveShot<TtiArgs> r;
        std::memset(&r, 0, sizeof(r));
        r.a = a;
        r.a.rec = nullptr;  // host pointer: never read on the device
        r.live = live ? 1 : 0;
        std::memcpy(dst1, &r, sizeof(r));
    }
}

template <int R>
static hipError_t launch_tti_multi_r(int ndim, const Geom &g, const void *recs1, const void *recs2, int n,
                                     int64_t max_rec, hipStream_t s) {
    if (ndim == 3) {
        constexpr int NY1 = 2, BY1 = 8, NY2 = 1, BY2 = 8;
        const int zc = tti_default_zchunk(g);
        hipError_t e = launch_stream3d_multi<R, NY1, tti_prefetch(R, 2, NY1, BY1), BY1>(
            static_cast<const TtiShot1 *>(recs1), n, max_rec, g, zc, s);
        if (e != hipSuccess) return e;
        return launch_stream3d_multi<R, NY2, 1, BY2>(static_cast<const TtiShot2 *>(recs2), n, 0, g, zc, s);
    }
    const auto *sh = static_cast<const NaiveShot<TtiArgs> *>(recs1);
    dim3 blk(64, 4, 1), grd((g.nx + 63) / 64, (g.nz + 3) / 4, n);
    hipLaunchKernelGGL((tti2d_naive_multi<R, 1>), grd, blk, 0, s, sh);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((tti2d_naive_multi<R, 2>), grd, blk, 0, s, sh);
    return hipGetLastError();
}

hipError_t launch_tti_multi(int ndim, int R, const Geom &g, const void *recs1, const void *recs2, int n,
                            int64_t max_rec, hipStream_t s) {
    if (n <= 0) return hipSuccess;
#define TTI_M(r) launch_tti_multi_r<r>(ndim, g, recs1, recs2, n, max_rec, s)
    FDW_DISPATCH_R(R, TTI_M)
#undef TTI_M
}

// orders whose 2D stages run on the flat ring engine (the others would copy
// their operator record to scratch memory there)
static bool tti2d_stream_order(int R) { return R <= kTti2DStreamMaxR; }

hipError_t launch_tti(int ndim, int R, TtiVariant v, const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define TTI_S3(r) launch_tti3d_stream<r>(a, s, ev)
    if (ndim == 3 && v == TtiVariant::Stream) { FDW_DISPATCH_R(R, TTI_S3) }
#undef TTI_S3
    if (ndim == 2 && v == TtiVariant::Stream && tti2d_stream_order(R)) return launch_tti2d_stream(R, a, s, ev);
#define TTI_N3(r) launch_tti_naive<3, r>(a, s, ev)
#define TTI_N2(r) launch_tti_naive<2, r>(a, s, ev)
    if (ndim == 3) { FDW_DISPATCH_R(R, TTI_N3) }
    FDW_DISPATCH_R(R, TTI_N2)
#undef TTI_N3
#undef TTI_N2
}
const char *tti_kernel_name(int ndim, int R, TtiVariant v, const Geom &g) {
    if (ndim == 2 && v == TtiVariant::Stream && tti2d_stream_order(R)) {
        static thread_local char buf2[80];
        std::snprintf(buf2, sizeof(buf2), "tti2d_stream 64-column wavefronts zchunk=%d", tti2d_stream_zchunk(g));
        return buf2;
    }
    if (ndim == 3 && v == TtiVariant::Stream) {
        static thread_local char buf[96];
        const TtiShape sh = tti_stream_shape(g, R);
        std::snprintf(buf, sizeof(buf), "tti3d_stream stage1 tile=64x%d stage2 tile=64x%d zchunk=%d%s",
                      sh.by1 * sh.ny1, sh.by2 * sh.ny2, sh.zc, tti_streaming_hint(g, R) ? " pointwise=nt" : "");
        return buf;
    }
    return ndim == 3 ? "tti_naive_stage1+2<3>" : "tti_naive_stage1+2<2>";
}

}  // namespace fdw
