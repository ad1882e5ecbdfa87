// Isotropic acoustic 2D step on the ring-buffer z-streaming engine (gfx950):
// one launch per step for 2D grids too large for the LDS-resident persistent
// kernel.
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer).
//
// The engine's flat mode: a workgroup is one wavefront of 64 x-columns walking
// a z-chunk; z neighbours come from the register ring, x neighbours from one
// LDS row per plane, so every value of level t is read from HBM once (plus
// the warm-up planes of each chunk).  The point update is the
// one-thread-per-point kernel's term for term (Laplacian pair terms x before z
// at each distance, leapfrog, damping eta_x + eta_z, fused injection), so the
// two give the same bits.
#include "fdw_stream2.h"

namespace fdw {

struct IsoOp2D {
    static constexpr bool kBufferAccess = true;
    static constexpr bool kFlatY = true;
    Coefs c;
    const float *ex, *ez;  // damping per axis (x, z), already times dt / 2
    float dt2;
    FusedSrc src;
    float *u_next;
    float *save;  // optional second destination of the new level
    int adjoint;  // injected terms divided by (1 + a)
    __device__ __forceinline__ bool begin_tile(int x0, int tx, int y0, int ty, int z0, int z1) const {
        return src_in_tile(src, x0, tx, y0, ty, z0, z1);
    }
    __device__ __forceinline__ float begin_column(int x, int) const { return ((const gfloat *)ex)[x]; }
    __device__ __forceinline__ float begin_plane(int z) const { return ((const gfloat *)ez)[z]; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool src_here, float a, bool live) const {
#pragma clang fp contract(off)
        const float uc = pt.qz(0, 0);
        float lap = 0.0f;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lap = lap_term(lap, c.w2[0][k], pt.qx(0, k), pt.qx(0, -k), uc);
            lap = lap_term(lap, c.w2[2][k], pt.qz(0, k), pt.qz(0, -k), uc);
        }
        const float rm = fast_rcp(pt.p(1));
        float v = leapfrog(uc, pt.p(0), dt2 * rm * lap, a);
        if (src_here) v = fused_inject(src, src.q, 2, pt.x, 0, pt.z, rm, v, adjoint ? 1.0f / (1.0f + a) : 1.0f);
        if (live) {
            pt.store(u_next, v);
            if (save) pt.store(save, v);
        }
    }
};

// Grids whose step working set (two levels and m) exceeds the 256 MB
// last-level cache read u(t-1) and m with the non-temporal hint, leaving L2 to
// the re-read halo columns and warm-up rows of u (FDW_ISO2D_NT=0/1 overrides).
struct IsoOp2DNT : IsoOp2D {
    static constexpr bool kStreamingPointwise = true;
};
static bool iso2d_streaming_hint(const Geom &g) {
    if (const char *e = std::getenv("FDW_ISO2D_NT")) return e[0] == '1';
    return 3.0 * (double)g.sz * (double)g.nz * 4.0 > 256.0 * 1024.0 * 1024.0;
}

// z-chunk: the longest of 64, 32, ... planes that still gives 2048
// workgroups (one 64-column wavefront each), at least 4 (FDW_ISO2D_ZC
// overrides the longest, for tuning: at 8001^2 so 8, 64 planes 230 us per
// step, 128: 269, 256: 252)
static int iso2d_zchunk(const Geom &g) {
    static const int zmax = [] {
        const char *e = std::getenv("FDW_ISO2D_ZC");
        const int v = e ? std::atoi(e) : 0;
        return v >= 4 ? v : 64;
    }();
    const int64_t cols = (g.nx + 63) / 64;
    return adaptive_zchunk(cols, g.nz, zmax, 2048, 2048);
}

template <int R>
static hipError_t launch_stream2d_r(const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
    IsoOp2D op;
    op.c = a.c;
    op.ex = a.eta_x;
    op.ez = a.eta_z;
    op.dt2 = a.dt2;
    op.src = a.src;
    op.u_next = a.u_next;
    op.save = a.save;
    op.adjoint = a.adjoint;
    StreamFields<1, 2> F;
    F.q[0] = a.u_cur;
    F.p[0] = a.u_prev;
    F.p[1] = a.m;
    if (iso2d_streaming_hint(a.g)) {
        IsoOp2DNT w;
        static_cast<IsoOp2D &>(w) = op;
        return launch_stream3d_ring<R, 1, 2, 1>(w, F, a.g, iso2d_zchunk(a.g), s, ev.start, ev.stop, nullptr);
    }
    return launch_stream3d_ring<R, 1, 2, 1>(op, F, a.g, iso2d_zchunk(a.g), s, ev.start, ev.stop, nullptr);
}

hipError_t launch_iso2d_stream(int R, const IsoArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define ISO_S2(r) launch_stream2d_r<r>(a, s, ev)
    FDW_DISPATCH_R(R, ISO_S2)
#undef ISO_S2
}

int iso2d_stream_zchunk(const Geom &g) { return iso2d_zchunk(g); }

}  // namespace fdw
