// TTI 2D stages on the ring-buffer z-streaming engine's flat mode (gfx950):
// one 64-column wavefront per workgroup walks a z-chunk, z neighbours from
// the register ring, x neighbours from one LDS row per plane.
// Paper: arXiv 1807.03032, Section 7.2 (two coupled acoustic equations with
// Laplacians built from rotated first derivatives), Section 6 (the
// producer/consumer split).
//
// The point updates are the one-thread-per-point 2D kernels' term for term
// (n = (sin th, cos th) over (x, z) with sincosf, first-derivative terms x
// before z at each distance, n . grad with the z term last, Laplacian pair
// terms x before z, the coupled leapfrog, damping eta_x + eta_z, the
// injected sum added to p and r), so both schedules, and the fused
// multi-shot 2D kernels, give the same bits.
#include "fdw_stream2.h"

namespace fdw {

// stage 1: stencil fields p, r; pointwise theta -> gp = n . grad p, gr = n . grad r
struct TtiS1Op2D {
    static constexpr bool kBufferAccess = true;
    static constexpr bool kFlatY = true;
    Coefs c;
    float *gp, *gr;
    __device__ __forceinline__ bool begin_tile(int, int, int, int, int, int) const { return false; }
    __device__ __forceinline__ float begin_column(int, int) const { return 0.0f; }
    __device__ __forceinline__ float begin_plane(int) const { return 0.0f; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool, float, bool live) const {
#pragma clang fp contract(off)
        float st, ct;
        sincosf(pt.p(0), &st, &ct);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx = d1_term(dx, c.w1[0][k], pt.qx(f, k), pt.qx(f, -k));
                dz = d1_term(dz, c.w1[2][k], pt.qz(f, k), pt.qz(f, -k));
            }
            if (live) pt.store(f == 0 ? gp : gr, dot3(st, dx, 0.0f, 0.0f, ct, dz));
        }
    }
};

// stage 2: stencil fields gp, gr, p; pointwise p(t-1), r(t), r(t-1), m, eps,
// delta, theta -> p, r at t + 1
struct TtiS2Op2D {
    static constexpr bool kBufferAccess = true;
    static constexpr bool kFlatY = true;
    Coefs c;
    const float *ex, *ez;  // damping per axis (x, z), already times dt / 2
    float dt2;
    FusedSrc src;
    float *p_next, *r_next;
    float *save_p, *save_r;
    __device__ __forceinline__ bool begin_tile(int, int, int, int, int, int) const { return false; }
    __device__ __forceinline__ float begin_column(int x, int) const { return ((const gfloat *)ex)[x]; }
    __device__ __forceinline__ float begin_plane(int z) const { return ((const gfloat *)ez)[z]; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool, float a, bool live) const {
#pragma clang fp contract(off)
        float st, ct;
        sincosf(pt.p(6), &st, &ct);
        float h[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx = d1_term(dx, c.w1[0][k], pt.qx(f, k), pt.qx(f, -k));
                dz = d1_term(dz, c.w1[2][k], pt.qz(f, k), pt.qz(f, -k));
            }
            h[f] = dot3(st, dx, 0.0f, 0.0f, ct, dz);
        }
        const float pc = pt.qz(2, 0);
        float lap = 0.0f;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lap = lap_term(lap, c.w2[0][k], pt.qx(2, k), pt.qx(2, -k), pc);
            lap = lap_term(lap, c.w2[2][k], pt.qz(2, k), pt.qz(2, -k), pc);
        }
        float pn, rn;
        tti_update(pc, pt.p(0), pt.p(1), pt.p(2), lap - h[0], h[1], pt.p(3), pt.p(4), pt.p(5), dt2, a, pn, rn);
        if (src.n) {  // the same injected sum into p and r
            const float inj = fused_inject(src, src.q, 2, pt.x, 0, pt.z, fast_rcp(pt.p(3)), 0.0f);
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

// z-chunk: as the isotropic 2D step (the longest of 64, 32, ... planes giving
// 2048 workgroups, at least 4)
static int tti2d_zchunk(const Geom &g) { return adaptive_zchunk((g.nx + 63) / 64, g.nz, 64, 2048, 2048); }

template <int R>
static hipError_t launch_tti2d_r(const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
    const int zc = tti2d_zchunk(a.g);
    TtiS1Op2D o1;
    o1.c = a.c;
    o1.gp = a.gp;
    o1.gr = a.gr;
    StreamFields<2, 1> F1;
    F1.q[0] = a.p_cur;
    F1.q[1] = a.r_cur;
    F1.p[0] = a.theta;
    hipError_t e = launch_stream3d_ring<R, 1, 2, 1>(o1, F1, a.g, zc, s, ev.start, nullptr, nullptr);
    if (e != hipSuccess) return e;
    TtiS2Op2D o2;
    o2.c = a.c;
    o2.ex = a.eta_x;
    o2.ez = a.eta_z;
    o2.dt2 = a.dt2;
    o2.src = a.src;
    o2.p_next = a.p_next;
    o2.r_next = a.r_next;
    o2.save_p = a.save_p;
    o2.save_r = a.save_r;
    StreamFields<3, 7> F2;
    F2.q[0] = a.gp;
    F2.q[1] = a.gr;
    F2.q[2] = a.p_cur;
    const float *pw[7] = {a.p_prev, a.r_cur, a.r_prev, a.m, a.eps, a.delta, a.theta};
    for (int i = 0; i < 7; ++i) F2.p[i] = pw[i];
    return launch_stream3d_ring<R, 1, 1, 1>(o2, F2, a.g, zc, s, nullptr, ev.stop, nullptr);
}

hipError_t launch_tti2d_stream(int R, const TtiArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define TTI_S2(r) launch_tti2d_r<r>(a, s, ev)
    FDW_DISPATCH_R(R, TTI_S2)
#undef TTI_S2
}

int tti2d_stream_zchunk(const Geom &g) { return tti2d_zchunk(g); }

}  // namespace fdw
