// Isotropic acoustic step at one point (gfx950 device code): the update
// every 3D isotropic kernel applies, and the operator functor of the
// z-streaming engines.
// Paper: arXiv 1807.03032, eq. WE and Listings fd-2/fd-3 (update), Listing
// finject (injection), Section 7.2 (damping layer).
#pragma once
#include "fdw_device.h"

namespace fdw {

// ---- isotropic step: stencil field u(t); pointwise u(t-1), m ----------------
// New level at one point from a StreamPoint-like view (qz/qx/qy of field 0 =
// u(t), p(0) = u(t-1), p(1) = m, grid coordinates x, y, z); a = damping
// factor eta dt / 2 at the point; q = this step's source samples.  Shared by every 3D isotropic kernel, so the
// per-step kernels and the temporal-blocking kernel give the same bits.
template <int R, class P>
__device__ __forceinline__ float iso_point_value(const P &pt, const Coefs &c, float dt2, const FusedSrc *src,
                                                 const float *q, bool src_here, float a, int adjoint) {
#pragma clang fp contract(off)
    const float uc = pt.qz(0, 0);
    // Laplacian as sum_k w_k ((u+k + u-k) - 2u): no centre weight, so
    // rounding the weights cannot add a spurious mass term
    float lap = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lap = lap_term(lap, c.w2[2][k], pt.qz(0, k), pt.qz(0, -k), uc);
        lap = lap_term(lap, c.w2[0][k], pt.qx(0, k), pt.qx(0, -k), uc);
        lap = lap_term(lap, c.w2[1][k], pt.qy(0, k), pt.qy(0, -k), uc);
    }
    const float rm = fast_rcp(pt.p(1));
    float v = leapfrog(uc, pt.p(0), dt2 * rm * lap, a);
    if (src_here) v = fused_inject(*src, q, 3, pt.x, pt.y, pt.z, rm, v, adjoint ? 1.0f / (1.0f + a) : 1.0f);
    return v;
}

struct IsoOp {
    static constexpr bool kBufferAccess = false;  // raw buffer (true) or global accesses
    Coefs c;
    DampTables eta;
    float dt2;
    FusedSrc src;
    float *u_next;
    float *save;   // optional second destination of the new level
    float *isave;  // optional: the step's imaging factor (from u(t+1), u(t), u(t-1), a)
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
        const float v = iso_point_value<R>(pt, c, dt2, &src, src.q, src_here, a, adjoint);
        if (live) {
            pt.store(u_next, v);
            if (save) pt.store(save, v);
            if (isave) pt.store(isave, imaging_factor(v, pt.qz(0, 0), pt.p(0), a));
        }
    }
};

// ---- adjoint step with the imaging condition of the previous step ----------
// Pointwise fields u(t-1), m as above, then the imaging factor S of the
// forward step paired with the centre level and the gradient: the centre
// level nu (final: the previous launch's injections included) images
// grad -= nu S / dt^2 at each point, beside the step itself.
struct IsoImgOp : IsoOp {
    float *grad;
    float inv_dt2;
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool src_here, float a, bool live) const {
        const float v = iso_point_value<R>(pt, c, dt2, &src, src.q, src_here, a, adjoint);
        if (live) {
            pt.store(u_next, v);
            if (save) pt.store(save, v);
            pt.store(grad, image_update(pt.p(3), pt.qz(0, 0), pt.p(2), inv_dt2));
        }
    }
};

}  // namespace fdw
