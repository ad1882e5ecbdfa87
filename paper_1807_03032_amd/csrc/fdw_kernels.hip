// HIP kernels (gfx950) for the finite-difference wave-equation operators of
// arXiv 1807.03032: isotropic acoustic and TTI pseudo-acoustic leapfrog steps
// with a damping layer (Section 7.2), sparse source injection and receiver
// interpolation (Section 3.3).
//
// Every kernel reads and writes fields in the padded x-fastest layout of
// fdw.h; halos hold zeros (Dirichlet) and are never written.
#include "fdw_internal.h"

namespace fdw {

// ---------------------------------------------------------------------------
// Shared device helpers
// ---------------------------------------------------------------------------

// 1/m with the hardware reciprocal (1 ulp); m = 1/v^2 is a normal float.
__device__ __forceinline__ float fast_rcp(float m) { return __builtin_amdgcn_rcpf(m); }

// Leapfrog update with the damping term (centred first time derivative):
//   u+ = [2u - (1 - a) u- + c L] / (1 + a),   a = eta dt / 2,  c = dt^2 / m.
// In the undamped interior a = 0 and no division is needed.
__device__ __forceinline__ float leapfrog(float u, float u_prev, float cl, float a) {
    float num = 2.0f * u - u_prev + cl;
    if (a != 0.0f) num = (num + a * u_prev) / (1.0f + a);
    return num;
}

// Fused injection for the point (x, y, z): adds dt^2 w_c q_s / m for every
// fused source s whose interpolation cell has this point as corner c.
__device__ __forceinline__ float fused_inject(const FusedSrc &src, int ndim, int x, int y, int z,
                                              float rcp_m, float val) {
    for (int s = 0; s < src.n; ++s) {
        const unsigned dx = (unsigned)(x - src.bx[s]);
        const unsigned dy = (unsigned)(y - src.by[s]);
        const unsigned dz = (unsigned)(z - src.bz[s]);
        if (dx <= 1u && dy <= 1u && dz <= 1u) {
            const int c = ndim == 3 ? (int)(dx + 2u * dy + 4u * dz) : (int)(dx + 2u * dz);
            val += src.w[s][c] * src.q[s] * rcp_m;
        }
    }
    return val;
}

__device__ __forceinline__ float damp_at(const float *ex, const float *ey, const float *ez, int ndim,
                                         int x, int y, int z) {
    float a = ex[x] + ez[z];
    if (ndim == 3) a += ey[y];
    return a;
}

// ---------------------------------------------------------------------------
// Naive kernels: one thread per grid point, every neighbour loaded from
// global memory (cache-served).  Kept as the simplest correct schedule and as
// the fallback for shapes the streaming kernels do not cover.
// ---------------------------------------------------------------------------

template <int NDIM, int R>
__global__ void __launch_bounds__(256) iso_naive(IsoArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    const float *u = a.u_cur;
    const float uc = u[i];
    float lap = a.c.c0 * uc;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lap += a.c.w2[0][k] * (u[i + k] + u[i - k]);
        lap += a.c.w2[2][k] * (u[i + k * a.g.sz] + u[i - k * a.g.sz]);
        if (NDIM == 3) lap += a.c.w2[1][k] * (u[i + k * a.g.sy] + u[i - k * a.g.sy]);
    }
    const float rm = fast_rcp(a.m[i]);
    const float d = damp_at(a.eta_x, a.eta_y, a.eta_z, NDIM, x, y, z);
    float un = leapfrog(uc, a.u_prev[i], a.dt2 * rm * lap, d);
    if (a.src.n) un = fused_inject(a.src, NDIM, x, y, z, rm, un);
    a.u_next[i] = un;
}

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
    float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        dx += c.w1[0][k] * (f[i + k] - f[i - k]);
        dz += c.w1[2][k] * (f[i + k * g.sz] - f[i - k * g.sz]);
        if (NDIM == 3) dy += c.w1[1][k] * (f[i + k * g.sy] - f[i - k * g.sy]);
    }
    float r = nx * dx + nz * dz;
    if (NDIM == 3) r += ny * dy;
    return r;
}

// TTI stage 1: gp = n . grad p, gr = n . grad r on every domain point.
template <int NDIM, int R>
__global__ void __launch_bounds__(256) tti_naive_stage1(TtiArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    float nx, ny, nz;
    tti_normal<NDIM>(a, i, nx, ny, nz);
    a.gp[i] = rot_grad<NDIM, R>(a.p_cur, i, a.g, a.c, nx, ny, nz);
    a.gr[i] = rot_grad<NDIM, R>(a.r_cur, i, a.g, a.c, nx, ny, nz);
}

// TTI stage 2: H p = n . grad gp, H r = n . grad gr, L p, coupled update.
template <int NDIM, int R>
__global__ void __launch_bounds__(256) tti_naive_stage2(TtiArgs a) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = NDIM == 3 ? (int)(blockIdx.y * blockDim.y + threadIdx.y) : 0;
    const int z = NDIM == 3 ? (int)blockIdx.z : (int)(blockIdx.y * blockDim.y + threadIdx.y);
    if (x >= a.g.nx || y >= a.g.ny || z >= a.g.nz) return;
    const int64_t i = a.g.off0 + (int64_t)z * a.g.sz + (int64_t)y * a.g.sy + x;
    float nx, ny, nz;
    tti_normal<NDIM>(a, i, nx, ny, nz);
    const float hp = rot_grad<NDIM, R>(a.gp, i, a.g, a.c, nx, ny, nz);
    const float hr = rot_grad<NDIM, R>(a.gr, i, a.g, a.c, nx, ny, nz);
    const float *p = a.p_cur;
    const float pc = p[i];
    float lap = a.c.c0 * pc;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lap += a.c.w2[0][k] * (p[i + k] + p[i - k]);
        lap += a.c.w2[2][k] * (p[i + k * a.g.sz] + p[i - k * a.g.sz]);
        if (NDIM == 3) lap += a.c.w2[1][k] * (p[i + k * a.g.sy] + p[i - k * a.g.sy]);
    }
    const float A = lap - hp;
    const float B = hr;
    const float s = sqrtf(1.0f + 2.0f * a.delta[i]);
    const float rm = fast_rcp(a.m[i]);
    const float cdt = a.dt2 * rm;
    const float d = damp_at(a.eta_x, a.eta_y, a.eta_z, NDIM, x, y, z);
    float pn = leapfrog(pc, a.p_prev[i], cdt * ((1.0f + 2.0f * a.eps[i]) * A + s * B), d);
    float rn = leapfrog(a.r_cur[i], a.r_prev[i], cdt * (s * A + B), d);
    if (a.src.n) {
        pn = fused_inject(a.src, NDIM, x, y, z, rm, pn);
        rn = fused_inject(a.src, NDIM, x, y, z, rm, rn);
    }
    a.p_next[i] = pn;
    a.r_next[i] = rn;
}

// ---------------------------------------------------------------------------
// Sparse kernels.  One group of ncorner lanes per sparse point: lane c owns
// corner c; interpolation reduces the group's products with cross-lane
// shuffles; injection scatters with atomics (sources may share points).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t corner_offset(const SparseArgs &a, int c) {
    return ((c & 1) ? a.cstride[0] : 0) + ((c & 2) ? a.cstride[1] : 0) + ((c & 4) ? a.cstride[2] : 0);
}

__global__ void __launch_bounds__(256) interp_kernel(SparseArgs a) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = lane / a.ncorner;
    const int c = lane % a.ncorner;
    float v = 0.0f;
    if (p < a.npoint) v = a.w[(int64_t)p * a.ncorner + c] * a.field[a.base[p] + corner_offset(a, c)];
    // groups of 4 or 8 lanes are aligned inside the 64-wide wavefront
    v += __shfl_xor(v, 1);
    v += __shfl_xor(v, 2);
    if (a.ncorner == 8) v += __shfl_xor(v, 4);
    if (p < a.npoint && c == 0) a.rec_row[p] = v;
}

__global__ void __launch_bounds__(256) inject_kernel(SparseArgs a) {
    const int lane = blockIdx.x * blockDim.x + threadIdx.x;
    const int p = lane / a.ncorner;
    const int c = lane % a.ncorner;
    if (p >= a.npoint) return;
    const int64_t i = a.base[p] + corner_offset(a, c);
    atomicAdd(a.field + i, a.w[(int64_t)p * a.ncorner + c] * a.q_row[p] * fast_rcp(a.m[i]));
}

// Writes zero to every element of one slot outside the domain.
__global__ void __launch_bounds__(256) zero_halo_kernel(int ndim, Geom g, int R, int64_t pitch_x,
                                                        int64_t pitch_y, int64_t planes, float *base) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t total = pitch_x * pitch_y * planes;
    if (e >= total) return;
    const int64_t xx = e % pitch_x;
    const int64_t row = e / pitch_x;
    const int64_t x = xx - (g.off0 % pitch_x);
    bool inside = x >= 0 && x < g.nx;
    if (ndim == 3) {
        const int64_t y = row % pitch_y - R;
        const int64_t z = row / pitch_y - R;
        inside = inside && y >= 0 && y < g.ny && z >= 0 && z < g.nz;
    } else {
        const int64_t z = row - R;
        inside = inside && z >= 0 && z < g.nz;
    }
    if (!inside) base[e] = 0.0f;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int NDIM, int R>
static hipError_t launch_iso_naive(const IsoArgs &a, hipStream_t s) {
    if (NDIM == 3) {
        dim3 blk(64, 4, 1), grd((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz);
        hipLaunchKernelGGL((iso_naive<NDIM, R>), grd, blk, 0, s, a);
    } else {
        dim3 blk(64, 4, 1), grd((a.g.nx + 63) / 64, (a.g.nz + 3) / 4, 1);
        hipLaunchKernelGGL((iso_naive<NDIM, R>), grd, blk, 0, s, a);
    }
    return hipGetLastError();
}

template <int NDIM, int R>
static hipError_t launch_tti_naive(const TtiArgs &a, hipStream_t s) {
    dim3 blk(64, 4, 1);
    dim3 grd = NDIM == 3 ? dim3((a.g.nx + 63) / 64, (a.g.ny + 3) / 4, a.g.nz)
                         : dim3((a.g.nx + 63) / 64, (a.g.nz + 3) / 4, 1);
    hipLaunchKernelGGL((tti_naive_stage1<NDIM, R>), grd, blk, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((tti_naive_stage2<NDIM, R>), grd, blk, 0, s, a);
    return hipGetLastError();
}

#define FDW_DISPATCH_R(R_, CALL) \
    switch (R_) {                \
    case 1: return CALL(1);      \
    case 2: return CALL(2);      \
    case 3: return CALL(3);      \
    case 4: return CALL(4);      \
    case 5: return CALL(5);      \
    case 6: return CALL(6);      \
    case 7: return CALL(7);      \
    case 8: return CALL(8);      \
    default: return hipErrorInvalidValue; \
    }

hipError_t launch_iso(int ndim, int R, IsoVariant v, const IsoArgs &a, hipStream_t s) {
    (void)v;
#define ISO_N3(r) launch_iso_naive<3, r>(a, s)
#define ISO_N2(r) launch_iso_naive<2, r>(a, s)
    if (ndim == 3) { FDW_DISPATCH_R(R, ISO_N3) }
    FDW_DISPATCH_R(R, ISO_N2)
#undef ISO_N3
#undef ISO_N2
}

hipError_t launch_tti(int ndim, int R, TtiVariant v, const TtiArgs &a, hipStream_t s) {
    (void)v;
#define TTI_N3(r) launch_tti_naive<3, r>(a, s)
#define TTI_N2(r) launch_tti_naive<2, r>(a, s)
    if (ndim == 3) { FDW_DISPATCH_R(R, TTI_N3) }
    FDW_DISPATCH_R(R, TTI_N2)
#undef TTI_N3
#undef TTI_N2
}

hipError_t launch_inject(const SparseArgs &a, hipStream_t s) {
    if (a.npoint <= 0) return hipSuccess;
    const int64_t lanes = (int64_t)a.npoint * a.ncorner;
    hipLaunchKernelGGL(inject_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_interp(const SparseArgs &a, hipStream_t s) {
    if (a.npoint <= 0) return hipSuccess;
    const int64_t lanes = (int64_t)a.npoint * a.ncorner;
    hipLaunchKernelGGL(interp_kernel, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_zero_halo(int ndim, const Geom &g, int R, int64_t pitch_x, int64_t pitch_y, int64_t planes,
                            float *base, hipStream_t s) {
    const int64_t total = pitch_x * pitch_y * planes;
    hipLaunchKernelGGL(zero_halo_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, ndim, g, R,
                       pitch_x, pitch_y, planes, base);
    return hipGetLastError();
}

const char *iso_kernel_name(int ndim, IsoVariant v) {
    (void)v;
    return ndim == 3 ? "iso_naive<3>" : "iso_naive<2>";
}

const char *tti_kernel_name(int ndim, TtiVariant v) {
    (void)v;
    return ndim == 3 ? "tti_naive_stage1+2<3>" : "tti_naive_stage1+2<2>";
}

}  // namespace fdw
