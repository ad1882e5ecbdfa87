// HIP kernels (gfx950) for the finite-difference wave-equation operators of
// arXiv 1807.03032: isotropic acoustic and TTI pseudo-acoustic leapfrog steps
// with a damping layer (Section 7.2), sparse source injection and receiver
// interpolation (Section 3.3).
//
// Every kernel reads and writes fields in the padded x-fastest layout of
// fdw.h; halos hold zeros (Dirichlet) and are never written.
#include "fdw_internal.h"

#include <cstdio>
#include <cstdlib>

namespace fdw {

// ---------------------------------------------------------------------------
// Shared device helpers
// ---------------------------------------------------------------------------

// 1/m with the hardware reciprocal (1 ulp); m = 1/v^2 is a normal float.
__device__ __forceinline__ float fast_rcp(float m) { return __builtin_amdgcn_rcpf(m); }

// Leapfrog update with the damping term (centred first time derivative):
//   u+ = [2u - (1 - a) u- + c L] / (1 + a),   a = eta dt / 2,  c = dt^2 / m.
// In the undamped interior a = 0 and no division is needed.
// Written as u + increment, with d = u - u-:
//   u+ = u + [(1 - a) d + c L] / (1 + a),
// which rounds once at the scale of u instead of twice.
__device__ __forceinline__ float leapfrog(float u, float u_prev, float cl, float a) {
    const float d = u - u_prev;
    if (a == 0.0f) return u + (d + cl);
    return u + ((1.0f - a) * d + cl) / (1.0f + a);
}

// Laplacian at element i as sum over axes and k of w_k ((u(+k) + u(-k)) - 2u).
// Summing differences instead of a separate centre weight keeps L exactly
// zero on constants after the weights are rounded to float.
template <int NDIM, int R>
__device__ __forceinline__ float laplacian_at(const float *u, int64_t i, const Geom &g, const Coefs &c) {
    const float u2 = 2.0f * u[i];
    float lap = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lap += c.w2[0][k] * ((u[i + k] + u[i - k]) - u2);
        lap += c.w2[2][k] * ((u[i + k * g.sz] + u[i - k * g.sz]) - u2);
        if (NDIM == 3) lap += c.w2[1][k] * ((u[i + k * g.sy] + u[i - k * g.sy]) - u2);
    }
    return lap;
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
    const float lap = laplacian_at<NDIM, R>(u, i, a.g, a.c);
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
    const float pc = a.p_cur[i];
    const float lap = laplacian_at<NDIM, R>(a.p_cur, i, a.g, a.c);
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
// 3D isotropic z-streaming kernel (2.5D blocking).
//
// A workgroup of 4 wavefronts owns a 64 x TY tile of (x, y) columns
// (TY = 4 * NY: each thread owns NY consecutive y columns at one x) and marches
// along z over a chunk [z0, z0 + zc).  For every plane:
//   * the u(t) values of the z-stencil live in a per-thread register queue of
//     2R + 1 planes, so each u(t) element of the tile is loaded from memory
//     once per chunk (plus 2R warm-up planes);
//   * the x/y neighbours come from an LDS copy of the plane with an R-wide
//     x and y halo (no corners), double buffered so one barrier per plane
//     suffices;
//   * loads for plane z + 1 (queue head, u(t-1), m, halo) are issued before
//     the plane-z arithmetic so their latency overlaps it.
// Points outside the domain are never read: the zero Dirichlet halo is
// written into LDS / the queue directly.  Workgroup ids are remapped so that
// the workgroups one XCD receives (ids congruent mod 8) form a contiguous
// block of tiles and share halo rows and warm-up planes in that XCD's L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int q = nb / 8, r = nb % 8, k = bid % 8;
    return k * q + (k < r ? k : r) + bid / 8;
}

// Loads of one plane that a thread issues ahead of use (prefetch ring entry).
template <int NY, int NHY, int NHX>
struct IsoPlaneLoads {
    float head[NY];  // u(t) at z + R (queue head)
    float prev[NY];  // u(t-1) at z
    float m[NY];     // m at z
    float hy[NHY];   // y-halo rows of u(t) at z
    float hx[NHX];   // x-halo elements of u(t) at z
};

template <int R, int NY, int PF>
__global__ void __launch_bounds__(256) iso3d_stream(IsoArgs a, int zc, int ntx, int nty) {
    constexpr int TX = 64, BY = 4, TY = BY * NY, LW = TX + 2 * R, LH = TY + 2 * R, Q = 2 * R + 1;
    constexpr int NHY = (2 * R + BY - 1) / BY;     // y-halo rows per wavefront
    constexpr int NHX = (TY * 2 * R + 255) / 256;  // x-halo elements per thread
    __shared__ float lds[2][LH][LW];
    const Geom &g = a.g;
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % ntx;
    tile /= ntx;
    const int ty = tile % nty;
    const int tz = tile / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int x = x0 + lane;
    const bool xin = x < g.nx;
    const float *__restrict__ u = a.u_cur;
    const float *__restrict__ up = a.u_prev;
    const float *__restrict__ mm = a.m;
    float *__restrict__ un = a.u_next;
    // 32-bit element offsets (a slot holds fewer than 2^31 elements)
    const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;

    const int yb = y0 + wy * NY;  // first y column of this thread
    bool in[NY];
    float ay[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        in[j] = xin && yb + j < g.ny;
        ay[j] = in[j] ? a.eta_y[yb + j] : 0.0f;
    }
    const uint32_t col0 = (uint32_t)(g.off0 + (int64_t)yb * g.sy + x);
    const float ax = xin ? a.eta_x[x] : 0.0f;

    // y-halo rows handled by this wavefront: hr = wy + BY * i
    bool hy_in[NHY];
    int hy_lds[NHY];
    uint32_t hy_col[NHY];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int hr = wy + BY * i;
        const int yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
        hy_lds[i] = hr < R ? hr : R + TY + (hr - R);
        hy_in[i] = hr < 2 * R && xin && yy >= 0 && yy < g.ny;
        hy_col[i] = hy_in[i] ? (uint32_t)(g.off0 + (int64_t)yy * g.sy + x) : 0u;
    }
    // x-halo elements handled by this thread (TY rows x 2R columns)
    bool hx_act[NHX], hx_in[NHX];
    int hx_lrow[NHX], hx_lcol[NHX];
    uint32_t hx_off[NHX];
#pragma unroll
    for (int i = 0; i < NHX; ++i) {
        const int xi = threadIdx.x + 256 * i;
        hx_act[i] = xi < TY * 2 * R;
        const int hx_r = xi / (2 * R), hx_c = xi % (2 * R);
        const int hx_x = hx_c < R ? x0 - R + hx_c : x0 + TX + (hx_c - R);
        hx_in[i] = hx_act[i] && hx_x >= 0 && hx_x < g.nx && y0 + hx_r < g.ny;
        hx_lrow[i] = R + hx_r;
        hx_lcol[i] = hx_c < R ? hx_c : R + TX + (hx_c - R);
        hx_off[i] = hx_in[i] ? (uint32_t)(g.off0 + (int64_t)(y0 + hx_r) * g.sy + hx_x) : 0u;
    }

    // does a fused source touch this workgroup's tile and chunk?
    bool src_here = false;
    for (int s = 0; s < a.src.n; ++s)
        src_here |= a.src.bx[s] + 1 >= x0 && a.src.bx[s] <= x0 + TX - 1 && a.src.by[s] + 1 >= y0 &&
                    a.src.by[s] <= y0 + TY - 1 && a.src.bz[s] + 1 >= z0 && a.src.bz[s] <= z1 - 1;

    auto zin = [&](int z) { return z >= 0 && z < g.nz; };
    auto issue = [&](IsoPlaneLoads<NY, NHY, NHX> &P, int z) {
        const uint32_t zo = (uint32_t)z * sz;
        const uint32_t zh = (uint32_t)(z + R) * sz;
        const bool hin = zin(z + R);
#pragma unroll
        for (int j = 0; j < NY; ++j) {
            P.head[j] = (in[j] && hin) ? u[col0 + j * sy + zh] : 0.0f;
            P.prev[j] = in[j] ? up[col0 + j * sy + zo] : 0.0f;
            P.m[j] = in[j] ? mm[col0 + j * sy + zo] : 1.0f;
        }
#pragma unroll
        for (int i = 0; i < NHY; ++i) P.hy[i] = hy_in[i] ? u[hy_col[i] + zo] : 0.0f;
#pragma unroll
        for (int i = 0; i < NHX; ++i) P.hx[i] = hx_in[i] ? u[hx_off[i] + zo] : 0.0f;
    };

    // warm-up: queue holds u(z0 - R .. z0 + R - 1)
    float q[NY][Q];
#pragma unroll
    for (int j = 0; j < NY; ++j)
#pragma unroll
        for (int k = 0; k < 2 * R; ++k) {
            const int z = z0 - R + k;
            q[j][k] = (in[j] && zin(z)) ? u[col0 + j * sy + (uint32_t)z * sz] : 0.0f;
        }
    IsoPlaneLoads<NY, NHY, NHX> P[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s)
        if (z0 + s < z1) issue(P[s], z0 + s);

    const float two = 2.0f;
    int buf = 0;
    for (int zb = z0; zb < z1; zb += PF) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int z = zb + s;
            if (z >= z1) break;
            float cp[NY], cm[NY], chy[NHY], chx[NHX];
#pragma unroll
            for (int i = 0; i < NHX; ++i) chx[i] = P[s].hx[i];
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                q[j][2 * R] = P[s].head[j];
                cp[j] = P[s].prev[j];
                cm[j] = P[s].m[j];
            }
#pragma unroll
            for (int i = 0; i < NHY; ++i) chy[i] = P[s].hy[i];
            if (z + PF < z1) issue(P[s], z + PF);
            // plane z into LDS
#pragma unroll
            for (int j = 0; j < NY; ++j) lds[buf][R + wy * NY + j][R + lane] = q[j][R];
#pragma unroll
            for (int i = 0; i < NHY; ++i)
                if (wy + BY * i < 2 * R) lds[buf][hy_lds[i]][R + lane] = chy[i];
#pragma unroll
            for (int i = 0; i < NHX; ++i)
                if (hx_act[i]) lds[buf][hx_lrow[i]][hx_lcol[i]] = chx[i];
            __syncthreads();
            const float az = a.eta_z[z];
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                const int ly = R + wy * NY + j, lx = R + lane;
                const float uc = q[j][R];
                const float u2 = two * uc;
                // Laplacian as sum_k w_k ((u+k + u-k) - 2u): no centre weight, so
                // rounding the weights cannot add a spurious mass term
                float lap = 0.0f;
#pragma unroll
                for (int k = 1; k <= R; ++k) {
                    lap += a.c.w2[2][k] * ((q[j][R + k] + q[j][R - k]) - u2);
                    lap += a.c.w2[0][k] * ((lds[buf][ly][lx + k] + lds[buf][ly][lx - k]) - u2);
                    lap += a.c.w2[1][k] * ((lds[buf][ly + k][lx] + lds[buf][ly - k][lx]) - u2);
                }
                const float rm = fast_rcp(cm[j]);
                const float cl = a.dt2 * rm * lap;
                const float d = uc - cp[j];
                const float damp = ax + ay[j] + az;
                float v;
                if (damp == 0.0f) {
                    v = uc + (d + cl);
                } else {
                    v = uc + ((1.0f - damp) * d + cl) / (1.0f + damp);
                }
                if (src_here) v = fused_inject(a.src, 3, x, yb + j, z, rm, v);
                if (in[j]) un[col0 + j * sy + (uint32_t)z * sz] = v;
            }
            // advance the queue
#pragma unroll
            for (int j = 0; j < NY; ++j)
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) q[j][k] = q[j][k + 1];
            buf ^= 1;
        }
    }
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

// Tile shape of the z-streaming kernel: NY y-columns per thread (tile 64 x 4NY),
// z-chunk length ZC and prefetch distance PF (planes in flight);
// FDW_ISO_TILE="NY,ZC[,PF]" overrides (tuning sweeps).
struct IsoShape {
    int ny, zc, pf;
};

static IsoShape iso_stream_shape(const Geom &g) {
    IsoShape sh{4, 16, 2};
    if (const char *e = std::getenv("FDW_ISO_TILE")) {
        int a = 0, b = 0, c = 2;
        const int n = std::sscanf(e, "%d,%d,%d", &a, &b, &c);
        if (n >= 2 && (a == 1 || a == 2 || a == 4 || a == 8) && b > 0 && (c == 1 || c == 2 || c == 3)) {
            sh.ny = a;
            sh.zc = b;
            sh.pf = c;
        }
    }
    if (sh.zc > g.nz) sh.zc = g.nz;
    return sh;
}

template <int R, int NY, int PF>
static hipError_t launch_iso3d_stream_cfg(const IsoArgs &a, int zc, hipStream_t s) {
    const int ntx = (a.g.nx + 63) / 64, nty = (a.g.ny + 4 * NY - 1) / (4 * NY), ntz = (a.g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    hipLaunchKernelGGL((iso3d_stream<R, NY, PF>), dim3((unsigned)nb), dim3(256), 0, s, a, zc, ntx, nty);
    return hipGetLastError();
}

template <int R, int NY>
static hipError_t launch_iso3d_stream_ny(const IsoArgs &a, const IsoShape &sh, hipStream_t s) {
    if (sh.pf == 1) return launch_iso3d_stream_cfg<R, NY, 1>(a, sh.zc, s);
    if (sh.pf == 3) return launch_iso3d_stream_cfg<R, NY, 3>(a, sh.zc, s);
    return launch_iso3d_stream_cfg<R, NY, 2>(a, sh.zc, s);
}

template <int R>
static hipError_t launch_iso3d_stream(const IsoArgs &a, hipStream_t s) {
    const IsoShape sh = iso_stream_shape(a.g);
    if (sh.ny == 1) return launch_iso3d_stream_ny<R, 1>(a, sh, s);
    if (sh.ny == 2) return launch_iso3d_stream_ny<R, 2>(a, sh, s);
    if (sh.ny == 8) return launch_iso3d_stream_ny<R, 8>(a, sh, s);
    return launch_iso3d_stream_ny<R, 4>(a, sh, s);
}

hipError_t launch_iso(int ndim, int R, IsoVariant v, const IsoArgs &a, hipStream_t s) {
#define ISO_S3(r) launch_iso3d_stream<r>(a, s)
    if (ndim == 3 && v == IsoVariant::Stream) { FDW_DISPATCH_R(R, ISO_S3) }
#undef ISO_S3
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
    if (ndim == 3 && v == IsoVariant::Stream) {
        static char buf[96];
        Geom g{};
        g.nz = 1 << 30;
        const IsoShape sh = iso_stream_shape(g);
        std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x%d zchunk=%d prefetch=%d", 4 * sh.ny, sh.zc, sh.pf);
        return buf;
    }
    return ndim == 3 ? "iso_naive<3>" : "iso_naive<2>";
}

const char *tti_kernel_name(int ndim, TtiVariant v) {
    (void)v;
    return ndim == 3 ? "tti_naive_stage1+2<3>" : "tti_naive_stage1+2<2>";
}

}  // namespace fdw
