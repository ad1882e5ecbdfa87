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
// 3D z-streaming engine (2.5D blocking), shared by the isotropic step and the
// two TTI stages.
//
// A workgroup of BY wavefronts owns a 64 x TY tile of (x, y) columns
// (TY = BY * NY: each thread owns NY consecutive y columns at one x) and marches
// along z over a chunk [z0, z0 + zc).  Two kinds of input fields:
//   * NQ "stencil" fields, read at z - R .. z + R: each thread keeps a
//     register queue of 2R + 1 planes per column (z neighbours), and the
//     workgroup keeps the current plane with an R-wide x/y halo (no corners) in
//     LDS (x/y neighbours), double buffered so one barrier per plane suffices;
//   * NP "pointwise" fields, read only at the output point.
// Loads for plane z + PF (queue heads, pointwise values, halo) are issued
// before the plane-z arithmetic, so PF planes of loads are in flight.
// Points outside the domain are never read: the zero Dirichlet halo is written
// into LDS / the queues directly.  Workgroup ids are remapped so that the
// workgroups one XCD receives (ids congruent mod 8) cover a contiguous block of
// tiles and share halo rows and warm-up planes in that XCD's L2.
// The operator functor Op computes and stores the outputs of one point from
// a StreamPoint view of the registers and LDS.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_tile(int bid, int nb) {
    const int q = nb / 8, r = nb % 8, k = bid % 8;
    return k * q + (k < r ? k : r) + bid / 8;
}

template <int NQ, int NP>
struct StreamFields {
    const float *q[NQ];  // stencil fields
    const float *p[NP];  // pointwise fields
    float pout[NP];      // value used outside the domain
};

// Loads of one plane that a thread issues ahead of use (prefetch ring entry).
template <int NQ, int NP, int NY, int NHY, int NHX>
struct PlaneLoads {
    float head[NQ][NY];  // stencil fields at z + R (queue heads)
    float pw[NP][NY];    // pointwise fields at z
    float hy[NQ][NHY];   // y-halo rows at z
    float hx[NQ][NHX];   // x-halo elements at z
};

// What an operator sees for one output point.
template <int R, int NQ, int NP, int NY, int LH, int LW>
struct StreamPoint {
    const float (&q)[NQ][NY][2 * R + 1];
    const float (&lds)[NQ][LH][LW];
    const float (&pw)[NP][NY];
    int j, ly, lx;        // column index in the thread, LDS coordinates
    int x, y, z;          // grid coordinates
    uint32_t off;         // element offset of the point
    // field f at (x, y, z + k), (x + k, y, z), (x, y + k, z); k in [-R, R]
    __device__ __forceinline__ float qz(int f, int k) const { return q[f][j][R + k]; }
    __device__ __forceinline__ float qx(int f, int k) const { return lds[f][ly][lx + k]; }
    __device__ __forceinline__ float qy(int f, int k) const { return lds[f][ly + k][lx]; }
    __device__ __forceinline__ float p(int i) const { return pw[i][j]; }
};

template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__global__ void __launch_bounds__(64 * BY) stream3d(Op op, StreamFields<NQ, NP> F, Geom g, int zc, int ntx, int nty) {
    constexpr int NT = 64 * BY;  // threads per workgroup
    constexpr int TX = 64, TY = BY * NY, LW = TX + 2 * R, LH = TY + 2 * R, Q = 2 * R + 1;
    constexpr int NHY = (2 * R + BY - 1) / BY;       // y-halo rows per wavefront
    constexpr int NHX = (TY * 2 * R + NT - 1) / NT;  // x-halo elements per thread
    __shared__ float lds[2][NQ][LH][LW];
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
    // 32-bit element offsets (a slot holds fewer than 2^31 elements)
    const uint32_t sy = (uint32_t)g.sy, sz = (uint32_t)g.sz;
    const int yb = y0 + wy * NY;  // first y column of this thread
    bool in[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) in[j] = xin && yb + j < g.ny;
    const uint32_t col0 = (uint32_t)(g.off0 + (int64_t)yb * g.sy + x);
    // per-column constants of the operator, computed once
    float colv[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) colv[j] = in[j] ? op.begin_column(x, yb + j) : 0.0f;

    // y-halo rows handled by this wavefront: hr = wy + BY * i
    bool hy_in[NHY], hy_act[NHY];
    int hy_lds[NHY];
    uint32_t hy_col[NHY];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int hr = wy + BY * i;
        const int yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
        hy_act[i] = hr < 2 * R;
        hy_lds[i] = hr < R ? hr : R + TY + (hr - R);
        hy_in[i] = hy_act[i] && xin && yy >= 0 && yy < g.ny;
        hy_col[i] = hy_in[i] ? (uint32_t)(g.off0 + (int64_t)yy * g.sy + x) : 0u;
    }
    // x-halo elements handled by this thread (TY rows x 2R columns)
    bool hx_act[NHX], hx_in[NHX];
    int hx_lrow[NHX], hx_lcol[NHX];
    uint32_t hx_off[NHX];
#pragma unroll
    for (int i = 0; i < NHX; ++i) {
        const int xi = threadIdx.x + NT * i;
        hx_act[i] = xi < TY * 2 * R;
        const int hx_r = xi / (2 * R), hx_c = xi % (2 * R);
        const int hx_x = hx_c < R ? x0 - R + hx_c : x0 + TX + (hx_c - R);
        hx_in[i] = hx_act[i] && hx_x >= 0 && hx_x < g.nx && y0 + hx_r < g.ny;
        hx_lrow[i] = R + hx_r;
        hx_lcol[i] = hx_c < R ? hx_c : R + TX + (hx_c - R);
        hx_off[i] = hx_in[i] ? (uint32_t)(g.off0 + (int64_t)(y0 + hx_r) * g.sy + hx_x) : 0u;
    }
    const bool tile_flag = op.begin_tile(x0, TX, y0, TY, z0, z1);

    auto zin = [&](int z) { return z >= 0 && z < g.nz; };
    auto issue = [&](PlaneLoads<NQ, NP, NY, NHY, NHX> &P, int z) {
        const uint32_t zo = (uint32_t)z * sz;
        const uint32_t zh = (uint32_t)(z + R) * sz;
        const bool hin = zin(z + R);
#pragma unroll
        for (int f = 0; f < NQ; ++f) {
#pragma unroll
            for (int j = 0; j < NY; ++j) P.head[f][j] = (in[j] && hin) ? F.q[f][col0 + j * sy + zh] : 0.0f;
#pragma unroll
            for (int i = 0; i < NHY; ++i) P.hy[f][i] = hy_in[i] ? F.q[f][hy_col[i] + zo] : 0.0f;
#pragma unroll
            for (int i = 0; i < NHX; ++i) P.hx[f][i] = hx_in[i] ? F.q[f][hx_off[i] + zo] : 0.0f;
        }
#pragma unroll
        for (int f = 0; f < NP; ++f)
#pragma unroll
            for (int j = 0; j < NY; ++j) P.pw[f][j] = in[j] ? F.p[f][col0 + j * sy + zo] : F.pout[f];
    };

    // warm-up: queues hold z0 - R .. z0 + R - 1
    float q[NQ][NY][Q];
#pragma unroll
    for (int f = 0; f < NQ; ++f)
#pragma unroll
        for (int j = 0; j < NY; ++j)
#pragma unroll
            for (int k = 0; k < 2 * R; ++k) {
                const int z = z0 - R + k;
                q[f][j][k] = (in[j] && zin(z)) ? F.q[f][col0 + j * sy + (uint32_t)z * sz] : 0.0f;
            }
    PlaneLoads<NQ, NP, NY, NHY, NHX> P[PF];
#pragma unroll
    for (int s = 0; s < PF; ++s)
        if (z0 + s < z1) issue(P[s], z0 + s);

    int buf = 0;
    for (int zb = z0; zb < z1; zb += PF) {
#pragma unroll
        for (int s = 0; s < PF; ++s) {
            const int z = zb + s;
            if (z >= z1) break;
            float cpw[NP][NY], chy[NQ][NHY], chx[NQ][NHX];
#pragma unroll
            for (int f = 0; f < NQ; ++f) {
#pragma unroll
                for (int j = 0; j < NY; ++j) q[f][j][2 * R] = P[s].head[f][j];
#pragma unroll
                for (int i = 0; i < NHY; ++i) chy[f][i] = P[s].hy[f][i];
#pragma unroll
                for (int i = 0; i < NHX; ++i) chx[f][i] = P[s].hx[f][i];
            }
#pragma unroll
            for (int f = 0; f < NP; ++f)
#pragma unroll
                for (int j = 0; j < NY; ++j) cpw[f][j] = P[s].pw[f][j];
            if (z + PF < z1) issue(P[s], z + PF);
            // plane z into LDS
#pragma unroll
            for (int f = 0; f < NQ; ++f) {
#pragma unroll
                for (int j = 0; j < NY; ++j) lds[buf][f][R + wy * NY + j][R + lane] = q[f][j][R];
#pragma unroll
                for (int i = 0; i < NHY; ++i)
                    if (hy_act[i]) lds[buf][f][hy_lds[i]][R + lane] = chy[f][i];
#pragma unroll
                for (int i = 0; i < NHX; ++i)
                    if (hx_act[i]) lds[buf][f][hx_lrow[i]][hx_lcol[i]] = chx[f][i];
            }
            __syncthreads();
            const float plane_val = op.begin_plane(z);
#pragma unroll
            for (int j = 0; j < NY; ++j) {
                StreamPoint<R, NQ, NP, NY, LH, LW> pt{q, lds[buf], cpw, j, R + wy * NY + j, R + lane,
                                                      x, yb + j, z, col0 + j * sy + (uint32_t)z * sz};
                // computed for every column (keeps the NY columns in one scheduling
                // region); only stores are predicated on the column being in the domain
                op.template point<R>(pt, tile_flag, colv[j] + plane_val, in[j]);
            }
            // advance the queues
#pragma unroll
            for (int f = 0; f < NQ; ++f)
#pragma unroll
                for (int j = 0; j < NY; ++j)
#pragma unroll
                    for (int k = 0; k < 2 * R; ++k) q[f][j][k] = q[f][j][k + 1];
            buf ^= 1;
        }
    }
}

// Does any fused source's interpolation cell touch the box
// [x0, x0 + tx) x [y0, y0 + ty) x [z0, z1)?
__device__ __forceinline__ bool src_in_tile(const FusedSrc &src, int x0, int tx, int y0, int ty, int z0, int z1) {
    bool hit = false;
    for (int s = 0; s < src.n; ++s)
        hit |= src.bx[s] + 1 >= x0 && src.bx[s] <= x0 + tx - 1 && src.by[s] + 1 >= y0 && src.by[s] <= y0 + ty - 1 &&
               src.bz[s] + 1 >= z0 && src.bz[s] <= z1 - 1;
    return hit;
}

// Damping factor a = eta dt / 2 at (x, y, z) from the per-axis tables.
struct DampTables {
    const float *ex, *ey, *ez;
    __device__ __forceinline__ float at(int x, int y, int z) const { return ex[x] + ey[y] + ez[z]; }
};

// ---- isotropic step: stencil field u(t); pointwise u(t-1), m ----------------
struct IsoOp {
    Coefs c;
    DampTables eta;
    float dt2;
    FusedSrc src;
    float *u_next;
    // does a fused source touch this tile and chunk?
    __device__ __forceinline__ bool begin_tile(int x0, int tx, int y0, int ty, int z0, int z1) const {
        return src_in_tile(src, x0, tx, y0, ty, z0, z1);
    }
    // damping: eta_x + eta_y per column, + eta_z per plane
    __device__ __forceinline__ float begin_column(int x, int y) const { return eta.ex[x] + eta.ey[y]; }
    __device__ __forceinline__ float begin_plane(int z) const { return eta.ez[z]; }
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
        if (src_here) v = fused_inject(src, 3, pt.x, pt.y, pt.z, rm, v);
        if (live) u_next[pt.off] = v;
    }
};

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
    Coefs c;
    float *gp, *gr;
    __device__ __forceinline__ bool begin_tile(int, int, int, int, int, int) const { return false; }
    __device__ __forceinline__ float begin_column(int, int) const { return 0.0f; }
    __device__ __forceinline__ float begin_plane(int) const { return 0.0f; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool, float, bool live) const {
        float nx, ny, nz;
        tti_normal3(pt.p(0), pt.p(1), nx, ny, nz);
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx += c.w1[0][k] * (pt.qx(f, k) - pt.qx(f, -k));
                dy += c.w1[1][k] * (pt.qy(f, k) - pt.qy(f, -k));
                dz += c.w1[2][k] * (pt.qz(f, k) - pt.qz(f, -k));
            }
            const float gv = nx * dx + ny * dy + nz * dz;
            if (live) (f == 0 ? gp : gr)[pt.off] = gv;
        }
    }
};

// ---- TTI stage 2: stencil fields gp, gr, p; pointwise p(t-1), r(t), r(t-1),
// m, eps, delta, theta, phi --------------------------------------------------
//   Hp = n . grad gp, Hr = n . grad gr, A = L p - Hp, B = Hr
//   p+ from (1 + 2 eps) A + sqrt(1 + 2 delta) B, r+ from sqrt(1 + 2 delta) A + B
struct TtiS2Op {
    Coefs c;
    DampTables eta;
    float dt2;
    FusedSrc src;
    float *p_next, *r_next;
    __device__ __forceinline__ bool begin_tile(int x0, int tx, int y0, int ty, int z0, int z1) const {
        return src_in_tile(src, x0, tx, y0, ty, z0, z1);
    }
    __device__ __forceinline__ float begin_column(int x, int y) const { return eta.ex[x] + eta.ey[y]; }
    __device__ __forceinline__ float begin_plane(int z) const { return eta.ez[z]; }
    template <int R, class P>
    __device__ __forceinline__ void point(const P &pt, bool src_here, float a, bool live) const {
        float nx, ny, nz;
        tti_normal3(pt.p(6), pt.p(7), nx, ny, nz);
        float h[2];
#pragma unroll
        for (int f = 0; f < 2; ++f) {
            float dx = 0.0f, dy = 0.0f, dz = 0.0f;
#pragma unroll
            for (int k = 1; k <= R; ++k) {
                dx += c.w1[0][k] * (pt.qx(f, k) - pt.qx(f, -k));
                dy += c.w1[1][k] * (pt.qy(f, k) - pt.qy(f, -k));
                dz += c.w1[2][k] * (pt.qz(f, k) - pt.qz(f, -k));
            }
            h[f] = nx * dx + ny * dy + nz * dz;
        }
        const float pc = pt.qz(2, 0);
        const float p2 = 2.0f * pc;
        float lap = 0.0f;
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            lap += c.w2[2][k] * ((pt.qz(2, k) + pt.qz(2, -k)) - p2);
            lap += c.w2[0][k] * ((pt.qx(2, k) + pt.qx(2, -k)) - p2);
            lap += c.w2[1][k] * ((pt.qy(2, k) + pt.qy(2, -k)) - p2);
        }
        const float A = lap - h[0];
        const float B = h[1];
        const float sd = __builtin_sqrtf(1.0f + 2.0f * pt.p(5));
        const float rm = fast_rcp(pt.p(3));
        const float cdt = dt2 * rm;
        float pn = leapfrog(pc, pt.p(0), cdt * ((1.0f + 2.0f * pt.p(4)) * A + sd * B), a);
        float rn = leapfrog(pt.p(1), pt.p(2), cdt * (sd * A + B), a);
        if (src_here) {
            pn = fused_inject(src, 3, pt.x, pt.y, pt.z, rm, pn);
            rn = fused_inject(src, 3, pt.x, pt.y, pt.z, rm, rn);
        }
        if (live) {
            p_next[pt.off] = pn;
            r_next[pt.off] = rn;
        }
    }
};

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

template <int R, int NY, int PF, int BY, int NQ, int NP, class Op>
static hipError_t launch_stream3d(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc, hipStream_t s) {
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + BY * NY - 1) / (BY * NY), ntz = (g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    hipLaunchKernelGGL((stream3d<R, NY, PF, NQ, NP, BY, Op>), dim3((unsigned)nb), dim3(64 * BY), 0, s, op, F, g, zc,
                       ntx, nty);
    return hipGetLastError();
}

// Tile shapes are (NY y-columns per thread, BY wavefronts per workgroup, z-chunk
// ZC, prefetch PF); tile = 64 x (NY * BY).  Environment overrides for tuning:
//   FDW_ISO_TILE="NY,ZC,PF,BY"   FDW_TTI_TILE="NY1,BY1,NY2,BY2,ZC"
struct IsoShape {
    int ny, zc, pf, by;
};

static IsoShape iso_stream_shape(const Geom &g) {
    IsoShape sh{4, 16, 1, 4};
    if (const char *e = std::getenv("FDW_ISO_TILE")) {
        int a = 0, b = 0, c = 1, d = 4;
        const int n = std::sscanf(e, "%d,%d,%d,%d", &a, &b, &c, &d);
        if (n >= 2 && (a == 1 || a == 2 || a == 4) && b > 0 && (c == 1 || c == 2) && (d == 4 || d == 8))
            sh = IsoShape{a, b, c, d};
    }
    if (sh.zc > g.nz) sh.zc = g.nz;
    return sh;
}

template <int R, int NY, int PF, int BY>
static hipError_t launch_iso3d_stream_cfg(const IsoArgs &a, int zc, hipStream_t s) {
    IsoOp op;
    op.c = a.c;
    op.eta = DampTables{a.eta_x, a.eta_y, a.eta_z};
    op.dt2 = a.dt2;
    op.src = a.src;
    op.u_next = a.u_next;
    StreamFields<1, 2> F;
    F.q[0] = a.u_cur;
    F.p[0] = a.u_prev;
    F.p[1] = a.m;
    F.pout[0] = 0.0f;
    F.pout[1] = 1.0f;
    return launch_stream3d<R, NY, PF, BY>(op, F, a.g, zc, s);
}

template <int R, int NY, int PF>
static hipError_t launch_iso3d_stream_by(const IsoArgs &a, const IsoShape &sh, hipStream_t s) {
    if (sh.by == 8) return launch_iso3d_stream_cfg<R, NY, PF, 8>(a, sh.zc, s);
    return launch_iso3d_stream_cfg<R, NY, PF, 4>(a, sh.zc, s);
}

template <int R, int NY>
static hipError_t launch_iso3d_stream_ny(const IsoArgs &a, const IsoShape &sh, hipStream_t s) {
    if (sh.pf == 2) return launch_iso3d_stream_by<R, NY, 2>(a, sh, s);
    return launch_iso3d_stream_by<R, NY, 1>(a, sh, s);
}

template <int R>
static hipError_t launch_iso3d_stream(const IsoArgs &a, hipStream_t s) {
    const IsoShape sh = iso_stream_shape(a.g);
    if (sh.ny == 1) return launch_iso3d_stream_ny<R, 1>(a, sh, s);
    if (sh.ny == 2) return launch_iso3d_stream_ny<R, 2>(a, sh, s);
    return launch_iso3d_stream_ny<R, 4>(a, sh, s);
}

struct TtiShape {
    int ny1, by1, ny2, by2, zc;
};

static TtiShape tti_stream_shape(const Geom &g) {
    TtiShape sh{2, 8, 1, 8, 32};
    if (const char *e = std::getenv("FDW_TTI_TILE")) {
        int a = 0, b = 0, c = 0, d = 0, z = 0;
        if (std::sscanf(e, "%d,%d,%d,%d,%d", &a, &b, &c, &d, &z) == 5 && (a == 1 || a == 2) && (b == 4 || b == 8) &&
            (c == 1 || c == 2) && (d == 4 || d == 8) && z > 0)
            sh = TtiShape{a, b, c, d, z};
    }
    if (sh.zc > g.nz) sh.zc = g.nz;
    return sh;
}

template <int R, int NY, int BY, class Op, int NQ, int NP>
static hipError_t launch_tti_stage(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc, hipStream_t s) {
    return launch_stream3d<R, NY, 1, BY>(op, F, g, zc, s);
}

template <int R, class Op, int NQ, int NP>
static hipError_t launch_tti_stage_shape(int ny, int by, const Op &op, const StreamFields<NQ, NP> &F, const Geom &g,
                                         int zc, hipStream_t s) {
    if (ny == 2) return by == 8 ? launch_tti_stage<R, 2, 8>(op, F, g, zc, s) : launch_tti_stage<R, 2, 4>(op, F, g, zc, s);
    return by == 8 ? launch_tti_stage<R, 1, 8>(op, F, g, zc, s) : launch_tti_stage<R, 1, 4>(op, F, g, zc, s);
}

template <int R>
static hipError_t launch_tti3d_stream(const TtiArgs &a, hipStream_t s) {
    const TtiShape sh = tti_stream_shape(a.g);
    TtiS1Op o1;
    o1.c = a.c;
    o1.gp = a.gp;
    o1.gr = a.gr;
    StreamFields<2, 2> F1;
    F1.q[0] = a.p_cur;
    F1.q[1] = a.r_cur;
    F1.p[0] = a.theta;
    F1.p[1] = a.phi;
    F1.pout[0] = F1.pout[1] = 0.0f;
    hipError_t e = launch_tti_stage_shape<R>(sh.ny1, sh.by1, o1, F1, a.g, sh.zc, s);
    if (e != hipSuccess) return e;
    TtiS2Op o2;
    o2.c = a.c;
    o2.eta = DampTables{a.eta_x, a.eta_y, a.eta_z};
    o2.dt2 = a.dt2;
    o2.src = a.src;
    o2.p_next = a.p_next;
    o2.r_next = a.r_next;
    StreamFields<3, 8> F2;
    F2.q[0] = a.gp;
    F2.q[1] = a.gr;
    F2.q[2] = a.p_cur;
    const float *pw[8] = {a.p_prev, a.r_cur, a.r_prev, a.m, a.eps, a.delta, a.theta, a.phi};
    for (int i = 0; i < 8; ++i) {
        F2.p[i] = pw[i];
        F2.pout[i] = 0.0f;
    }
    F2.pout[3] = 1.0f;  // m
    return launch_tti_stage_shape<R>(sh.ny2, sh.by2, o2, F2, a.g, sh.zc, s);
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
#define TTI_S3(r) launch_tti3d_stream<r>(a, s)
    if (ndim == 3 && v == TtiVariant::Stream) { FDW_DISPATCH_R(R, TTI_S3) }
#undef TTI_S3
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
        std::snprintf(buf, sizeof(buf), "iso3d_stream tile=64x%d (%d waves) zchunk=%d prefetch=%d", sh.by * sh.ny,
                      sh.by, sh.zc, sh.pf);
        return buf;
    }
    return ndim == 3 ? "iso_naive<3>" : "iso_naive<2>";
}

const char *tti_kernel_name(int ndim, TtiVariant v) {
    if (ndim == 3 && v == TtiVariant::Stream) {
        static char buf[96];
        Geom g{};
        g.nz = 1 << 30;
        const TtiShape sh = tti_stream_shape(g);
        std::snprintf(buf, sizeof(buf), "tti3d_stream stage1 tile=64x%d stage2 tile=64x%d zchunk=%d", sh.by1 * sh.ny1,
                      sh.by2 * sh.ny2, sh.zc);
        return buf;
    }
    return ndim == 3 ? "tti_naive_stage1+2<3>" : "tti_naive_stage1+2<2>";
}

}  // namespace fdw
