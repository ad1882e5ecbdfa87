// Device-side building blocks shared by the HIP kernels of the wave-equation
// operators (arXiv 1807.03032; Section 7.2 test cases, Section 3.2 sparse
// points): leapfrog update, Laplacian, fused source injection, and the 3D
// z-streaming engine that the isotropic step and both TTI stages run on.
//
// Every kernel reads and writes fields in the padded x-fastest layout of
// fdw.h; halos hold zeros (Dirichlet) and are never written.
#pragma once
#include "fdw_internal.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace fdw {

// ---------------------------------------------------------------------------
// Shared device helpers
// ---------------------------------------------------------------------------

// 1/m with the hardware reciprocal (1 ulp); m = 1/v^2 is a normal float.
__device__ __forceinline__ float fast_rcp(float m) { return __builtin_amdgcn_rcpf(m); }

// Workgroup barrier that orders LDS only: waits for this wave's LDS accesses
// (lgkmcnt), not for its global loads, so loads issued for later planes stay
// in flight across the barrier.  (__syncthreads also drains vmcnt.)
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Leapfrog update with the damping term (centred first time derivative):
//   u+ = [2u - (1 - a) u- + c L] / (1 + a),   a = eta dt / 2,  c = dt^2 / m.
// Written as u + increment, with d = u - u-:
//   u+ = u + [(1 - a) d + c L] * (1 / (1 + a)),
// which rounds once at the scale of u instead of twice.  The division is a
// hardware reciprocal (1 ulp) and a product: no branch, and in the undamped
// interior (a = 0) every step is exact, so the result there is u + (d + c L)
// bit for bit.
// The multiply-adds of the point updates are written out (fmaf) and nothing
// else is fused (contract off), so every kernel that inlines them rounds the
// same way whatever code surrounds them.
__device__ __forceinline__ float leapfrog(float u, float u_prev, float cl, float a) {
#pragma clang fp contract(off)
    const float d = u - u_prev;
    return __builtin_fmaf(__builtin_fmaf(1.0f - a, d, cl), __builtin_amdgcn_rcpf(1.0f + a), u);
}

// Coupled TTI update of p and r from A = L p - H p, B = H r (one rounding
// pattern for every TTI kernel):
//   p+ from (1 + 2 eps) A + sqrt(1 + 2 delta) B,  r+ from sqrt(1 + 2 delta) A + B
__device__ __forceinline__ void tti_update(float pc, float pp, float rc, float rp, float A, float B, float m, float eps,
                                           float delta, float dt2, float a, float &pn, float &rn) {
#pragma clang fp contract(off)
    const float sd = __builtin_sqrtf(__builtin_fmaf(2.0f, delta, 1.0f));
    const float cdt = dt2 * fast_rcp(m);
    pn = leapfrog(pc, pp, cdt * __builtin_fmaf(__builtin_fmaf(2.0f, eps, 1.0f), A, sd * B), a);
    rn = leapfrog(rc, rp, cdt * __builtin_fmaf(sd, A, B), a);
}

// One pair term of the difference-form Laplacian: acc + w ((a + b) - 2u).
__device__ __forceinline__ float lap_term(float acc, float w, float a, float b, float u) {
#pragma clang fp contract(off)
    return __builtin_fmaf(w, __builtin_fmaf(-2.0f, u, a + b), acc);
}

// One term of a centred first derivative: acc + w (a - b).
__device__ __forceinline__ float d1_term(float acc, float w, float a, float b) {
#pragma clang fp contract(off)
    return __builtin_fmaf(w, a - b, acc);
}

// n . (dx, dy, dz) with the same roundings everywhere: x first, z last, so
// that for the small tilts of the workloads the dominant z term enters the
// last multiply-add unrounded.
__device__ __forceinline__ float dot3(float nx, float dx, float ny, float dy, float nz, float dz) {
#pragma clang fp contract(off)
    return __builtin_fmaf(nz, dz, __builtin_fmaf(ny, dy, nx * dx));
}

// Zero-lag imaging condition of the gradient with respect to m (the adjoint
// state nu times the time derivatives of the forward field, Section 3.2's
// injection being the adjoint of interpolation):
//   dJ/dm -= nu(t+1) [(u+ - 2u + u-)/dt^2 + eta (u+ - u-)/(2 dt)].
// imaging_factor is the bracket times dt^2, (u+ - 2u + u-) + a (u+ - u-)
// with a = eta dt / 2, from levels t + 1, t, t - 1 of one point;
// image_update accumulates one term, g - (nu S) / dt^2.
__device__ __forceinline__ float imaging_factor(float un, float uc, float up, float a) {
#pragma clang fp contract(off)
    return ((un - uc) - (uc - up)) + a * (un - up);
}
__device__ __forceinline__ float image_update(float g, float nu, float s, float inv_dt2) {
#pragma clang fp contract(off)
    return g - (nu * s) * inv_dt2;
}

// Laplacian at element i as sum over axes and k of w_k ((u(+k) + u(-k)) - 2u).
// Summing differences instead of a separate centre weight keeps L exactly
// zero on constants after the weights are rounded to float.
template <int NDIM, int R>
__device__ __forceinline__ float laplacian_at(const float *u, int64_t i, const Geom &g, const Coefs &c) {
    const float uc = u[i];
    float lap = 0.0f;
#pragma unroll
    for (int k = 1; k <= R; ++k) {
        lap = lap_term(lap, c.w2[0][k], u[i + k], u[i - k], uc);
        lap = lap_term(lap, c.w2[2][k], u[i + k * g.sz], u[i - k * g.sz], uc);
        if (NDIM == 3) lap = lap_term(lap, c.w2[1][k], u[i + k * g.sy], u[i - k * g.sy], uc);
    }
    return lap;
}

// Fused injection for the point (x, y, z): adds dt^2 w_c q_s / m (times scale)
// for every fused source s whose interpolation cell has this point as corner c.
// (q: this step's samples; the overload below takes them from src.q)
__device__ __forceinline__ float fused_inject(const FusedSrc &src, const float *q, int ndim, int x, int y, int z,
                                              float rcp_m, float val, float scale = 1.0f) {
    // every product and sum rounded on its own: the result does not depend on
    // whether the compiler can see that scale is 1 (kernels that inline this
    // with a constant or a run-time scale give the same bits)
#pragma clang fp contract(off)
    for (int s = 0; s < src.n; ++s) {
        const unsigned dx = (unsigned)(x - src.bx[s]);
        const unsigned dy = (unsigned)(y - src.by[s]);
        const unsigned dz = (unsigned)(z - src.bz[s]);
        if (dx <= 1u && dy <= 1u && dz <= 1u) {
            const int c = ndim == 3 ? (int)(dx + 2u * dy + 4u * dz) : (int)(dx + 2u * dz);
            val += src.w[s][c] * q[s] * rcp_m * scale;
        }
    }
    return val;
}

__device__ __forceinline__ float fused_inject(const FusedSrc &src, int ndim, int x, int y, int z,
                                              float rcp_m, float val, float scale = 1.0f) {
    return fused_inject(src, src.q, ndim, x, y, z, rcp_m, val, scale);
}

__device__ __forceinline__ float damp_at(const float *ex, const float *ey, const float *ez, int ndim,
                                         int x, int y, int z) {
    float a = ex[x] + ez[z];
    if (ndim == 3) a += ey[y];
    return a;
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

// ---------------------------------------------------------------------------
// Sparse-point helpers (receiver sampling can run inside a stencil launch)
// ---------------------------------------------------------------------------
// support point c of a sparse point: digit k of c in base r is the offset
// along axis k (x first)
__device__ __forceinline__ void corner_digits(const SparseArgs &a, int c, int &j0, int &j1, int &j2) {
    if (a.r == 2) {
        j0 = c & 1;
        j1 = (c >> 1) & 1;
        j2 = (c >> 2) & 1;
    } else {
        j0 = c % a.r;
        j1 = (c / a.r) % a.r;
        j2 = c / (a.r * a.r);
    }
}

__device__ __forceinline__ int64_t corner_offset(const SparseArgs &a, int c) {
    if (a.r == 2) return ((c & 1) ? a.cstride[0] : 0) + ((c & 2) ? a.cstride[1] : 0) + ((c & 4) ? a.cstride[2] : 0);
    int j0, j1, j2;
    corner_digits(a, c, j0, j1, j2);
    return j0 * a.cstride[0] + j1 * a.cstride[1] + j2 * a.cstride[2];
}

// damping factor a = eta dt / 2 at corner c of sparse point p (adjoint modes)
__device__ __forceinline__ float corner_damp(const SparseArgs &a, int p, int c) {
    const int *b = a.idx + 3 * p;
    int j0, j1, j2;
    corner_digits(a, c, j0, j1, j2);
    if (a.ndim == 3) return a.eta_x[b[0] + j0] + a.eta_y[b[1] + j1] + a.eta_z[b[2] + j2];
    return a.eta_x[b[0] + j0] + a.eta_z[b[2] + j1];
}

// Receiver sampling with linear weights (4 or 8 support points), one thread
// per receiver p: the product of corner c, w[p][c] * u[base[p] + offset(c)]
// (times 1 + a in the adjoint mode), summed as a fixed tree,
// (c0 + c1) + (c2 + c3), plus (c4 + c5) + (c6 + c7) for 8 corners, so that
// every kernel that samples a receiver gives the same bits.
__device__ __forceinline__ void interp_receiver(const SparseArgs &a, int p) {
#pragma clang fp contract(off)
    // global address space named: the arguments may come from a record in memory
    using gf = __attribute__((address_space(1))) const float;
    using gi = __attribute__((address_space(1))) const int64_t;
    if (p >= a.npoint) return;
    const int nc = a.ncorner;
    const int64_t b = ((gi *)a.base)[p];
    gf *w = (gf *)a.w + (int64_t)p * nc;
    gf *u = (gf *)a.field;
    float v[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        if (c < nc) {
            v[c] = w[c] * u[b + corner_offset(a, c)];
            if (a.damp_mode == 2) v[c] *= 1.0f + corner_damp(a, p, c);
        }
    }
    float s = (v[0] + v[1]) + (v[2] + v[3]);
    if (nc == 8) s += (v[4] + v[5]) + (v[6] + v[7]);
    ((__attribute__((address_space(1))) float *)a.rec_row)[p] = s;
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
// A neighbour outside the domain reads as zero without touching the halo
// memory (see load_at); addresses are a wave-uniform plane offset plus a
// loop-invariant 32-bit byte offset per lane.  Workgroup ids are remapped so
// that the workgroups one XCD receives (ids congruent mod 8) cover a
// contiguous block of tiles and share halo rows and warm-up planes in that
// XCD's L2.
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
};

// Raw buffer accesses for the streaming engines.  The descriptor holds a
// wave-uniform base (scalar registers) and a record count; the per-lane
// offset is a 32-bit byte offset and the plane offset a scalar (soffset), so
// no per-lane 64-bit address arithmetic is needed and a descriptor is built
// once per workgroup.  The hardware bounds-checks every access against the
// record count: a load at or past it returns zero and a store there is
// dropped, which is how the engines read the zero Dirichlet exterior without
// branches or memory traffic -- lanes outside the domain carry the offset
// kBufOut, and a plane outside the domain is read with that offset on every
// lane.  The record count is larger than any valid offset and below kBufOut,
// so an out-of-domain offset is out of range whether or not the hardware adds
// the scalar offset before the check.  Descriptor word 3 is the gfx9-family
// raw-buffer format.
//
// Chunk-based addressing (ring engine): a workgroup walking planes [z0, z1)
// reads planes z0 - R - PF .. z1 - 1 + R + PF at most, so its descriptors are
// based at plane zlo = z0 - R - PF and plane z lies (z - zlo) * plane_bytes
// further.  The launcher keeps that span, zc + 2 (R + PF) planes, below 2 GiB
// (buffer_zchunk), which holds for fields of any size whose planes are small
// enough (buffer_planes_fit).
constexpr uint32_t kBufOut = 0x80000000u;
constexpr int kRecords2 = 0x7fffffff;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc2(const float *base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, kRecords2, 0x00020000);
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, uint32_t vb, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vb, soff, 0));
}
// The same load with the non-temporal hint: for fields read once per step,
// so that the cache keeps the lines that are read again (halo rows, warm-up
// planes of the stencil field) instead.
__device__ __forceinline__ float bload_nt(__amdgpu_buffer_rsrc_t r, uint32_t vb, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)vb, soff, 2));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, uint32_t vb, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)vb, soff, 0);
}
// the same store with the non-temporal hint
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t vb, int soff, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, (int)vb, soff, 2);
}

// Planes one chunk descriptor spans beyond the chunk itself.
constexpr int buffer_extra_planes(int R, int PF) { return 2 * (R + PF); }
// Can a buffer-addressed launch of this order run on these planes (a chunk
// of one plane within the 2 GiB span)?
inline bool buffer_planes_fit(const Geom &g, int R, int PF) {
    return (int64_t)(1 + buffer_extra_planes(R, PF)) * g.sz * 4 < ((int64_t)1 << 31);
}
// z-chunk of a buffer-addressed launch: at most zc (and nz), and short enough
// that the descriptor span stays below 2 GiB (at least 1 where the planes fit).
inline int buffer_zchunk(int zc, const Geom &g, int R, int PF) {
    if (zc > g.nz) zc = g.nz;
    const int64_t fit = (((int64_t)1 << 31) - 1) / (g.sz * 4) - buffer_extra_planes(R, PF);
    return (int)std::max<int64_t>(1, std::min<int64_t>(zc, fit));
}

// The shifting-queue engine addresses plane by plane instead: element at byte
// offset vb within plane zo (element offset of the plane's (0, 0),
// wave-uniform) of a field; vb = kBufOut or valid = false (a plane outside the
// domain) read as zero and drop stores.  BUF = true: a raw buffer descriptor
// based at the plane (rebuilt per plane from the field pointer: with up to
// fifteen fields, one descriptor per field and workgroup does not fit the
// scalar registers), no branches.  BUF = false: global accesses at the
// field's base (scalar) + a 32-bit byte offset, branching around the lanes
// and planes outside the domain; the field must be below 4 GiB.  Each
// operator picks the form that measures faster for it: the TTI stages, with
// many loads per point and VALU-bound, gain from the buffer form; the
// isotropic step, bound by HBM bandwidth, runs slightly faster with global
// accesses.  (Global accesses name the global address space: field pointers
// read from a record in memory, as in the multi-shot kernels, would otherwise
// be generic and compile to flat accesses, which also count against the LDS
// wait counter and so stall every LDS wait behind the loads in flight.)
using gfloat = __attribute__((address_space(1))) float;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_at(const float *base, bool valid) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, valid ? (int)kBufOut : 0, 0x00020000);
}
// Operators declare kStreamingPointwise to have their pointwise fields read
// with the non-temporal hint (raw buffer accesses only; the launchers pick
// such operator types by grid size).  kStreamingMask narrows the ring
// engine's hint to some of the fields; the shifting-queue engine hints all.
template <class Op, class = void>
struct streaming_pw : std::false_type {};
template <class Op>
struct streaming_pw<Op, std::void_t<decltype(Op::kStreamingPointwise)>>
    : std::integral_constant<bool, Op::kStreamingPointwise> {};
// the pointwise fields that take the hint (bit f: field f), all by default
template <class Op, class = void>
struct streaming_mask : std::integral_constant<unsigned, ~0u> {};
template <class Op>
struct streaming_mask<Op, std::void_t<decltype(Op::kStreamingMask)>>
    : std::integral_constant<unsigned, Op::kStreamingMask> {};

template <bool BUF, bool NT = false>
__device__ __forceinline__ float load_at(const float *f, int64_t zo, uint32_t vb, bool valid = true) {
    if constexpr (BUF)
        return __builtin_bit_cast(
            float, __builtin_amdgcn_raw_buffer_load_b32(buffer_at(f + zo, valid), (int)vb, 0, NT ? 2 : 0));
    else
        return valid && vb != kBufOut ? *(const gfloat *)((const char *)f + ((uint32_t)zo * 4u + vb)) : 0.0f;
}
// the stores of operators that declare kStreamingStores take the hint too
template <class Op, class = void>
struct streaming_st : std::false_type {};
template <class Op>
struct streaming_st<Op, std::void_t<decltype(Op::kStreamingStores)>>
    : std::integral_constant<bool, Op::kStreamingStores> {};

template <bool BUF, bool NT = false>
__device__ __forceinline__ void store_at(float *f, int64_t zo, uint32_t vb, float v) {
    if constexpr (BUF)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), buffer_at(f + zo, true), (int)vb, 0,
                                              NT ? 2 : 0);
    else if (vb != kBufOut)
        *(gfloat *)((char *)f + ((uint32_t)zo * 4u + vb)) = v;
}

// Loads of one plane that a thread issues ahead of use (prefetch ring entry).
template <int NQ, int NP, int NY, int NHY, int NHX>
struct PlaneLoads {
    float head[NQ][NY];  // stencil fields at z + R (queue heads)
    float pw[NP][NY];    // pointwise fields at z
    float hy[NQ][NHY];   // y-halo rows at z
    float hx[NQ][NHX];   // x-halo elements at z
    float pv;            // the operator's per-plane value at z
};

// What an operator sees for one output point.
template <int R, int NQ, int NP, int NY, int LH, int LW, int DIR, bool BUF, bool NTS = false>
struct StreamPoint {
    const float (&q)[NQ][NY][2 * R + 1];
    const float (&lds)[NQ][LH][LW];
    const float (&pw)[NP][NY];
    int j, ly, lx;        // column index in the thread, LDS coordinates
    int x, y, z;          // grid coordinates
    int64_t zb;           // element offset of (0, 0) in plane z (uniform)
    uint32_t vb;          // byte offset of the point from there (kBufOut outside the domain)
    // field f at (x, y, z + k), (x + k, y, z), (x, y + k, z); k in [-R, R]
    // (queue entry R + i holds plane z + DIR * i)
    __device__ __forceinline__ float qz(int f, int k) const { return q[f][j][R + DIR * k]; }
    __device__ __forceinline__ float qx(int f, int k) const { return lds[f][ly][lx + k]; }
    __device__ __forceinline__ float qy(int f, int k) const { return lds[f][ly + k][lx]; }
    __device__ __forceinline__ float p(int i) const { return pw[i][j]; }
    // stores v at the point's element of an output field in the same layout
    __device__ __forceinline__ void store(float *f, float v) const { store_at<BUF, NTS>(f, zb, vb, v); }
};

template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__device__ __forceinline__ void stream3d_body(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc,
                                              int ntx, int nty, int zfast, const SparseArgs &sp, int nb_stencil,
                                              int bid, bool stencil_live) {
    constexpr int NT = 64 * BY;  // threads per workgroup
    // workgroups past the stencil tiles sample the receivers of the previous
    // step from the current level, which this launch only reads
    if (bid >= nb_stencil) {
        // a few workgroups loop over the receivers, one thread per receiver
        const int stride = ((int)gridDim.x - nb_stencil) * NT;
        for (int p = (bid - nb_stencil) * NT + (int)threadIdx.x; p < sp.npoint; p += stride) interp_receiver(sp, p);
        return;
    }
    if (!stencil_live) return;
    // LDS rows are padded to a multiple of 64 floats: the offset of a y
    // neighbour is then a multiple of 256 bytes, which the paired LDS reads
    // encode as an immediate (no per-neighbour address arithmetic)
    constexpr int TX = 64, TY = BY * NY, LW = (TX + 2 * R + 63) / 64 * 64, LH = TY + 2 * R, Q = 2 * R + 1;
    constexpr bool BUF = Op::kBufferAccess;
    constexpr int NHY = (2 * R + BY - 1) / BY;       // y-halo rows per wavefront
    constexpr int NHX = (TY * 2 * R + NT - 1) / NT;  // x-halo elements per thread
    __shared__ float lds[2][NQ][LH][LW];
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    int tile = xcd_tile(bid, nb_stencil);
    int tx, ty, tz;
    if (zfast) {  // z-chunk fastest: every chunk of a column on one XCD
        const int ntz = (g.nz + zc - 1) / zc;
        tz = tile % ntz;
        tile /= ntz;
        tx = tile % ntx;
        ty = tile / ntx;
    } else {  // x fastest, then y, then z-chunk
        tx = tile % ntx;
        tile /= ntx;
        ty = tile % nty;
        tz = tile / nty;
    }
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int x = x0 + lane;
    const bool xin = x < g.nx;
    // plane z's element (0, 0) is at pbase + z * sz; (x, y) is y * sy + x
    // elements further, or out of bounds (kBufOut) outside the domain
    const int64_t pbase = g.off0;
    // stencil field f / pointwise field f at plane z, byte offset vb in the plane
    // (valid = false: a plane outside the domain, read as zero)
    auto ldq = [&](int f, int z, uint32_t vb, bool valid) -> float {
        return load_at<BUF>(F.q[f], pbase + (int64_t)z * g.sz, vb, valid);
    };
    auto ldp = [&](int f, int z, uint32_t vb) -> float {
        return load_at<BUF, streaming_pw<Op>::value>(F.p[f], pbase + (int64_t)z * g.sz, vb, true);
    };
    auto vbyte = [&](int xx, int yy) {
        return xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny ? (uint32_t)(((int64_t)yy * g.sy + xx) * 4) : kBufOut;
    };
    const int yb = y0 + wy * NY;  // first y column of this thread
    bool in[NY];
    uint32_t vcol[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        in[j] = xin && yb + j < g.ny;
        vcol[j] = vbyte(x, yb + j);
    }
    // per-column constants of the operator, computed once
    float colv[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) colv[j] = in[j] ? op.begin_column(x, yb + j) : 0.0f;

    // y-halo rows handled by this wavefront: hr = wy + BY * i
    bool hy_act[NHY];
    int hy_lds[NHY];
    uint32_t hy_vb[NHY];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int hr = wy + BY * i;
        const int yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
        hy_act[i] = hr < 2 * R;
        hy_lds[i] = hr < R ? hr : R + TY + (hr - R);
        hy_vb[i] = hy_act[i] ? vbyte(x, yy) : kBufOut;
    }
    // x-halo elements handled by this thread (TY rows x 2R columns)
    bool hx_act[NHX];
    int hx_lrow[NHX], hx_lcol[NHX];
    uint32_t hx_vb[NHX];
#pragma unroll
    for (int i = 0; i < NHX; ++i) {
        const int xi = threadIdx.x + NT * i;
        hx_act[i] = xi < TY * 2 * R;
        const int hx_r = xi / (2 * R), hx_c = xi % (2 * R);
        const int hx_x = hx_c < R ? x0 - R + hx_c : x0 + TX + (hx_c - R);
        hx_lrow[i] = R + hx_r;
        hx_lcol[i] = hx_c < R ? hx_c : R + TX + (hx_c - R);
        hx_vb[i] = hx_act[i] ? vbyte(hx_x, y0 + hx_r) : kBufOut;
    }
    const bool tile_flag = op.begin_tile(x0, TX, y0, TY, z0, z1);

    // Chunks alternate their walking direction along z (even chunk index: up,
    // odd: down), so the two chunks that share a boundary read its warm-up
    // planes at the same time -- both at their start or both at their end --
    // and the second read can be served by the cache instead of HBM.  The
    // queue entry R + i holds plane z + DIR * i.
    auto run = [&](auto dir_tag) {
        constexpr int DIR = decltype(dir_tag)::value;
        const int nplanes = z1 - z0;
        const int zs = DIR > 0 ? z0 : z1 - 1;  // first plane walked
        auto issue = [&](PlaneLoads<NQ, NP, NY, NHY, NHX> &P, int z) {
            const int zhp = z + DIR * R;
            const bool hin = zhp >= 0 && zhp < g.nz;
#pragma unroll
            for (int f = 0; f < NQ; ++f) {
#pragma unroll
                for (int j = 0; j < NY; ++j) P.head[f][j] = ldq(f, zhp, vcol[j], hin);
#pragma unroll
                for (int i = 0; i < NHY; ++i) P.hy[f][i] = ldq(f, z, hy_vb[i], true);
#pragma unroll
                for (int i = 0; i < NHX; ++i) P.hx[f][i] = ldq(f, z, hx_vb[i], true);
            }
#pragma unroll
            for (int f = 0; f < NP; ++f)
#pragma unroll
                for (int j = 0; j < NY; ++j) P.pw[f][j] = ldp(f, z, vcol[j]);
            P.pv = op.begin_plane(z);
        };

        // warm-up: queue entries 0 .. 2R-1 hold planes zs + DIR * (k - R)
        float q[NQ][NY][Q];
#pragma unroll
        for (int f = 0; f < NQ; ++f)
#pragma unroll
            for (int j = 0; j < NY; ++j)
#pragma unroll
                for (int k = 0; k < 2 * R; ++k) {
                    const int z = zs + DIR * (k - R);
                    q[f][j][k] = ldq(f, z, vcol[j], z >= 0 && z < g.nz);
                }
        PlaneLoads<NQ, NP, NY, NHY, NHX> P[PF];
#pragma unroll
        for (int s = 0; s < PF; ++s)
            if (s < nplanes) issue(P[s], zs + DIR * s);

        int buf = 0;
        for (int ib = 0; ib < nplanes; ib += PF) {
#pragma unroll
            for (int s = 0; s < PF; ++s) {
                const int i = ib + s;
                if (i >= nplanes) break;
                const int z = zs + DIR * i;
                float cpw[NP][NY], chy[NQ][NHY], chx[NQ][NHX];
                const float plane_val = P[s].pv;
#pragma unroll
                for (int f = 0; f < NQ; ++f) {
#pragma unroll
                    for (int j = 0; j < NY; ++j) q[f][j][2 * R] = P[s].head[f][j];
#pragma unroll
                    for (int h = 0; h < NHY; ++h) chy[f][h] = P[s].hy[f][h];
#pragma unroll
                    for (int h = 0; h < NHX; ++h) chx[f][h] = P[s].hx[f][h];
                }
#pragma unroll
                for (int f = 0; f < NP; ++f)
#pragma unroll
                    for (int j = 0; j < NY; ++j) cpw[f][j] = P[s].pw[f][j];
                if (i + PF < nplanes) issue(P[s], z + DIR * PF);
                // plane z into LDS (one branch per halo element for all fields)
#pragma unroll
                for (int f = 0; f < NQ; ++f)
#pragma unroll
                    for (int j = 0; j < NY; ++j) lds[buf][f][R + wy * NY + j][R + lane] = q[f][j][R];
#pragma unroll
                for (int h = 0; h < NHY; ++h)
                    if (hy_act[h])
#pragma unroll
                        for (int f = 0; f < NQ; ++f) lds[buf][f][hy_lds[h]][R + lane] = chy[f][h];
#pragma unroll
                for (int h = 0; h < NHX; ++h)
                    if (hx_act[h])
#pragma unroll
                        for (int f = 0; f < NQ; ++f) lds[buf][f][hx_lrow[h]][hx_lcol[h]] = chx[f][h];
                lds_barrier();
#pragma unroll
                for (int j = 0; j < NY; ++j) {
                    StreamPoint<R, NQ, NP, NY, LH, LW, DIR, BUF, streaming_st<Op>::value> pt{q,
                                                                    lds[buf],
                                                                    cpw,
                                                                    j,
                                                                    R + wy * NY + j,
                                                                    R + lane,
                                                                    x,
                                                                    yb + j,
                                                                    z,
                                                                    pbase + (int64_t)z * g.sz,
                                                                    vcol[j]};
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
    };
    if (tz & 1)
        run(std::integral_constant<int, -1>{});
    else
        run(std::integral_constant<int, 1>{});
}

template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__global__ void __launch_bounds__(64 * BY) stream3d(Op op, StreamFields<NQ, NP> F, Geom g, int zc, int ntx, int nty,
                                                   int zfast, SparseArgs sp, int nb_stencil) {
    stream3d_body<R, NY, PF, NQ, NP, BY>(op, F, g, zc, ntx, nty, zfast, sp, nb_stencil, (int)blockIdx.x, true);
}

// One shot's share of a fused multi-shot launch: its operator and fields for
// this step, the receiver row it samples (npoint = 0: none), and whether its
// stencil runs (a shot whose range has ended only samples its last row).
template <class Op, int NQ, int NP>
struct StreamShot {
    Op op;
    StreamFields<NQ, NP> F;
    SparseArgs rec;
    int live;
};

// Same-geometry shots in one launch: blockIdx.y selects the shot.
template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__global__ void __launch_bounds__(64 * BY) stream3d_multi(const StreamShot<Op, NQ, NP> *__restrict__ shots, Geom g,
                                                         int zc, int ntx, int nty, int zfast, int nb_stencil) {
    const StreamShot<Op, NQ, NP> &S = shots[blockIdx.y];
    // the field pointers, read once into registers (the operator and the
    // receiver arguments stay in the record)
    const StreamFields<NQ, NP> F = S.F;
    stream3d_body<R, NY, PF, NQ, NP, BY>(S.op, F, g, zc, ntx, nty, zfast, S.rec, nb_stencil, (int)blockIdx.x,
                                         S.live != 0);
}

// z-chunk length for a grid: the longest chunk (up to zc_max) that still gives
// `full` workgroups -- long chunks re-read fewer warm-up planes, which decides
// large grids -- else the longest that gives `latency` workgroups, since each
// workgroup walks its chunk plane by plane and small grids are bound by that
// serial latency; 4 at least.
static inline int adaptive_zchunk(int64_t columns, int nz, int zc_max, int64_t full, int64_t latency) {
    auto wgs = [&](int zc) { return columns * (int64_t)((nz + zc - 1) / zc); };
    if (wgs(zc_max) >= full) return std::min(zc_max, nz);
    for (int zc = zc_max / 2; zc >= 4; zc /= 2)
        if (wgs(zc) >= latency) return std::min(zc, nz);
    return std::min(4, nz);
}

// Workgroups that sample receivers inside a streaming launch (each loops over
// its share; FDW_INTERP_WG overrides the default for tuning).
static inline int64_t interp_workgroups() {
    static const int64_t n = [] {
        const char *e = std::getenv("FDW_INTERP_WG");
        const long v = e ? std::strtol(e, nullptr, 10) : 0;
        return (int64_t)(v > 0 ? v : 1024);
    }();
    return n;
}

// Fused launch of n same-geometry shots (records in device memory); max_rec
// = the most receivers of any shot's receiver row.
template <int R, int NY, int PF, int BY, int NQ, int NP, class Op>
static hipError_t launch_stream3d_multi(const StreamShot<Op, NQ, NP> *shots, int n, int64_t max_rec, const Geom &g,
                                        int zc, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (zc > g.nz) zc = g.nz;
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + BY * NY - 1) / (BY * NY), ntz = (g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    const int64_t ni = std::min<int64_t>((max_rec + 64 * BY - 1) / (64 * BY), interp_workgroups());
    hipLaunchKernelGGL((stream3d_multi<R, NY, PF, NQ, NP, BY, Op>), dim3((unsigned)(nb + ni), (unsigned)n),
                       dim3(64 * BY), 0, s, shots, g, zc, ntx, nty, 0, (int)nb);
    return hipGetLastError();
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
    // a_x + a_y of a column and a_z of a plane (global address space named:
    // the tables may be read through a record in memory)
    __device__ __forceinline__ float column(int x, int y) const {
        return ((const gfloat *)ex)[x] + ((const gfloat *)ey)[y];
    }
    __device__ __forceinline__ float plane(int z) const { return ((const gfloat *)ez)[z]; }
};

template <int R, int NY, int PF, int BY, int NQ, int NP, class Op>
static hipError_t launch_stream3d(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc, hipStream_t s,
                                  hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, const SparseArgs *sp = nullptr) {
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + BY * NY - 1) / (BY * NY), ntz = (g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    SparseArgs spv{};
    int64_t ni = 0;  // extra workgroups for receiver sampling
    if (sp && sp->npoint > 0) {
        spv = *sp;
        ni = std::min<int64_t>(((int64_t)sp->npoint + 64 * BY - 1) / (64 * BY), interp_workgroups());
    }
    // tile order: FDW_TILE_ORDER=z puts the z-chunk index fastest (tuning knob)
    const char *order = std::getenv("FDW_TILE_ORDER");
    const int zfast = (order && order[0] == 'z') ? 1 : 0;
    hipExtLaunchKernelGGL((stream3d<R, NY, PF, NQ, NP, BY, Op>), dim3((unsigned)(nb + ni)), dim3(64 * BY), 0, s, e0, e1,
                          0, op, F, g, zc, ntx, nty, zfast, spv, (int)nb);
    return hipGetLastError();
}

}  // namespace fdw
