// Ring-buffer z-streaming engine for 3D stencil operators on gfx950.
//
// Same decomposition as stream3d_body (a workgroup of BY wavefronts owns a
// 64 x (BY * NY) tile of (x, y) columns and walks a z-chunk; z neighbours in
// registers, x/y neighbours through a double-buffered LDS plane; the same
// operator functors), organised to issue as few instructions per point as
// possible:
//   * every field is read through a raw buffer descriptor built once per
//     workgroup, based at its chunk (see rsrc2); a lane's 32-bit byte offset
//     within a plane is computed once, and the plane offset is a scalar
//     (soffset) -- per plane no address arithmetic and no descriptor rebuild.  A lane outside the domain carries
//     an offset past the descriptor's record count, so its loads read zero and
//     its stores are dropped by the hardware bounds check, with no branch;
//     planes outside the domain are skipped by a wave-uniform branch and read
//     as zero (the halo memory is never read);
//   * the register queue of z neighbours is a ring of 2R + 1 + PF planes
//     (PF = planes of loads in flight) and the plane loop is unrolled over the
//     whole ring, so every ring index is a compile-time constant: no register
//     shifts between planes;
//   * pointwise fields and the in-plane halo are prefetched PF planes ahead
//     into rings of PF + 1 entries (the ring length is a multiple of PF + 1);
//     pointwise fields can be read with the non-temporal hint (streaming_pw),
//     so that the cache keeps the stencil field's re-read rows and planes.
// Fields of any size whose planes fit the chunk span (buffer_planes_fit).
#pragma once
#include "fdw_device.h"

#include <utility>

namespace fdw {

// f(integral_constant<int, I>) for I = 0 .. N - 1, unrolled at compile time
template <class F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    static_for_seq(f, std::make_integer_sequence<int, N>{});
}

// Operators of 2D grids declare kFlatY: the engine then keeps no y halo (the
// tile is one row of 64 x-columns per wavefront, y = 0 only) and the operator
// reads no y neighbours.
template <class Op, class = void>
struct flat_y : std::false_type {};
template <class Op>
struct flat_y<Op, std::void_t<decltype(Op::kFlatY)>> : std::integral_constant<bool, Op::kFlatY> {};

// Ring length: 2R + 1 + PF rounded up to a multiple of PF + 1 (pointwise
// rings) and of 2 (LDS double buffer).
constexpr int ring_len(int R, int PF) {
    int n = 2 * R + 1 + PF;
    while (n % (PF + 1) != 0 || n % 2 != 0) ++n;
    return n;
}

// What an operator sees for one output point (the StreamPoint interface).
template <int R, int NQ, int NP, int NY, int LH, int LW, int RING, int PR, bool NTS = false>
struct RingPoint {
    const float (&q)[NQ][NY][RING];
    const float (&lds)[NQ][LH][LW];
    const float (&pw)[NP][NY][PR];
    int j, ly, lx;  // column index in the thread, LDS coordinates
    int x, y, z;    // grid coordinates
    int slot;       // ring slot of the point's plane (compile-time after unrolling)
    int pslot;      // pointwise ring slot
    int zdir;       // +1 / -1: walking direction
    int soff;       // byte offset of plane z from the chunk descriptors' base (uniform)
    uint32_t vb;    // byte offset of the column within a plane (out of range outside the domain)
    int64_t cbase;  // element offset of the chunk descriptors' base in the layout
    // field f at (x, y, z + k), (x + k, y, z), (x, y + k, z); k in [-R, R]
    __device__ __forceinline__ float qz(int f, int k) const {
        const int s = slot + zdir * k;
        return q[f][j][(s % RING + RING) % RING];
    }
    __device__ __forceinline__ float qx(int f, int k) const { return lds[f][ly][lx + k]; }
    __device__ __forceinline__ float qy(int f, int k) const { return lds[f][ly + k][lx]; }
    __device__ __forceinline__ float p(int i) const { return pw[i][j][pslot]; }
    // stores v at the point's element of an output field in the same layout
    __device__ __forceinline__ void store(float *f, float v) const {
        if constexpr (NTS)
            bstore_nt(rsrc2(f + cbase), vb, soff, v);
        else
            bstore(rsrc2(f + cbase), vb, soff, v);
    }
};

template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__device__ __forceinline__ void stream3d_ring_body(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g,
                                                   int zc, int ntx, int nty, const SparseArgs &sp, int nb_stencil,
                                                   int bid) {
    constexpr int NT = 64 * BY;
    if (bid >= nb_stencil) {  // receiver sampling of the previous step (see stream3d_body)
        const int stride = ((int)gridDim.x - nb_stencil) * NT;
        for (int p = (bid - nb_stencil) * NT + (int)threadIdx.x; p < sp.npoint; p += stride) interp_receiver(sp, p);
        return;
    }
    constexpr bool FLAT = flat_y<Op>::value;
    constexpr bool SPW = streaming_pw<Op>::value;
    constexpr int RY = FLAT ? 0 : R;  // y-halo rows above the tile in LDS
    constexpr int TX = 64, TY = BY * NY, LW = (TX + 2 * R + 63) / 64 * 64, LH = TY + 2 * RY;
    constexpr int RING = ring_len(R, PF), PR = PF + 1;
    constexpr int NHY = FLAT ? 0 : (2 * R + BY - 1) / BY;
    constexpr int NHYA = NHY > 0 ? NHY : 1;  // array extent
    constexpr int NHX = (TY * 2 * R + NT - 1) / NT;
    __shared__ float lds[2][NQ][LH][LW];
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    int tile = xcd_tile(bid, nb_stencil);
    const int tx = tile % ntx;
    tile /= ntx;
    const int ty = tile % nty, tz = tile / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int x = x0 + lane;
    const int plane_bytes = (int)(g.sz * 4);
    auto vbyte = [&](int xx, int yy) {
        return xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny ? (uint32_t)(((int64_t)yy * g.sy + xx) * 4) : kBufOut;
    };
    // descriptors based at plane zlo of the chunk; plane z is (z - zlo) planes further
    const int zlo = z0 - R - PF;
    const int64_t cbase = g.off0 + (int64_t)zlo * g.sz;
    __amdgpu_buffer_rsrc_t rq[NQ], rp[NP];
#pragma unroll
    for (int f = 0; f < NQ; ++f) rq[f] = rsrc2(F.q[f] + cbase);
#pragma unroll
    for (int f = 0; f < NP; ++f) rp[f] = rsrc2(F.p[f] + cbase);
    const int yb = y0 + wy * NY;
    bool in[NY];
    uint32_t vcol[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) {
        in[j] = x < g.nx && yb + j < g.ny;
        vcol[j] = vbyte(x, yb + j);
    }
    float colv[NY];
#pragma unroll
    for (int j = 0; j < NY; ++j) colv[j] = in[j] ? op.begin_column(x, yb + j) : 0.0f;
    bool hy_act[NHYA];
    int hy_lds[NHYA];
    uint32_t hy_vb[NHYA];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int hr = wy + BY * i;
        const int yy = hr < R ? y0 - R + hr : y0 + TY + (hr - R);
        hy_act[i] = hr < 2 * R;
        hy_lds[i] = hr < R ? hr : R + TY + (hr - R);
        hy_vb[i] = hy_act[i] ? vbyte(x, yy) : kBufOut;
    }
    bool hx_act[NHX];
    int hx_lrow[NHX], hx_lcol[NHX];
    uint32_t hx_vb[NHX];
#pragma unroll
    for (int i = 0; i < NHX; ++i) {
        const int xi = threadIdx.x + NT * i;
        hx_act[i] = xi < TY * 2 * R;
        const int hx_r = xi / (2 * R), hx_c = xi % (2 * R);
        const int hx_x = hx_c < R ? x0 - R + hx_c : x0 + TX + (hx_c - R);
        hx_lrow[i] = RY + hx_r;
        hx_lcol[i] = hx_c < R ? hx_c : R + TX + (hx_c - R);
        hx_vb[i] = hx_act[i] ? vbyte(hx_x, y0 + hx_r) : kBufOut;
    }
    const bool tile_flag = op.begin_tile(x0, TX, y0, TY, z0, z1);

    auto run = [&](auto dir_tag) __attribute__((always_inline)) {
        constexpr int DIR = decltype(dir_tag)::value;
        const int nplanes = z1 - z0;
        const int zs = DIR > 0 ? z0 : z1 - 1;
        // plane j of the walk (z = zs + DIR j) lives in ring slot (j + R) % RING
        float q[NQ][NY][RING];
        float pw[NP][NY][PR];
        float hy[NQ][NHYA][PR], hx[NQ][NHX][PR];
        float pv[PR];
        // stencil-field plane j into its ring slot S (zero outside the domain)
        auto load_head = [&](int j, auto slot_tag) __attribute__((always_inline)) {
            constexpr int S = decltype(slot_tag)::value;
            const int z = zs + DIR * j;
            if (z >= 0 && z < g.nz) {
                const int so = (z - zlo) * plane_bytes;
#pragma unroll
                for (int f = 0; f < NQ; ++f)
#pragma unroll
                    for (int c = 0; c < NY; ++c) q[f][c][S] = bload(rq[f], vcol[c], so);
            } else {
#pragma unroll
                for (int f = 0; f < NQ; ++f)
#pragma unroll
                    for (int c = 0; c < NY; ++c) q[f][c][S] = 0.0f;
            }
        };
        // pointwise values and in-plane halo of plane j (inside the chunk) into pointwise slot P
        auto load_plane = [&](int j, auto slot_tag) __attribute__((always_inline)) {
            constexpr int P = decltype(slot_tag)::value;
            const int z = zs + DIR * j;
            const int so = (z - zlo) * plane_bytes;
#pragma unroll
            for (int f = 0; f < NP; ++f)
#pragma unroll
                for (int c = 0; c < NY; ++c)
                    pw[f][c][P] = SPW && ((streaming_mask<Op>::value >> f) & 1u) ? bload_nt(rp[f], vcol[c], so)
                                                                                : bload(rp[f], vcol[c], so);
#pragma unroll
            for (int f = 0; f < NQ; ++f) {
#pragma unroll
                for (int i = 0; i < NHY; ++i) hy[f][i][P] = bload(rq[f], hy_vb[i], so);
#pragma unroll
                for (int i = 0; i < NHX; ++i) hx[f][i][P] = bload(rq[f], hx_vb[i], so);
            }
            pv[P] = op.begin_plane(z);
        };
        // warm-up: planes -R .. R + PF - 1 of the ring, pointwise planes 0 .. PF - 1
        static_for<2 * R + PF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
            load_head(K - R, std::integral_constant<int, K % RING>{});
        });
        static_for<PF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
            if (K < nplanes) load_plane(K, std::integral_constant<int, K % PR>{});
        });

        for (int ib = 0; ib < nplanes; ib += RING) {
            static_for<RING>([&](auto sc) __attribute__((always_inline)) {
                        constexpr int s = decltype(sc)::value;
                        const int i = ib + s;
                        if (i >= nplanes) return;
                        // planes are scheduled one at a time: moving loads or LDS reads
                        // across planes only lengthens register lifetimes
                        __builtin_amdgcn_sched_barrier(0);
                        constexpr int buf = s & 1;
                        constexpr int cs = (s + R) % RING;  // centre slot
                        constexpr int cp = s % PR;          // pointwise slot of this plane
                        const int z = zs + DIR * i;
                        // plane i into LDS
#pragma unroll
                        for (int f = 0; f < NQ; ++f)
#pragma unroll
                            for (int c = 0; c < NY; ++c) lds[buf][f][RY + wy * NY + c][R + lane] = q[f][c][cs];
#pragma unroll
                        for (int h = 0; h < NHY; ++h)
                            if (hy_act[h])
#pragma unroll
                                for (int f = 0; f < NQ; ++f) lds[buf][f][hy_lds[h]][R + lane] = hy[f][h][cp];
#pragma unroll
                        for (int h = 0; h < NHX; ++h)
                            if (hx_act[h])
#pragma unroll
                                for (int f = 0; f < NQ; ++f) lds[buf][f][hx_lrow[h]][hx_lcol[h]] = hx[f][h][cp];
                        // loads of later planes: the ring head (plane i + PF + R) into the slot
                        // plane i - R - 1 left, pointwise and halo of plane i + PF
                        if (i + PF < nplanes) {
                            load_head(i + PF + R, std::integral_constant<int, (s + PF + 2 * R) % RING>{});
                            load_plane(i + PF, std::integral_constant<int, (s + PF) % PR>{});
                        }
                        lds_barrier();
                        const float plane_val = pv[cp];
                        const int so = (z - zlo) * plane_bytes;
#pragma unroll
                        for (int c = 0; c < NY; ++c) {
                            RingPoint<R, NQ, NP, NY, LH, LW, RING, PR, streaming_st<Op>::value> pt{
                                q, lds[buf], pw, c, RY + wy * NY + c, R + lane, x, yb + c, z, cs, cp, DIR, so,
                                vcol[c], cbase};
                            op.template point<R>(pt, tile_flag, colv[c] + plane_val, true);
                        }
            });
        }
    };
    if (tz & 1)
        run(std::integral_constant<int, -1>{});
    else
        run(std::integral_constant<int, 1>{});
}

// Wavefronts per SIMD the register allocation must allow: 4 (128 VGPRs) for
// the one-stencil-field shapes of order <= 8 and the two-field shape with one
// column per thread, where it costs no spills (below 4 a chip-filling grid of
// 256-thread workgroups no longer runs in one round); no bound elsewhere.
constexpr int ring_min_waves(int R, int NQ, int NY) {
    return (NQ == 1 && R <= 4 && NY <= 2) || (NQ == 2 && NY == 1) ? 4 : 1;
}

template <int R, int NY, int PF, int NQ, int NP, int BY, class Op>
__global__ void __launch_bounds__(64 * BY, ring_min_waves(R, NQ, NY))
    stream3d_ring(Op op, StreamFields<NQ, NP> F, Geom g, int zc, int ntx, int nty, SparseArgs sp, int nb_stencil) {
    stream3d_ring_body<R, NY, PF, NQ, NP, BY>(op, F, g, zc, ntx, nty, sp, nb_stencil, (int)blockIdx.x);
}

template <int R, int NY, int PF, int BY, int NQ, int NP, class Op>
static hipError_t launch_stream3d_ring(const Op &op, const StreamFields<NQ, NP> &F, const Geom &g, int zc,
                                       hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr,
                                       const SparseArgs *sp = nullptr) {
    zc = buffer_zchunk(zc, g, R, PF);
    const int ntx = (g.nx + 63) / 64, nty = (g.ny + BY * NY - 1) / (BY * NY), ntz = (g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    SparseArgs spv{};
    int64_t ni = 0;
    if (sp && sp->npoint > 0) {
        spv = *sp;
        ni = std::min<int64_t>(((int64_t)sp->npoint + 64 * BY - 1) / (64 * BY), interp_workgroups());
    }
    hipExtLaunchKernelGGL((stream3d_ring<R, NY, PF, NQ, NP, BY, Op>), dim3((unsigned)(nb + ni)), dim3(64 * BY), 0, s,
                          e0, e1, 0, op, F, g, zc, ntx, nty, spv, (int)nb);
    return hipGetLastError();
}

}  // namespace fdw
