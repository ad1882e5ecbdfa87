// 3D isotropic temporal blocking (gfx950): two leapfrog steps per pass over
// HBM, the paper's "time tiling" (Section 8, further work) for the isotropic
// operator of Section 7.2.
//
// A workgroup owns an output tile of (64 - 2R) x (BY NY - 2R) columns and
// walks a z-chunk on the ring-buffer engine's plan (fdw_stream2.h).  Around
// the tile it keeps an extended region E1 = tile + R in x and y: 64 x BY NY
// columns, one wavefront row per 64 columns.  Per plane i of the walk:
//   step 1: u(t+1) at plane i + R on every E1 column, from the u(t) ring
//           (z neighbours), an LDS plane of u(t) over E1 + R (x/y neighbours),
//           u(t-1) and m; out-of-domain columns and planes are zero;
//   step 2: u(t+2) at plane i on the tile, from the u(t+1) ring and an LDS
//           plane of u(t+1) over E1;
//   u(t+1) and u(t+2) at plane i are written for the tile.
// Both steps use the per-step kernels' point update (iso_point_value), so the
// two levels equal two per-step launches bit for bit.  Reads: u(t-1), u(t),
// m (the E1 halo mostly from L2); writes: u(t+1), u(t+2) -- 20 B per point per
// two steps instead of 32.  Levels are read from one buffer pair and written
// to another (a neighbour tile may still read u(t) where this tile writes).
// Receivers of the previous pass (two rows, from the input levels) are
// sampled by extra workgroups of the same launch.
#include "fdw_iso_op.h"
#include "fdw_stream2.h"

namespace fdw {

// One point of either step: z ring of the stencil level, its LDS plane, and
// the point's previous level and m.
template <int NY, int RING, int LH, int LW>
struct TBPoint {
    const float (&q)[NY][RING];
    const float (&lds)[LH][LW];
    float prev, m;
    int j, ly, lx;
    int x, y, z;
    int slot, zdir;
    __device__ __forceinline__ float qz(int, int k) const {
        const int s = slot + zdir * k;
        return q[j][(s % RING + RING) % RING];
    }
    __device__ __forceinline__ float qx(int, int k) const { return lds[ly][lx + k]; }
    __device__ __forceinline__ float qy(int, int k) const { return lds[ly + k][lx]; }
    __device__ __forceinline__ float p(int i) const { return i == 0 ? prev : m; }
};

template <int R, int NY, int BY, int PF>
__global__ void __launch_bounds__(64 * BY) iso3d_tb2(TB3DFields a, Coefs cf, const FusedSrc *__restrict__ fsrc,
                                                     const float *qs1, const float *qs2, SparseArgs rec0, SparseArgs rec1,
                                                     int zc, int ntx, int nty, int nb_stencil) {
    constexpr int NT = 64 * BY;
    const int bid = (int)blockIdx.x;
    if (bid >= nb_stencil) {  // receiver rows of the previous pass, one after the other
        const int stride = ((int)gridDim.x - nb_stencil) * NT;
        const int first = (bid - nb_stencil) * NT + (int)threadIdx.x;
        for (int p = first; p < rec0.npoint; p += stride) interp_receiver(rec0, p);
        for (int p = first; p < rec1.npoint; p += stride) interp_receiver(rec1, p);
        return;
    }
    constexpr int TX = 64 - 2 * R, TY1 = BY * NY, TY = TY1 - 2 * R;
    static_assert(TY > 0, "the tile needs rows beyond the halo");
    constexpr int LW = (64 + 2 * R + 63) / 64 * 64, LH = TY1 + 2 * R;
    constexpr int RING = ring_len(R, PF), PR = PF + 1;
    constexpr int NHY = (2 * R + BY - 1) / BY;
    constexpr int NHX = (TY1 * 2 * R + NT - 1) / NT;
    __shared__ float lds_a[2][LH][LW];  // u(t) over E1 + R
    __shared__ float lds_b[2][LH][LW];  // u(t+1) over E1 (same indexing; its border is never read)
    const Geom &g = a.g;
    const int lane = threadIdx.x & 63, wy = threadIdx.x >> 6;
    int tile = xcd_tile(bid, nb_stencil);
    const int tx = tile % ntx;
    tile /= ntx;
    const int ty = tile % nty, tz = tile / nty;
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int ex0 = x0 - R, ey0 = y0 - R;  // origin of E1
    const int x = ex0 + lane;
    const int plane_bytes = (int)(g.sz * 4);
    auto vbyte = [&](int xx, int yy) {
        return xx >= 0 && xx < g.nx && yy >= 0 && yy < g.ny ? (uint32_t)(((int64_t)yy * g.sy + xx) * 4) : kBufOut;
    };
    const __amdgpu_buffer_rsrc_t r_cur = rsrc2(a.in_cur + g.off0), r_prev = rsrc2(a.in_prev + g.off0);
    const __amdgpu_buffer_rsrc_t r_m = rsrc2(a.m + g.off0);
    const __amdgpu_buffer_rsrc_t r_o1 = rsrc2(a.out_prev + g.off0), r_o2 = rsrc2(a.out_cur + g.off0);
    const DampTables eta{a.eta_x, a.eta_y, a.eta_z};
    const int rb = wy * NY;  // first E1 row of this thread
    bool indom[NY];
    uint32_t vcol[NY], vout[NY];
    float colv[NY];
    bool tile_rows = false;  // does this wavefront hold any tile row?
#pragma unroll
    for (int c = 0; c < NY; ++c) {
        const int r = rb + c, y = ey0 + r;
        indom[c] = x >= 0 && x < g.nx && y >= 0 && y < g.ny;
        vcol[c] = vbyte(x, y);
        const bool tc = indom[c] && lane >= R && lane < 64 - R && r >= R && r < TY1 - R;
        vout[c] = tc ? vcol[c] : kBufOut;
        colv[c] = indom[c] ? eta.column(x, y) : 0.0f;
        tile_rows |= r >= R && r < TY1 - R;
    }
    // halo of the u(t) plane beyond E1: R rows above and below E1 (64 wide)
    // and R columns left and right of it (E1's rows)
    bool hy_act[NHY];
    int hy_lds[NHY];
    uint32_t hy_vb[NHY];
#pragma unroll
    for (int i = 0; i < NHY; ++i) {
        const int hr = wy + BY * i;
        const int yy = hr < R ? ey0 - R + hr : ey0 + TY1 + (hr - R);
        hy_act[i] = hr < 2 * R;
        hy_lds[i] = hr < R ? hr : R + TY1 + (hr - R);
        hy_vb[i] = hy_act[i] ? vbyte(x, yy) : kBufOut;
    }
    bool hx_act[NHX];
    int hx_lrow[NHX], hx_lcol[NHX];
    uint32_t hx_vb[NHX];
#pragma unroll
    for (int i = 0; i < NHX; ++i) {
        const int xi = threadIdx.x + NT * i;
        hx_act[i] = xi < TY1 * 2 * R;
        const int hx_r = xi / (2 * R), hx_c = xi % (2 * R);
        const int hx_x = hx_c < R ? ex0 - R + hx_c : ex0 + 64 + (hx_c - R);
        hx_lrow[i] = R + hx_r;
        hx_lcol[i] = hx_c < R ? hx_c : R + 64 + (hx_c - R);
        hx_vb[i] = hx_act[i] ? vbyte(hx_x, ey0 + hx_r) : kBufOut;
    }
    // fused sources near what each step computes (step 1 on E1 over the
    // chunk's planes extended by R, step 2 on the tile)
    const bool src1_here = fsrc && src_in_tile(*fsrc, ex0, 64, ey0, TY1, z0 - R, z1 + R);
    const bool src2_here = fsrc && src_in_tile(*fsrc, x0, TX, y0, TY, z0, z1);

    auto run = [&](auto dir_tag) __attribute__((always_inline)) {
        constexpr int DIR = decltype(dir_tag)::value;
        const int nplanes = z1 - z0;
        const int zs = DIR > 0 ? z0 : z1 - 1;
        // walk index j <-> z = zs + DIR j.  u(t) plane j (j >= -2R) and u(t+1)
        // plane j (j >= -R) live in ring slot (j + 2R) % RING; iteration i
        // (from -2R) computes step 1 at plane i + R and step 2 at plane i;
        // the pointwise values of iteration i live in slot (i + 2R) % PR
        float q1[NY][RING], q2[NY][RING];
        float pu[NY][PR], pm1[NY][PR], pm2[NY][PR];
        float hy[NHY][PR], hx[NHX][PR];
        float ez1[PR], ez2[PR];
        auto load_head = [&](int j, auto slot_tag) __attribute__((always_inline)) {
            constexpr int S = decltype(slot_tag)::value;
            const int z = zs + DIR * j;
            if (z >= 0 && z < g.nz) {
#pragma unroll
                for (int c = 0; c < NY; ++c) q1[c][S] = bload(r_cur, vcol[c], z * plane_bytes);
            } else {
#pragma unroll
                for (int c = 0; c < NY; ++c) q1[c][S] = 0.0f;
            }
        };
        auto load_iter = [&](int i, auto slot_tag) __attribute__((always_inline)) {
            constexpr int P = decltype(slot_tag)::value;
            const int za = zs + DIR * (i + R);
            if (za >= 0 && za < g.nz) {
                const int so = za * plane_bytes;
#pragma unroll
                for (int c = 0; c < NY; ++c) {
                    pu[c][P] = bload(r_prev, vcol[c], so);
                    pm1[c][P] = bload(r_m, vcol[c], so);
                }
#pragma unroll
                for (int h = 0; h < NHY; ++h) hy[h][P] = bload(r_cur, hy_vb[h], so);
#pragma unroll
                for (int h = 0; h < NHX; ++h) hx[h][P] = bload(r_cur, hx_vb[h], so);
                ez1[P] = eta.plane(za);
            }
            if (i >= 0) {
                const int zb = zs + DIR * i;
#pragma unroll
                for (int c = 0; c < NY; ++c) pm2[c][P] = bload(r_m, vout[c], zb * plane_bytes);
                ez2[P] = eta.plane(zb);
            }
        };
        static_for<2 * R + PF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
            load_head(K - 2 * R, std::integral_constant<int, K % RING>{});
        });
        static_for<PF>([&](auto kc) __attribute__((always_inline)) {
            constexpr int K = decltype(kc)::value;
            if (K - 2 * R < nplanes) load_iter(K - 2 * R, std::integral_constant<int, K % PR>{});
        });

        for (int ib = -2 * R; ib < nplanes; ib += RING) {
            static_for<RING>([&](auto sc) __attribute__((always_inline)) {
                constexpr int s = decltype(sc)::value;
                const int i = ib + s;
                if (i >= nplanes) return;
                __builtin_amdgcn_sched_barrier(0);
                constexpr int buf = s & 1;
                constexpr int cA = (s + R) % RING;  // u(t) and u(t+1) slot of plane i + R
                constexpr int cB = s % RING;        // u(t) and u(t+1) slot of plane i
                constexpr int cp = s % PR;          // pointwise slot of iteration i
                const int za = zs + DIR * (i + R), zb = zs + DIR * i;
                const bool step1 = za >= 0 && za < g.nz;
                const bool step2 = i >= 0;
                // u(t) plane i + R (E1 and its halo) and u(t+1) plane i into LDS
#pragma unroll
                for (int c = 0; c < NY; ++c) lds_a[buf][R + rb + c][R + lane] = q1[c][cA];
#pragma unroll
                for (int h = 0; h < NHY; ++h)
                    if (hy_act[h]) lds_a[buf][hy_lds[h]][R + lane] = hy[h][cp];
#pragma unroll
                for (int h = 0; h < NHX; ++h)
                    if (hx_act[h]) lds_a[buf][hx_lrow[h]][hx_lcol[h]] = hx[h][cp];
                if (step2) {
#pragma unroll
                    for (int c = 0; c < NY; ++c) lds_b[buf][R + rb + c][R + lane] = q2[c][cB];
                }
                // loads of later planes: u(t) plane i + 2R + PF into the slot plane
                // i - 1 left; pointwise and halo values of iteration i + PF
                if (i + PF < nplanes) {
                    load_head(i + 2 * R + PF, std::integral_constant<int, (s + 2 * R + PF) % RING>{});
                    load_iter(i + PF, std::integral_constant<int, (s + PF) % PR>{});
                }
                lds_barrier();
                // step 1: u(t+1) at plane i + R on E1 (zero outside the domain)
                if (step1) {
#pragma unroll
                    for (int c = 0; c < NY; ++c) {
                        TBPoint<NY, RING, LH, LW> pt{q1, lds_a[buf], pu[c][cp], pm1[c][cp], c, R + rb + c, R + lane,
                                                    x, ey0 + rb + c, za, cA, DIR};
                        const float v =
                            iso_point_value<R>(pt, cf, a.dt2, fsrc, qs1, src1_here, colv[c] + ez1[cp], 0);
                        q2[c][cA] = indom[c] ? v : 0.0f;
                    }
                } else {
#pragma unroll
                    for (int c = 0; c < NY; ++c) q2[c][cA] = 0.0f;
                }
                // step 2: u(t+2) at plane i on the tile; levels t+1, t+2 stored
                if (step2 && tile_rows) {
                    const int so = zb * plane_bytes;
#pragma unroll
                    for (int c = 0; c < NY; ++c) {
                        TBPoint<NY, RING, LH, LW> pt{q2, lds_b[buf], q1[c][cB], pm2[c][cp], c, R + rb + c, R + lane,
                                                    x, ey0 + rb + c, zb, cB, DIR};
                        const float v =
                            iso_point_value<R>(pt, cf, a.dt2, fsrc, qs2, src2_here, colv[c] + ez2[cp], 0);
                        bstore(r_o1, vout[c], so, q2[c][cB]);
                        bstore(r_o2, vout[c], so, v);
                    }
                }
            });
        }
    };
    if (tz & 1)
        run(std::integral_constant<int, -1>{});
    else
        run(std::integral_constant<int, 1>{});
}

// Tile shape of the 3D temporal blocking: NY E1 rows per thread, BY
// wavefronts (output tile (64 - 2R) x (BY NY - 2R)), PF planes of loads in
// flight.
constexpr int kTB3NY = 2, kTB3BY = 16;
constexpr int tb3d_prefetch(int R) { return R <= 4 ? 2 : 1; }

TB3DShape tb3d_shape(int R) { return TB3DShape{64 - 2 * R, kTB3BY * kTB3NY - 2 * R}; }

// z-chunk: the longest chunk (up to 128 planes) that still gives 2 workgroups
// per CU, at least 32 planes (each chunk re-reads 4R planes of u(t) and
// recomputes 2R planes of step 1)
static int tb3d_zchunk(const Geom &g, int R) {
    const TB3DShape sh = tb3d_shape(R);
    const int64_t cols = (int64_t)((g.nx + sh.tx - 1) / sh.tx) * ((g.ny + sh.ty - 1) / sh.ty);
    auto wgs = [&](int zc) { return cols * (int64_t)((g.nz + zc - 1) / zc); };
    for (int zc = 128; zc >= 32; zc /= 2)
        if (wgs(zc) >= 512) return std::min(zc, g.nz);
    return std::min(32, g.nz);
}

template <int R>
static hipError_t launch_iso3d_tb2_r(const TB3DArgs &a, hipStream_t s, const LaunchEvents &ev) {
    constexpr int NY = kTB3NY, BY = kTB3BY, PF = tb3d_prefetch(R);
    const TB3DShape sh = tb3d_shape(R);
    const Geom &g = a.f.g;
    const int zc = tb3d_zchunk(g, R);
    const int ntx = (g.nx + sh.tx - 1) / sh.tx, nty = (g.ny + sh.ty - 1) / sh.ty, ntz = (g.nz + zc - 1) / zc;
    const int64_t nb = (int64_t)ntx * nty * ntz;
    const int64_t nrec = std::max<int64_t>(a.rec[0].npoint, a.rec[1].npoint);
    const int64_t ni = nrec > 0 ? std::min<int64_t>((nrec + 64 * BY - 1) / (64 * BY), interp_workgroups()) : 0;
    hipExtLaunchKernelGGL((iso3d_tb2<R, NY, BY, PF>), dim3((unsigned)(nb + ni)), dim3(64 * BY), 0, s, ev.start,
                          ev.stop, 0, a.f, a.c, a.fsrc, a.q1, a.q2, a.rec[0], a.rec[1], zc, ntx, nty, (int)nb);
    return hipGetLastError();
}

hipError_t launch_iso3d_tb2(int R, const TB3DArgs &a, hipStream_t s, const LaunchEvents &ev) {
#define TB3(r) launch_iso3d_tb2_r<r>(a, s, ev)
    FDW_DISPATCH_R(R, TB3)
#undef TB3
}

const char *tb3d_kernel_name(const Geom &g, int R) {
    static thread_local char buf[128];
    const TB3DShape sh = tb3d_shape(R);
    std::snprintf(buf, sizeof(buf), "iso3d_tb2 (temporal blocking, 2 steps per launch) tile=%dx%d (%d waves) zchunk=%d",
                  sh.tx, sh.ty, kTB3BY, tb3d_zchunk(g, R));
    return buf;
}

}  // namespace fdw
