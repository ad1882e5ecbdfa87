// Internal declarations shared by the host ABI (fdw_host.cpp) and the HIP
// kernels (fdw_*.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fdw {

constexpr int kMaxR = 8;         // space order 16
constexpr int kMaxFusedSrc = 4;  // sources injected inside the stencil kernel

// Finite-difference coefficients, computed on the host in double from the
// closed-form Taylor weights and rounded once to float.
//   w2[a][k] = W2_k / h_a^2   (second derivative along axis a, k = 0..R)
//   w1[a][k] = W1_k / h_a     (first derivative along axis a, k = 1..R)
//   c0       = sum_a W2_0 / h_a^2 (centre weight of the Laplacian)
// Axis index a: 0 = x, 1 = y, 2 = z (2D grids use 0 and 2).
struct Coefs {
    float w2[3][kMaxR + 1];
    float w1[3][kMaxR + 1];
    float c0;
};

// Up to kMaxFusedSrc point sources injected by the thread that owns each
// target point, right after it computes the point's update.
//   b[s]      base grid indices (x, y, z) of source s (y = 0 in 2D)
//   w[s][c]   dt^2 * interpolation weight of corner c (bit 0: +x, bit 1: +y
//             in 3D or +z in 2D, bit 2: +z in 3D)
//   q         device pointer to the source samples of this step (row t)
struct FusedSrc {
    int n;
    int bx[kMaxFusedSrc], by[kMaxFusedSrc], bz[kMaxFusedSrc];
    float w[kMaxFusedSrc][8];
    const float *q;
};

// Geometry of the padded layout (all fields of one operator share it).
struct Geom {
    int nx, ny, nz;    // domain points (ny = 1 in 2D)
    int64_t sy, sz;    // strides of +y and +z in elements (2D: sy = 0, sz = pitch_x)
    int64_t off0;      // element offset of logical (0, 0, 0)
};

// Does a 3D field of this geometry reach 4 GiB (beyond 32-bit byte offsets)?
inline bool iso_wide_fields(const Geom &g) { return (g.off0 + (int64_t)g.nz * g.sz) * 4 > (int64_t)UINT32_MAX; }

struct IsoArgs {
    Geom g;
    const float *u_cur, *u_prev, *m;
    float *u_next;
    const float *eta_x, *eta_y, *eta_z;  // damping per axis, already times dt/2
    float dt2;
    Coefs c;
    FusedSrc src;
    int adjoint;   // 1: injected terms are divided by the damping factor (1 + a)
    float *save;   // optional: the new level is also stored here (same layout)
    float *isave;  // optional: the step's imaging factor is stored here (3D streaming kernels)
    int sampling;  // the operator samples its receivers inside its 3D streaming launches
    // optional (3D streaming kernels): imaging condition of the centre level,
    // grad -= u_cur img_s / dt^2
    const float *img_s;
    float *grad;
    float inv_dt2;
    const struct SparseArgs *rec;  // optional: receiver sampling of the previous step
};

struct TtiArgs {
    Geom g;
    const float *p_cur, *p_prev, *r_cur, *r_prev;
    float *p_next, *r_next;
    const float *m, *eps, *delta, *theta, *phi;
    float *gp, *gr;  // stage buffers: rotated gradients n . grad p, n . grad r
    float *save_p, *save_r;  // optional: the new levels are also stored here (same layout)
    const float *eta_x, *eta_y, *eta_z;
    float dt2;
    Coefs c;
    FusedSrc src;
    const struct SparseArgs *rec;  // optional: receiver sampling of the previous step
};

struct SparseArgs {
    // adjoint mode: injection divides by (1 + a) and interpolation weights
    // each corner by (1 + a), a = eta dt / 2 from the per-axis tables
    int damp_mode;               // 0: none, 1: inject / (1 + a), 2: interp * (1 + a)
    const int *idx;              // [npoint][3] base grid indices (x, y, z); y = 0 in 2D
    const float *eta_x, *eta_y, *eta_z;
    int ndim;
    int npoint;
    int r;                       // support points per axis (2: linear weights)
    int ncorner;                 // r^ndim (4 or 8 for linear weights)
    const int64_t *base;         // [npoint] element offset of corner 0
    const float *w;              // [npoint][ncorner] weights (times scale for injection)
    int64_t cstride[3];          // offsets of +axis0, +axis1, +axis2 corners
    const float *m;              // injection: divisor field; NULL for interpolation
    float *field;                // injection target / interpolation source
    const float *q_row;          // injection: samples of this step
    float *rec_row;              // interpolation: output row of this step
    // injection by gather (many points): the distinct target elements tgt[j]
    // and, for each, its lanes (ascending p * ncorner + c) at
    // goff[j] .. goff[j + 1] - 1 of gp (sparse point) and gw (its weight);
    // gd[j] = 1 + a at the target (adjoint injection); ntarget = 0: scatter
    // with atomics
    int ntarget;
    const int64_t *tgt;
    const int *goff, *gp;
    const float *gw, *gd;
};

// One shot of a fused multi-shot launch of the one-thread-per-point kernels.
template <class A>
struct NaiveShot {
    A a;
    int live;
};

// ---- fused multi-shot steps (same geometry, space order and kind) ----------
// The host packs one record per shot and step (multi_pack_*), the caller
// uploads the records, and one launch per stage runs every shot.  3D steps
// sample the receiver row `rec` inside the stencil launch; 2D steps sample it
// with launch_interp_multi after the step.  live = 0: the shot's stencil is
// skipped (its receiver row, if any, is still sampled).
// logical (x fastest) device array -> domain of a padded slot of geometry g
hipError_t launch_pad_copy(const Geom &g, const float *src, float *dst, hipStream_t s);

// sets the thread-local message fdw_last_error returns; returns code
int set_error(int code, const char *msg);

size_t iso_multi_record_bytes(int ndim);
size_t tti_multi_record_bytes(int ndim, int stage);  // stage 1 or 2
void multi_pack_iso(int ndim, const IsoArgs &a, bool live, const SparseArgs &rec, void *dst);
void multi_pack_tti(int ndim, const TtiArgs &a, bool live, const SparseArgs &rec, void *dst1, void *dst2);
hipError_t launch_iso_multi(int ndim, int R, const Geom &g, const void *recs, int n, int64_t max_rec,
                            hipStream_t s);
hipError_t launch_tti_multi(int ndim, int R, const Geom &g, const void *recs1, const void *recs2, int n,
                            int64_t max_rec, hipStream_t s);
hipError_t launch_interp_multi(const SparseArgs *recs, int n, int64_t max_rec, hipStream_t s);

// receivers with linear weights (4 or 8 support points): sampled by
// interp_receiver, also inside the stencil launches
inline bool interp_linear(const SparseArgs &a) { return a.r == 2 && (a.ncorner == 4 || a.ncorner == 8); }

// Whole-run 2D isotropic kernel: one workgroup runs steps time_m..time_M of
// a small 2D grid with the current level resident in LDS.
struct Persist2DArgs {
    Geom g;
    float *u;            // TimeFunction base (nslots slots)
    int64_t slot;        // elements per slot
    int nslots;          // 3, or 2 for in-place storage
    int64_t pitch_x;     // row pitch of the padded layout
    const float *m;
    const float *eta_x, *eta_z;
    float dt2;
    Coefs c;
    int time_m, time_M;
    // sources (any number): padded element offset of corner 0, dt^2 * weights
    int nsrc;
    const int64_t *src_base;
    const float *src_w;
    const float *src_data;  // [nt][nsrc]
    // receivers
    int nrec;
    const int64_t *rec_base;
    const float *rec_w;
    float *rec_data;        // [nt][nrec]
};

// Temporal blocking of the 2D isotropic step: every workgroup advances an
// overlapped patch (its inner tile plus a halo of K R + 1 points) by up to K
// steps in LDS, then writes the inner tile's last two levels.  Reads and
// writes go to different buffers (levels are read from in_*, written to
// out_*), so one launch needs no grid-wide synchronisation.
struct TB2DArgs {
    Geom g;
    const float *in_prev, *in_cur;  // levels t0 - 1, t0
    float *out_prev, *out_cur;      // levels t0 + nsteps - 1, t0 + nsteps (inner tiles)
    const float *m;
    const float *eta_x, *eta_z;
    float dt2;
    Coefs c;
    FusedSrc src;                   // src.q: samples of step t0
    int src_stride;                 // samples per step (row stride of src.q)
    int nsteps;                     // 1 .. K
    int nrec;
    const int *rec_idx;             // [nrec][3] base grid indices (x, 0, z)
    const float *rec_w;             // [nrec][4]
    float *rec_rows;                // row of step t0 (row stride nrec)
};

// Temporal blocking of the 3D isotropic step (two steps per launch): levels
// t - 1, t are read from one buffer pair, levels t + 1, t + 2 written to the
// other; the sources of steps t and t + 1 are fused (their cells and weights
// read from device memory, only by workgroups they touch); rec[0], rec[1] are
// receiver rows sampled in the same launch from levels the launch only reads
// (npoint = 0: none).
struct TB3DFields {
    Geom g;
    const float *in_prev, *in_cur;
    float *out_prev, *out_cur;
    const float *m;
    const float *eta_x, *eta_y, *eta_z;
    float dt2;
};
struct TB3DArgs {
    TB3DFields f;
    Coefs c;
    const FusedSrc *fsrc;     // device copy of the fused sources (n = 0: none)
    const float *q1, *q2;     // source samples of steps t and t + 1
    SparseArgs rec[2];
};
struct TB3DShape {
    int tx, ty;  // output tile
};
TB3DShape tb3d_shape(int R);

// steps per pass and inner tile of the 2D temporal blocking at radius R
struct TB2DShape {
    int k, ix, iz;
};
TB2DShape tb2d_shape(int R);
size_t tb2d_lds_bytes(int R);

// Largest LDS footprint (bytes) the persistent 2D kernel may use.
constexpr int kPersist2DMaxLds = 152 * 1024;

// Kernel variants selectable per operator (FDW_KERNEL environment knob).
enum class IsoVariant { Naive = 0, Stream = 1 };
enum class TtiVariant { Naive = 0, Stream = 1 };

// Optional events recorded by the runtime at the start of the first kernel and
// the end of the last kernel of one step launch (hipExtLaunchKernelGGL), so
// that their elapsed time is the kernels' own execution time.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};

hipError_t launch_iso3d_tb2(int R, const TB3DArgs &a, hipStream_t s, const LaunchEvents &ev);
const char *tb3d_kernel_name(const Geom &g, int R);

// Launchers (fdw_iso.hip, fdw_tti.hip, fdw_sparse.hip).  Each returns the
// hipError_t of its launch.
hipError_t launch_iso(int ndim, int R, IsoVariant v, const IsoArgs &a, hipStream_t s, const LaunchEvents &ev);
// 2D step on the ring engine's flat mode (fdw_iso2d_stream.hip): the same
// bits as the one-thread-per-point 2D kernel; its z-chunk
hipError_t launch_iso2d_stream(int R, const IsoArgs &a, hipStream_t s, const LaunchEvents &ev);
int iso2d_stream_zchunk(const Geom &g);
// TTI 2D stages on the same mode (fdw_tti2d_stream.hip): the same bits as the
// one-thread-per-point 2D stages; their z-chunk
hipError_t launch_tti2d_stream(int R, const TtiArgs &a, hipStream_t s, const LaunchEvents &ev);
int tti2d_stream_zchunk(const Geom &g);
hipError_t launch_tti(int ndim, int R, TtiVariant v, const TtiArgs &a, hipStream_t s, const LaunchEvents &ev);
hipError_t launch_inject(const SparseArgs &a, hipStream_t s);
hipError_t launch_interp(const SparseArgs &a, hipStream_t s);
hipError_t launch_iso2d_persistent(int R, const Persist2DArgs &a, hipStream_t s, const LaunchEvents &ev);
// Several shots of one geometry (shots: device array of n argument records),
// one workgroup each.
hipError_t launch_iso2d_persistent_multi(int R, const Geom &g, const Persist2DArgs *shots, int n, hipStream_t s);
// the two LDS forms of the persistent kernel (zero halo around the level in
// LDS, or the level alone): one shot (one != NULL, its arguments by value) or
// n shots (shots: device array of argument records)
hipError_t launch_iso2d_persistent_halo(int R, const Persist2DArgs *one, const Geom &g, const Persist2DArgs *shots,
                                        int n, size_t lds, hipStream_t s, const LaunchEvents &ev);
hipError_t launch_iso2d_persistent_nohalo(int R, const Persist2DArgs *one, const Geom &g, const Persist2DArgs *shots,
                                          int n, size_t lds, hipStream_t s, const LaunchEvents &ev);
hipError_t launch_iso2d_tb(int R, const TB2DArgs &a, hipStream_t s, const LaunchEvents &ev);
// grad += -nu [(u+ - 2u + u-)/dt^2 + eta (u+ - u-)/(2 dt)] over the domain
struct GradArgs {
    Geom g;
    const float *nu, *u_next, *u_cur, *u_prev;
    float *grad;
    const float *eta_x, *eta_y, *eta_z;  // damping a = eta dt / 2 per axis
    float inv_dt2;                       // 1 / dt^2
};
hipError_t launch_gradient(int ndim, const GradArgs &a, hipStream_t s);
// Standalone imaging kernels (where the step kernels do not fuse them):
// S = imaging_factor(u_next, u_cur, u_prev, a) into grad's place (ImageArgs
// .s_out), and grad -= nu S / dt^2.
struct ImageArgs {
    Geom g;
    const float *u_next, *u_cur, *u_prev;  // factor: levels t + 1, t, t - 1
    float *s_out;
    const float *nu, *s_in;                // update: adjoint level and factor
    float *grad;
    const float *eta_x, *eta_y, *eta_z;
    float inv_dt2;
};
hipError_t launch_imaging_factor(int ndim, const ImageArgs &a, hipStream_t s);
hipError_t launch_image_update(int ndim, const ImageArgs &a, hipStream_t s);
hipError_t launch_zero_halo(int ndim, const Geom &g, int R, int64_t pitch_x, int64_t pitch_y,
                            int64_t planes, float *base, hipStream_t s);

}  // namespace fdw
struct fdw_op;
namespace fdw {
// Floats of TTI gradient buffers an operator's apply needs (2 slots; 0 for
// the isotropic operator), and the apply loop with those buffers at `stage`
// instead of the operator's own, without kernel timing (no event creation).
int64_t operator_stage_floats(const fdw_op *op);
int operator_apply_stage(fdw_op *op, int time_m, int time_M, void *stream, float *stage);
// zero n floats (a fill kernel: no memset node when the stream is captured)
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s);

// Bandwidth probes: kind 0 copies dst = a, kind 1 is the triad dst = a + s b
// (n floats, a multiple of 4, 16-byte aligned pointers).
hipError_t launch_bandwidth_probe(int kind, float *dst, const float *a, const float *b, float s, int64_t n,
                                  hipStream_t st);

// Human-readable description of the launch plan of the dominant kernel.
const char *iso_kernel_name(int ndim, int R, IsoVariant v, const Geom &g, bool sampling);
const char *tti_kernel_name(int ndim, int R, TtiVariant v, const Geom &g);

}  // namespace fdw
