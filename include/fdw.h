/*
 * fdw.h — C ABI of the MI355X (gfx950) finite-difference wave-equation
 * operators: isotropic acoustic and TTI pseudo-acoustic time marching with a
 * damping layer, sparse source injection and receiver interpolation.
 *
 * The calls mirror the problem statement of arXiv 1807.03032 (Devito):
 *   Grid(shape, extent, origin)                 -> fdw_grid_create        (Section 3.1)
 *   Function / TimeFunction(space_order, ...)   -> fdw_function_bind,
 *                                                  fdw_timefunction_bind  (Section 3.1, 3.4)
 *   domain / halo / padding regions             -> fdw_field_layout       (Section 3.5)
 *   SparseTimeFunction(coordinates), inject,
 *   interpolate                                 -> fdw_sparse_bind        (Section 3.2)
 *   PrecomputedSparseFunction                   -> fdw_sparse_bind_precomputed (Section 3.2)
 *   Operator(eqs) ... op.apply(time=...)        -> fdw_operator_create,
 *                                                  fdw_operator_apply     (Section 4 intro, 4.8)
 *
 * Conventions shared by every call
 *  - Status: every int-returning call returns FDW_OK (0) or a negative FDW_ERR_*
 *    code; fdw_last_error() returns a thread-local message for the last
 *    failure on the calling thread.  No C++ exception crosses the ABI.  A
 *    failed call leaves no partially built object and writes nothing to *out.
 *  - Ownership: device buffers passed in (fields, sparse data, receiver
 *    traces) are BORROWED: the library never frees them and the caller keeps
 *    them alive while any handle that references them exists.  Handles
 *    (fdw_grid, fdw_func, fdw_tfunc, fdw_sparse, fdw_op) are owned by the
 *    library and released with the matching *_destroy call.  A handle may be
 *    destroyed only after every handle built from it has been destroyed.
 *  - Threads: handles are not thread-safe; distinct operators may be used from
 *    distinct threads and streams.
 *  - Axes: 2D grids have axes (x, z), 3D grids (x, y, z), z being depth.
 *    Memory is x-fastest (see fdw_field_layout).
 *  - Precision: fields are float32; coordinates and scalars are double and
 *    every derived coefficient is computed in double and rounded once.
 */
#ifndef FDW_H
#define FDW_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FDW_OK 0
#define FDW_ERR_ARG (-1)      /* invalid argument (NULL, range, mismatch)           */
#define FDW_ERR_DOMAIN (-2)   /* a sparse coordinate lies outside the grid          */
#define FDW_ERR_UNSTABLE (-3) /* dt above the stability bound                       */
#define FDW_ERR_LAYOUT (-4)   /* buffer too small for the layout, or misaligned     */
#define FDW_ERR_DEVICE (-5)   /* HIP runtime error (message carries its string)     */
#define FDW_ERR_NOMEM (-6)    /* host or device allocation failed                   */
#define FDW_ERR_STATE (-7)    /* call not valid in the object's current state       */

#define FDW_ISO 0 /* isotropic acoustic:  m u_tt - lap u = q                        */
#define FDW_TTI 1 /* TTI pseudo-acoustic: coupled p, r with rotated operators      */

#define FDW_MAX_SO 16
#define FDW_MAX_SUPPORT 4 /* support points per axis of a precomputed sparse function */
#define FDW_X_OFFSET 32 /* floats before logical x = 0 in each row (128-byte alignment) */

typedef struct fdw_grid fdw_grid;
typedef struct fdw_func fdw_func;
typedef struct fdw_tfunc fdw_tfunc;
typedef struct fdw_sparse fdw_sparse;
typedef struct fdw_op fdw_op;

/* Memory layout of one field (one time slot) for a grid and space order.
 * Section 3.5 (domain, halo, padding): the halo is R = space_order/2 points
 * on every side of every axis and must hold zeros (Dirichlet, Section 7.2);
 * padding aligns logical x = 0 of every row to 128 bytes.
 *   3D element (x, y, z) at  origin_offset + (z * pitch_y + y) * pitch_x + x
 *   2D element (x, z)    at  origin_offset +  z * pitch_x + x
 * A field occupies elems_per_slot floats; a TimeFunction with time_order 2
 * holds nslots = 3 slots back to back, logical time level t in slot t mod 3
 * (Section 3.4: u[t % 3]; level -1 lives in slot 2), or nslots = 2 slots with
 * level t in slot t mod 2 (in-place leapfrog storage, see
 * fdw_timefunction_bind). */
typedef struct {
    int ndim;              /* 2 or 3                                              */
    int halo;              /* R = space_order / 2                                 */
    int64_t shape[3];      /* points per axis (x, y, z) or (x, z)                 */
    int64_t pitch_x;       /* floats per row, a multiple of 32                     */
    int64_t pitch_y;       /* rows per plane: ny + 2R in 3D; nz + 2R in 2D         */
    int64_t planes;        /* nz + 2R in 3D; 1 in 2D                              */
    int64_t origin_offset; /* element offset of logical (0, 0[, 0])               */
    int64_t elems_per_slot;/* pitch_x * pitch_y * planes                          */
    int alignment_bytes;   /* required alignment of every bound pointer (256)     */
} fdw_layout;

/* Operator description (Section 4: Operator built once from its equations,
 * then applied to any data; Section 7.2: the isotropic and TTI test cases).
 * The library copies the struct; the handles it names must outlive the op. */
typedef struct {
    int kind;            /* FDW_ISO or FDW_TTI                                       */
    int space_order;     /* even, 2..16 (the paper measures 4, 8, 12, 16)             */
    double dt;           /* time step; must not exceed fdw_stable_dt(...)             */
    int nbl;             /* damping-layer width in points (0: no damping)             */
    double damp_rc;      /* layer reflection coefficient, (0,1); 0 selects 1e-3       */
    double vmax;         /* largest velocity: damping strength and stability check    */
    double eps_max;      /* TTI: largest epsilon (stability check); ignored for ISO   */
    fdw_tfunc *u;        /* ISO: wavefield u;   TTI: wavefield p                      */
    fdw_tfunc *r;        /* TTI: wavefield r;   ISO: NULL                             */
    fdw_func *m;         /* squared slowness m = 1/v^2 (required)                     */
    fdw_func *eps;       /* TTI: Thomsen epsilon                                      */
    fdw_func *delta;     /* TTI: Thomsen delta                                        */
    fdw_func *theta;     /* TTI: tilt angle (radians)                                 */
    fdw_func *phi;       /* TTI 3D: azimuth angle (radians); NULL in 2D               */
    fdw_sparse *src;     /* sources, injected into u (p and r); may be NULL           */
    fdw_sparse *rec;     /* receivers, sampling u (p); may be NULL                    */
    int mode;            /* FDW_FORWARD, or FDW_ADJOINT (isotropic only), see below   */
} fdw_op_desc;

/* Operator modes.  FDW_ADJOINT builds the transpose of the isotropic
 * source-to-receiver map (the adjoint of Section 3.2's injection/interpolation
 * pair, extended to the whole time loop): with nu = (dt^2/m) D^-1 lambda,
 * D = 1 + eta dt/2, the transposed recurrence is the same leapfrog step run
 * backwards in time.  An adjoint operator is the forward one with two changes:
 * its sources' injected terms dt^2 w q / m are divided by D at each target
 * point (they enter before the damping division), and its receivers sample
 * D u.  To apply F^T to residual traces d[nt][nrec]: bind the receivers as
 * the adjoint operator's src with data d reversed in time, the sources as its
 * rec, run steps 0..nt-1, and reverse the recorded traces in time. */
#define FDW_FORWARD 0
#define FDW_ADJOINT 1

/* Grid(shape, extent, origin), Section 3.1.  ndim in {2, 3}; shape[a] >= 2;
 * extent[a] > 0; spacing h_a = extent[a] / (shape[a] - 1).  origin may be
 * NULL (all zeros).  The shape is the computational domain, absorbing layer
 * included (Section 3.5).  Errors: FDW_ERR_ARG. */
int fdw_grid_create(int ndim, const int64_t *shape, const double *extent, const double *origin,
                    fdw_grid **out);
int fdw_grid_destroy(fdw_grid *grid);

/* Layout of a field of this grid at this space order (Section 3.5); pure host
 * arithmetic, no device call.  Errors: FDW_ERR_ARG. */
int fdw_field_layout(const fdw_grid *grid, int space_order, fdw_layout *out);

/* Function (Section 3.1): a time-invariant parameter field (m, eps, delta,
 * theta, phi).  dptr: device float buffer of nelem floats in the layout of
 * (grid, space_order), 256-byte aligned; only domain points are read.
 * name: informational, copied (may be NULL).
 * Errors: FDW_ERR_ARG (NULL, bad order), FDW_ERR_LAYOUT (nelem < elems_per_slot
 * or misaligned). */
int fdw_function_bind(fdw_grid *grid, const char *name, float *dptr, int64_t nelem, int space_order,
                      fdw_func **out);
int fdw_function_destroy(fdw_func *f);

/* TimeFunction (Section 3.1, 3.4): a wavefield of time order 2 (time_order
 * must be 2) stored in nslots slots, level t in slot t mod nslots:
 *   nslots = 3: the paper's modulo buffer u[t % 3] (time_order + 1 slots);
 *   nslots = 2: in-place leapfrog storage -- step t overwrites level t-1 with
 *               level t+1 point by point (each point's u(t-1) is read only by
 *               the update of that point), one third less memory and per-step
 *               working set; after an apply the slots hold the last two levels.
 * dptr holds nelem >= nslots * elems_per_slot floats, 256-byte aligned.  The
 * caller writes the initial levels -1 and 0 (zeros give the zero initial
 * conditions of eq. WE).  fdw_operator_create zeroes the halo of every slot;
 * the library never writes it afterwards.
 * Errors: FDW_ERR_ARG (time_order, nslots), FDW_ERR_LAYOUT. */
int fdw_timefunction_bind(fdw_grid *grid, const char *name, float *dptr, int64_t nelem,
                          int space_order, int time_order, int nslots, fdw_tfunc **out);
int fdw_timefunction_destroy(fdw_tfunc *f);

/* SparseTimeFunction (Section 3.2, eq. interp, Listing finject).
 * coords_host: host array [npoint][ndim] of physical coordinates (copied);
 * ddata: device float array [nt][npoint] (time-major), source samples read by
 * injection or receiver samples written by interpolation; may be NULL when
 * npoint == 0.  Each point must lie in [o_a, o_a + (shape_a - 1) h_a] on
 * every axis.  Interpolation base b = floor((c - o)/h), clamped to shape - 2;
 * fraction f = (c - o)/h - b; (bi/tri)linear weights, all in double.
 * Allocates library-owned device buffers for the derived indices/weights.
 * Errors: FDW_ERR_ARG, FDW_ERR_DOMAIN, FDW_ERR_NOMEM, FDW_ERR_DEVICE. */
int fdw_sparse_bind(fdw_grid *grid, const char *name, int npoint, int nt, const double *coords_host,
                    float *ddata, fdw_sparse **out);

/* PrecomputedSparseFunction (Section 3.2: grid points and coefficients
 * computed by the caller for a custom interpolation scheme).  Point p is
 * supported on the r^ndim grid points gridpoints[p][a] + j_a, j_a = 0..r-1 on
 * every axis a (axes in grid order, indices of the computational domain), with
 * weight prod_a coeffs[p][a][j_a] (formed in double on the host).  Support
 * point c enumerates (j_0, j_1, ...) with j_0 fastest.  Injection and
 * interpolation use these supports and weights exactly as fdw_sparse_bind's
 * linear ones; r = 2 with coefficients (1 - f, f) and base floor reproduces
 * fdw_sparse_bind.  gridpoints [npoint][ndim] and coeffs [npoint][ndim][r] are
 * host arrays (copied); ddata as for fdw_sparse_bind.
 * Errors: FDW_ERR_ARG (r outside 1..FDW_MAX_SUPPORT, NULL), FDW_ERR_DOMAIN (a
 * support point outside the domain), FDW_ERR_NOMEM. */
int fdw_sparse_bind_precomputed(fdw_grid *grid, const char *name, int npoint, int nt, int r,
                                const int64_t *gridpoints, const double *coeffs, float *ddata,
                                fdw_sparse **out);
int fdw_sparse_destroy(fdw_sparse *s);

/* Operator construction (Section 4: built once, applied many times).
 * Validates kinds, orders, that every field is bound on the same grid at the
 * operator's space order, dt against fdw_stable_dt, and the sparse data
 * lengths; builds the per-axis damping tables and FD coefficients (double,
 * rounded once); allocates the TTI stage buffers; zeroes the halos of the
 * wavefield slots (on the null stream, synchronously).
 * Errors: FDW_ERR_ARG, FDW_ERR_UNSTABLE, FDW_ERR_LAYOUT, FDW_ERR_NOMEM,
 * FDW_ERR_DEVICE. */
int fdw_operator_create(const fdw_op_desc *desc, fdw_op **out);

/* Operator application (Section 4.8: the generated entry point; the time loop
 * of Section 4.5: stencil, then injection, inside t).
 * Runs steps t = time_m .. time_M.  Step t computes level t+1 from levels t
 * and t-1 into slot (t+1) mod 3, injects src[t] (dt^2 q / m at each target
 * point) into level t+1 (into p and r for TTI) and writes rec[t][:] by
 * interpolating level t+1 (p for TTI).  time_M = -1 selects the largest step
 * with no out-of-range sparse access (Section 4.2: nt_src - 1, or
 * nt_rec - 1, the smaller).  Splitting a run into consecutive applies gives
 * the same result as one apply.  Asynchronous: work is enqueued on `stream`
 * (a hipStream_t; NULL = the null stream) and the call returns; launch errors
 * are reported here, execution errors at the next call or fdw_sync.
 * Graphs (Section 4.5's loop captured once): when a call repeats the range and
 * the saving settings of the operator's previous call, its launch sequence is
 * captured into a hipGraph, which that call and later calls with the same key
 * replay on a private stream ordered after `stream`'s earlier work and before
 * its later work (kernel timing on, receiver sampling on a second stream, an
 * open range (time_M = -1) or FDW_APPLY_GRAPH=0: plain launches).  The
 * results are the same bits either way.
 * Errors: FDW_ERR_ARG (range), FDW_ERR_DEVICE. */
int fdw_operator_apply(fdw_op *op, int time_m, int time_M, void *stream);

/* Graphs the operator's applies built and replays launched so far.
 * Errors: FDW_ERR_ARG (NULL op). */
int fdw_operator_graph_stats(const fdw_op *op, int64_t *builds, int64_t *replays);

/* Allocation-free variant of fdw_operator_apply, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same time loop and kernels, with the
 * TTI gradient buffers (2 * elems_per_slot floats, the only scratch the
 * kernels use) taken from a library-owned device array of 64 MiB per GPU
 * instead of the operator's own buffers; the isotropic operator uses no
 * scratch.  It calls no allocating routine and creates no events (kernel
 * timing is not recorded).  The scratch region is cleared on `stream` at the
 * start of each call.  Every call on one GPU shares that GPU's array: calls
 * whose work overlaps on one GPU (several streams, or concurrent host threads)
 * race and must be serialised by the caller.
 * Errors: FDW_ERR_ARG (range; an operator whose gradient buffers exceed the
 * 64 MiB scratch: 3D TTI grids up to about 180^3 fit), FDW_ERR_DEVICE. */
int fdw_operator_apply_noalloc(fdw_op *op, int time_m, int time_M, void *stream);

/* Subsampled level saving (Section 3.4, ConditionalDimension / save=): while
 * the operator runs, every level L >= first_level with
 * (L - first_level) % every == 0 and k = (L - first_level) / every < nlevels
 * is also stored in the buffer (same layout; halos untouched): the isotropic
 * operator stores u at buf + k * elems_per_slot, the TTI operator p at
 * buf + 2k * elems_per_slot and r at buf + (2k + 1) * elems_per_slot (buf
 * holds 2 * nlevels slots).  Level L is the one step L - 1 computes (after
 * injection); the initial level 0 (slot 0) is stored when an apply starts at
 * time_m = 0.  buf = NULL disables saving.  The store is fused into the
 * stencil kernel (TTI: stage 2) when the sources are fused.
 * Errors: FDW_ERR_ARG (every < 1, nlevels < 0). */
int fdw_operator_set_save(fdw_op *op, float *buf, int64_t nlevels, int every, int first_level);

/* Imaging factors of forward steps (the time derivatives the gradient with
 * respect to m needs, Section 3.2's adjoint pairing of injection and
 * interpolation): while set, every step t of an apply with
 * first_step <= t < first_step + nsteps also stores
 *   S(t) = (u(t+1) - 2 u(t) + u(t-1)) + a (u(t+1) - u(t-1)),  a = eta dt / 2,
 * (the imaging bracket times dt^2, from the final level t + 1, sources
 * included) at buf + (t - first_step) * elems_per_slot, same layout, halos
 * untouched; buf holds nsteps slots.  The 3D streaming kernels store it
 * themselves when the sources are fused (4 bytes per point and step more
 * traffic); otherwise a standalone kernel follows the step.  buf = NULL
 * disables it.  Isotropic forward operators whose wavefield has three time
 * slots (u(t-1) must survive the step).
 * Errors: FDW_ERR_ARG (kind or mode, fewer than three slots, nsteps < 1,
 * first_step < 0). */
int fdw_operator_set_imaging_save(fdw_op *op, float *buf, int64_t nsteps, int first_step);

/* Adjoint steps time_m .. time_M of the isotropic adjoint operator `adj`
 * (reversed time: adjoint step tau is forward step nt - 1 - tau) with the
 * zero-lag imaging condition accumulated on `stream`:
 *   grad -= nu(tau + 1) S(nt - 1 - tau) / dt^2
 * for every step of the range, nu(tau + 1) being the level the step computes
 * (its injected residuals included) and S the imaging factors stored by
 * fdw_operator_set_imaging_save (factor of forward step t at
 * imaging + (t - first_step) * elems_per_slot).  The 3D streaming kernels fold
 * the imaging of a level into the next step's launch (it reads that level
 * anyway), the last level of the range getting a launch of its own; other
 * schedules launch it after every step.  Calls over consecutive ranges
 * accumulate the same sums in the same order as one call over their union.
 * grad: one slot in the operator's layout.
 * Errors: FDW_ERR_ARG (kind or mode, steps outside 0 .. nt - 1, forward steps
 * of the range not all among the nsteps factors), FDW_ERR_DEVICE. */
int fdw_gradient_apply(fdw_op *adj, int time_m, int time_M, int nt, const float *imaging, int first_step,
                       int64_t nsteps, float *grad, void *stream);

/* Adjoint-state gradient with respect to m (zero-lag imaging condition of the
 * isotropic operator of `op`): for one step t,
 *   grad += -nu [(u(t+1) - 2 u(t) + u(t-1)) / dt^2 + eta (u(t+1) - u(t-1)) / (2 dt)]
 * over the domain, where nu is the adjoint wavefield level of that step.  All
 * pointers are single slots in the operator's layout.  Enqueued on `stream`.
 * Errors: FDW_ERR_ARG, FDW_ERR_DEVICE. */
int fdw_gradient_accumulate(fdw_op *op, const float *nu, const float *u_next, const float *u_cur,
                            const float *u_prev, float *grad, void *stream);

/* Wait for all work the operator enqueued.  Errors: FDW_ERR_DEVICE. */
int fdw_sync(fdw_op *op);
int fdw_operator_destroy(fdw_op *op);

/* ---------------------------------------------------------------------------
 * Fused multi-shot steps.  fdw_batch_apply advances n operators of the same
 * kind, space order and grid shape (distinct wavefields, models, sources and
 * receivers) over their own step ranges time_m[i]..time_M[i] with one launch
 * per stage and step for all of them (the shot index is a grid dimension);
 * shots with shorter ranges sit out the later launches; 2D isotropic grids
 * small enough for the LDS-resident kernel run one workgroup per shot over
 * its whole range in a single launch.  Each shot's results are those of
 * fdw_operator_apply over the same range, bit for bit.
 * Restrictions: forward mode, no level saving, at most 4 sources with linear
 * weights (fused injection), receivers with linear weights, 3D operators on
 * the streaming kernels.  A batch object owns pinned and device buffers for
 * the per-shot records of one call; on a stream other than the null stream
 * the call's launch sequence is captured in a hipGraph, kept, and replayed by
 * later calls with the same shot count, step count and receiver width.  A
 * call with a single 3D shot runs it through fdw_operator_apply (same bits;
 * no graph and no record upload).
 * Calls on one batch object are ordered on their stream; the object may be
 * reused immediately (the record upload of the previous call is awaited).
 * Errors: FDW_ERR_ARG (mismatch, restriction, range), FDW_ERR_NOMEM,
 * FDW_ERR_DEVICE. */
typedef struct fdw_batch fdw_batch;
int fdw_batch_create(fdw_batch **out);
int fdw_batch_apply(fdw_batch *b, fdw_op *const *ops, int n, const int *time_m, const int *time_M, void *stream);
int fdw_batch_stats(const fdw_batch *b, int64_t *graph_builds, int64_t *graph_launches);
int fdw_batch_destroy(fdw_batch *b);

/* ---------------------------------------------------------------------------
 * Shot server: continuous batching of forward-modelling requests on one GPU.
 * Requests (kind, grid, space order, step count, model, sources, receivers)
 * are queued by fdw_server_submit.  Each fdw_server_progress call is one
 * non-blocking scheduling round: it retires shots whose work has completed
 * (receiver traces already copied to host memory), admits queued requests in
 * arrival order while their device footprint fits in the budget left (later
 * requests may pass one that does not fit; a few milliseconds of admissions
 * per call, the rest in later calls), and enqueues the next chunk of steps of
 * every bucket of running shots -- shots of one kind, grid and space order --
 * as fused multi-shot launches (fdw_batch_apply, replayed hipGraphs).  Buckets
 * of shots that fill the GPU alone (4 Mi grid points or more) advance one at a
 * time, oldest first, on the first stream; the others share the remaining
 * nstreams - 1 streams and overlap with them on the device (nstreams = 1: one
 * stream for all).  Shots join and leave their bucket between chunks; chunk
 * length aims at chunk_target_us of device time (0: 20 ms).
 * Ownership: the host arrays a description points to are borrowed until the
 * shot is admitted (fdw_server_info state RUNNING or DONE); the server owns
 * all device memory (wavefields in two-slot in-place storage).  budget_bytes
 * <= 0 selects 80 % of the free device memory.  Single-threaded: calls on one
 * server must not overlap.
 * A request whose operator cannot be built (for instance dt above the
 * stability bound), or that cannot be allocated even with nothing else
 * resident, ends in state FDW_SHOT_FAILED instead of blocking the queue;
 * fdw_server_fetch then returns FDW_ERR_STATE with the reason.
 * Errors: FDW_ERR_ARG, FDW_ERR_NOMEM (footprint above the budget at submit),
 * FDW_ERR_STATE (fetch before completion, failed shot), FDW_ERR_DEVICE. */
#define FDW_SHOT_QUEUED 0
#define FDW_SHOT_RUNNING 1
#define FDW_SHOT_DONE 2
#define FDW_SHOT_FAILED 3  /* rejected at admission or a chunk refused (operator errors); see fdw_server_fetch */

typedef struct {
    int kind;                  /* FDW_ISO or FDW_TTI                                     */
    int ndim;                  /* 2 or 3                                                 */
    int64_t shape[3];          /* as fdw_grid_create                                     */
    double extent[3], origin[3];
    int space_order;           /* even, 2..16                                            */
    int nt;                    /* steps 0..nt-1                                          */
    double dt;
    int nbl;
    double damp_rc, vmax, eps_max;
    const float *m;            /* host logical arrays, x fastest (numpy order reversed)  */
    const float *eps, *delta, *theta, *phi;  /* TTI (phi 3D only); NULL for ISO          */
    int nsrc;                  /* 0..4                                                   */
    const double *src_coords;  /* [nsrc][ndim]                                           */
    const float *src;          /* [nt][nsrc]                                             */
    int nrec;
    const double *rec_coords;  /* [nrec][ndim]                                           */
    int keep_field;            /* 1: keep the last level of u (p) for fdw_server_fetch   */
} fdw_shot_desc;

typedef struct {
    int state;                 /* FDW_SHOT_QUEUED / RUNNING / DONE                       */
    int steps_done;
    int64_t footprint;         /* device bytes held while running                        */
    double t_submit, t_admit, t_done;  /* seconds on the server's clock                  */
} fdw_shot_info;

typedef struct {
    int64_t budget, used, pool_bytes;  /* bytes                                          */
    int64_t chunks, admitted, completed, buckets;
    int64_t graph_builds, graph_launches;
    double now;                /* the server's clock (seconds since creation)            */
    double admit_seconds;      /* host time spent admitting (uploads, operator set-up)   */
    double launch_seconds;     /* host time spent packing and enqueueing chunks          */
} fdw_server_stats_t;

typedef struct fdw_server fdw_server;
int fdw_server_create(int64_t budget_bytes, int chunk_target_us, int nstreams, fdw_server **out);
int fdw_server_footprint(const fdw_shot_desc *d, int64_t *bytes);  /* host only */
int fdw_server_submit(fdw_server *sv, const fdw_shot_desc *d, int64_t *ticket);
int fdw_server_progress(fdw_server *sv, int *queued, int *running);
int fdw_server_info(fdw_server *sv, int64_t ticket, fdw_shot_info *out);
/* rec_host [nt][nrec] and/or field_host (logical last level) of a DONE shot */
int fdw_server_fetch(fdw_server *sv, int64_t ticket, float *rec_host, float *field_host);
int fdw_server_release(fdw_server *sv, int64_t ticket);
int fdw_server_stats(fdw_server *sv, fdw_server_stats_t *out);
int fdw_server_destroy(fdw_server *sv);

/* Per-kernel timing (measurement support).  enable = k > 0 times the launches
 * of the operator's dominant stencil kernel in runs of k consecutive launches:
 * the first launch of a run carries a HIP start event and the last a stop
 * event, on the apply stream (an apply that ends inside a run closes it with
 * an event after its last launch); 0 disables.  Every launch is covered; the
 * per-launch average includes the (small) gaps between the launches of a run
 * and 1/k of the events' own cost of a few microseconds.  k = 1 brackets each
 * launch alone.  fdw_operator_kernel_time synchronises and returns the summed
 * milliseconds of all runs and the number of launches they cover since the
 * last reset.  Errors: FDW_ERR_ARG (NULL op, k < 0), FDW_ERR_DEVICE. */
int fdw_operator_set_timing(fdw_op *op, int enable);
int fdw_operator_kernel_time(fdw_op *op, double *total_ms, int64_t *launches, int reset);

/* Description of the launch plan apply will use (kernel name, tile sizes,
 * algorithmic bytes per grid point per step of the dominant kernel).
 * Writes a NUL-terminated string of at most buflen bytes.  Errors: FDW_ERR_ARG. */
int fdw_operator_describe(const fdw_op *op, char *buf, int buflen, double *alg_bytes_per_point);

/* Bandwidth probe (measurement support; Section 7.1 takes the STREAM triad
 * rate as the attainable memory bandwidth of its roofline plots): one launch
 * of a plain streaming kernel over n floats on `stream`.  kind 0: copy
 * dst = a (reads and writes 4 n bytes each); kind 1: triad dst = a + s b
 * (reads 8 n, writes 4 n bytes).  dst, a, b: device buffers owned by the
 * caller, 16-byte aligned, n a multiple of 4 (b unused for kind 0).
 * Asynchronous.  Errors: FDW_ERR_ARG (NULL pointer, misalignment, n not a
 * multiple of 4, unknown kind), FDW_ERR_DEVICE. */
int fdw_bandwidth_probe(int kind, float *dst, const float *a, const float *b, float s, int64_t n, void *stream);

/* Largest stable dt for the leapfrog scheme at this order (von Neumann bound
 * of the order-so Laplacian: dt <= 2 / (v_eff sqrt(sum_a lambda_so / h_a^2)),
 * with equal spacing hmin on every axis; v_eff = vmax for ISO and
 * vmax sqrt(1 + 2 eps_max) for TTI).  Returns a negative value on bad input. */
double fdw_stable_dt(int kind, int ndim, int space_order, double vmax, double eps_max, double hmin);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *fdw_last_error(void);

/* Library version string. */
const char *fdw_version(void);

#ifdef __cplusplus
}
#endif
#endif /* FDW_H */
