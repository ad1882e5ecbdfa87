// Host implementation of the fdw C ABI (include/fdw.h): handle objects,
// argument validation, layout arithmetic, coefficient and damping tables,
// sparse-point preprocessing and the per-step launch sequence.
//
// Paper: arXiv 1807.03032.  Grid / Function / TimeFunction /
// SparseTimeFunction follow Section 3.1; domain/halo/padding Section 3.5;
// interpolation and injection Section 3.2 (eq. interp, Listing finject);
// the operator and its time loop Sections 4 and 4.5.
#include "fdw.h"
#include "fdw_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace fdw;

// ---------------------------------------------------------------------------
// Error reporting: thread-local message, status codes, no exceptions out.
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

static int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int fdw::set_error(int code, const char *msg) {
    g_last_error = msg;
    return code;
}

static int fail_hip(hipError_t e, const char *where) {
    return fail(FDW_ERR_DEVICE, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

#define FDW_GUARD_BEGIN try {
#define FDW_GUARD_END                                                   \
    }                                                                   \
    catch (const std::bad_alloc &) {                                    \
        return fail(FDW_ERR_NOMEM, "host allocation failed");           \
    }                                                                   \
    catch (...) {                                                       \
        return fail(FDW_ERR_ARG, "unexpected internal exception");      \
    }

// ---------------------------------------------------------------------------
// Objects
// ---------------------------------------------------------------------------
struct fdw_grid {
    int ndim;
    int64_t shape[3];  // as given: (x, y, z) or (x, z)
    double extent[3], origin[3], h[3];
    int refs = 0;      // live handles built on this grid
};

struct fdw_func {
    fdw_grid *grid;
    std::string name;
    float *d;
    int64_t nelem;
    int so;
    fdw_layout lay;
    int refs = 0;
};

struct fdw_tfunc {
    fdw_grid *grid;
    std::string name;
    float *d;
    int64_t nelem;
    int so;
    int time_order;
    int nslots;  // 3: level t in slot t mod 3; 2: in-place leapfrog
    fdw_layout lay;
    int refs = 0;
};

struct fdw_sparse {
    fdw_grid *grid;
    std::string name;
    int npoint, nt;
    float *data;                      // caller's [nt][npoint]
    int r = 2;                        // support points per axis
    int ncorner = 0;                  // r^ndim
    std::vector<int64_t> base;        // [npoint][ndim] grid indices of the first support point
    std::vector<double> w;            // [npoint][ncorner] weights
    int refs = 0;
};

struct fdw_op {
    fdw_op_desc d;
    int ndim, R;
    fdw_layout lay;
    Geom geom;
    Coefs coefs;
    float dt2;
    IsoVariant iso_v = IsoVariant::Naive;
    TtiVariant tti_v = TtiVariant::Naive;
    bool use_persist2d = false;  // 2D iso grid small enough for the LDS-resident kernel
    bool use_tb2d = false;       // 2D iso: K steps per launch on overlapped LDS patches
    bool use_tb3d = false;       // 3D iso: two steps per launch
    float *d_tb = nullptr;       // temporal blocking: second pair of level buffers
    FusedSrc *d_fsrc = nullptr;  // device copy of the fused sources (3D temporal blocking)
    // library-owned device memory
    float *d_eta = nullptr;           // eta_x | eta_y | eta_z (times dt/2)
    float *d_stage = nullptr;         // TTI: gp | gr (each elems_per_slot)
    int64_t *d_src_base = nullptr, *d_rec_base = nullptr;
    float *d_src_w = nullptr, *d_rec_w = nullptr;
    int *d_src_idx = nullptr, *d_rec_idx = nullptr;  // [npoint][3] base grid indices
    // injection by gather (SparseArgs::ntarget): targets, offsets, lane
    // points, lane weights, damping divisors
    int src_ntarget = 0;
    int64_t *d_src_tgt = nullptr;
    int *d_src_goff = nullptr, *d_src_gp = nullptr;
    float *d_src_gw = nullptr, *d_src_gd = nullptr;
    // subsampled level saving
    float *save_buf = nullptr;
    int64_t save_nlevels = 0;
    int save_every = 1, save_first = 0;
    // imaging factors of forward steps first .. first + n - 1 (isotropic forward)
    float *isave_buf = nullptr;
    int64_t isave_n = 0;
    int isave_first = 0;
    // host copies of the fused-source description
    FusedSrc fsrc_template;
    bool src_fused = false;
    // timing
    bool timing = false;
    int timing_every = 1;    // launches per timed run
    int run_len = 0;         // launches in the open run
    bool run_open = false;
    hipEvent_t run_start = nullptr, run_stop = nullptr;
    std::vector<hipEvent_t> ev_pool;  // pairs
    size_t ev_used = 0;
    double acc_ms = 0.0;
    int64_t acc_launches = 0;
    hipStream_t last_stream = nullptr;
    // receiver sampling overlapped with the next steps on a second stream
    bool overlap_interp = false;
    hipStream_t side = nullptr;
    std::vector<hipEvent_t> ev_step, ev_interp;  // ring of nslots + 1 each
    // apply graph: a range applied a second time with the same settings is
    // captured then, and replayed on a private stream from then on
    std::vector<int64_t> graph_key, graph_seen;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t graph_stream = nullptr;
    hipEvent_t graph_ev[2] = {nullptr, nullptr};
    int64_t graph_builds = 0, graph_replays = 0;
};

// ---------------------------------------------------------------------------
// Layout (Section 3.5: domain, halo, padding)
// ---------------------------------------------------------------------------
static bool valid_so(int so) { return so >= 2 && so <= FDW_MAX_SO && (so % 2) == 0; }

static void compute_layout(const fdw_grid *g, int so, fdw_layout *L) {
    const int R = so / 2;
    std::memset(L, 0, sizeof(*L));
    L->ndim = g->ndim;
    L->halo = R;
    for (int a = 0; a < g->ndim; ++a) L->shape[a] = g->shape[a];
    const int64_t nx = g->shape[0];
    const int64_t need = FDW_X_OFFSET + nx + R;
    L->pitch_x = (need + 31) / 32 * 32;
    if (g->ndim == 3) {
        L->pitch_y = g->shape[1] + 2 * R;
        L->planes = g->shape[2] + 2 * R;
        L->origin_offset = (int64_t)R * L->pitch_y * L->pitch_x + (int64_t)R * L->pitch_x + FDW_X_OFFSET;
    } else {
        L->pitch_y = g->shape[1] + 2 * R;
        L->planes = 1;
        L->origin_offset = (int64_t)R * L->pitch_x + FDW_X_OFFSET;
    }
    L->elems_per_slot = L->pitch_x * L->pitch_y * L->planes;
    L->alignment_bytes = 256;
}

// ---------------------------------------------------------------------------
// Finite-difference weights: closed forms of the centred Taylor stencils of
// order so = 2R (Section 3.2, the `.dx`/`.laplace` shortcuts):
//   W2_k = 2 (-1)^(k+1) (R!)^2 / (k^2 (R-k)! (R+k)!),  W2_0 = -2 sum_k W2_k
//   W1_k =   (-1)^(k+1) (R!)^2 / (k   (R-k)! (R+k)!)
// ---------------------------------------------------------------------------
static double lfact(int n) { return std::lgamma((double)n + 1.0); }

static void taylor_weights(int R, double *w1, double *w2) {
    double s = 0.0;
    w1[0] = 0.0;
    for (int k = 1; k <= R; ++k) {
        const double mag = std::exp(2.0 * lfact(R) - lfact(R - k) - lfact(R + k));
        const double sign = (k % 2) ? 1.0 : -1.0;
        w1[k] = sign * mag / k;
        w2[k] = 2.0 * sign * mag / ((double)k * k);
        s += w2[k];
    }
    w2[0] = -2.0 * s;
}

// max over the Nyquist band of the symbol of -d2/dx2 (unit spacing)
static double laplace_symbol_max(int R) {
    double w1[kMaxR + 1], w2[kMaxR + 1];
    taylor_weights(R, w1, w2);
    double best = 0.0;
    for (int j = 0; j <= 2048; ++j) {
        const double th = M_PI * j / 2048.0;
        double s = -w2[0];
        for (int k = 1; k <= R; ++k) s -= 2.0 * w2[k] * std::cos(k * th);
        best = std::max(best, s);
    }
    return best;
}

static double stable_dt_axes(int kind, int ndim, int so, double vmax, double eps_max, const double *h) {
    if ((kind != FDW_ISO && kind != FDW_TTI) || (ndim != 2 && ndim != 3) || !valid_so(so) || !(vmax > 0.0) ||
        !(eps_max >= 0.0))
        return -1.0;
    const double lam = laplace_symbol_max(so / 2);
    double sum = 0.0;
    for (int a = 0; a < ndim; ++a) {
        if (!(h[a] > 0.0)) return -1.0;
        sum += lam / (h[a] * h[a]);
    }
    const double veff = kind == FDW_TTI ? vmax * std::sqrt(1.0 + 2.0 * eps_max) : vmax;
    return 2.0 / (veff * std::sqrt(sum));
}

// ---------------------------------------------------------------------------
// Public ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fdw_last_error(void) { return g_last_error.c_str(); }
const char *fdw_version(void) { return "fdw 0.1 (gfx950)"; }

double fdw_stable_dt(int kind, int ndim, int space_order, double vmax, double eps_max, double hmin) {
    const double h[3] = {hmin, hmin, hmin};
    return stable_dt_axes(kind, ndim, space_order, vmax, eps_max, h);
}

int fdw_grid_create(int ndim, const int64_t *shape, const double *extent, const double *origin,
                    fdw_grid **out) {
    FDW_GUARD_BEGIN
    if (!out) return fail(FDW_ERR_ARG, "grid_create: out is NULL");
    if (ndim != 2 && ndim != 3) return fail(FDW_ERR_ARG, "grid_create: ndim must be 2 or 3 (got %d)", ndim);
    if (!shape || !extent) return fail(FDW_ERR_ARG, "grid_create: shape/extent is NULL");
    for (int a = 0; a < ndim; ++a) {
        if (shape[a] < 2 || shape[a] > (1 << 20))
            return fail(FDW_ERR_ARG, "grid_create: shape[%d] = %lld out of range [2, 2^20]", a,
                        (long long)shape[a]);
        if (!(extent[a] > 0.0) || !std::isfinite(extent[a]))
            return fail(FDW_ERR_ARG, "grid_create: extent[%d] must be positive", a);
        if (origin && !std::isfinite(origin[a])) return fail(FDW_ERR_ARG, "grid_create: origin[%d] not finite", a);
    }
    fdw_grid *g = new fdw_grid();
    g->ndim = ndim;
    for (int a = 0; a < 3; ++a) {
        g->shape[a] = a < ndim ? shape[a] : 1;
        g->extent[a] = a < ndim ? extent[a] : 0.0;
        g->origin[a] = (a < ndim && origin) ? origin[a] : 0.0;
        g->h[a] = a < ndim ? extent[a] / (double)(shape[a] - 1) : 1.0;
    }
    *out = g;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_grid_destroy(fdw_grid *grid) {
    if (!grid) return FDW_OK;
    if (grid->refs > 0) return fail(FDW_ERR_STATE, "grid_destroy: %d handles still use this grid", grid->refs);
    delete grid;
    return FDW_OK;
}

int fdw_field_layout(const fdw_grid *grid, int space_order, fdw_layout *out) {
    if (!grid || !out) return fail(FDW_ERR_ARG, "field_layout: NULL argument");
    if (!valid_so(space_order)) return fail(FDW_ERR_ARG, "field_layout: space_order %d not even in [2,16]", space_order);
    compute_layout(grid, space_order, out);
    return FDW_OK;
}

static int check_buffer(const char *what, const void *p, int64_t nelem, int64_t need) {
    if (!p) return fail(FDW_ERR_ARG, "%s: device pointer is NULL", what);
    if (((uintptr_t)p) % 256 != 0) return fail(FDW_ERR_LAYOUT, "%s: pointer not 256-byte aligned", what);
    if (nelem < need)
        return fail(FDW_ERR_LAYOUT, "%s: buffer holds %lld floats, layout needs %lld", what, (long long)nelem,
                    (long long)need);
    return FDW_OK;
}

int fdw_function_bind(fdw_grid *grid, const char *name, float *dptr, int64_t nelem, int space_order,
                      fdw_func **out) {
    FDW_GUARD_BEGIN
    if (!grid || !out) return fail(FDW_ERR_ARG, "function_bind: NULL grid/out");
    if (!valid_so(space_order)) return fail(FDW_ERR_ARG, "function_bind: space_order %d not even in [2,16]", space_order);
    fdw_layout L;
    compute_layout(grid, space_order, &L);
    int st = check_buffer("function_bind", dptr, nelem, L.elems_per_slot);
    if (st) return st;
    fdw_func *f = new fdw_func();
    f->grid = grid;
    f->name = name ? name : "";
    f->d = dptr;
    f->nelem = nelem;
    f->so = space_order;
    f->lay = L;
    grid->refs++;
    *out = f;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_function_destroy(fdw_func *f) {
    if (!f) return FDW_OK;
    if (f->refs > 0) return fail(FDW_ERR_STATE, "function_destroy: used by %d operators", f->refs);
    f->grid->refs--;
    delete f;
    return FDW_OK;
}

int fdw_timefunction_bind(fdw_grid *grid, const char *name, float *dptr, int64_t nelem, int space_order,
                          int time_order, int nslots, fdw_tfunc **out) {
    FDW_GUARD_BEGIN
    if (!grid || !out) return fail(FDW_ERR_ARG, "timefunction_bind: NULL grid/out");
    if (!valid_so(space_order))
        return fail(FDW_ERR_ARG, "timefunction_bind: space_order %d not even in [2,16]", space_order);
    if (time_order != 2) return fail(FDW_ERR_ARG, "timefunction_bind: time_order must be 2 (got %d)", time_order);
    if (nslots != 2 && nslots != 3) return fail(FDW_ERR_ARG, "timefunction_bind: nslots must be 2 or 3 (got %d)", nslots);
    fdw_layout L;
    compute_layout(grid, space_order, &L);
    int st = check_buffer("timefunction_bind", dptr, nelem, (int64_t)nslots * L.elems_per_slot);
    if (st) return st;
    fdw_tfunc *f = new fdw_tfunc();
    f->grid = grid;
    f->name = name ? name : "";
    f->d = dptr;
    f->nelem = nelem;
    f->so = space_order;
    f->time_order = time_order;
    f->nslots = nslots;
    f->lay = L;
    grid->refs++;
    *out = f;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_timefunction_destroy(fdw_tfunc *f) {
    if (!f) return FDW_OK;
    if (f->refs > 0) return fail(FDW_ERR_STATE, "timefunction_destroy: used by %d operators", f->refs);
    f->grid->refs--;
    delete f;
    return FDW_OK;
}

int fdw_sparse_bind(fdw_grid *grid, const char *name, int npoint, int nt, const double *coords_host,
                    float *ddata, fdw_sparse **out) {
    FDW_GUARD_BEGIN
    if (!grid || !out) return fail(FDW_ERR_ARG, "sparse_bind: NULL grid/out");
    if (npoint < 0 || nt < 0) return fail(FDW_ERR_ARG, "sparse_bind: negative npoint/nt");
    if (npoint > 0 && (!coords_host || !ddata)) return fail(FDW_ERR_ARG, "sparse_bind: NULL coords/data");
    if (npoint > 0 && nt < 1) return fail(FDW_ERR_ARG, "sparse_bind: nt must be >= 1");
    const int nd = grid->ndim, nc = 1 << nd;
    std::vector<int64_t> base((size_t)npoint * nd);
    std::vector<double> w((size_t)npoint * nc);
    for (int p = 0; p < npoint; ++p) {
        double f[3];
        for (int a = 0; a < nd; ++a) {
            const double c = coords_host[(size_t)p * nd + a];
            const double xi = (c - grid->origin[a]) / grid->h[a];
            if (!(xi >= 0.0 && xi <= (double)(grid->shape[a] - 1)))
                return fail(FDW_ERR_DOMAIN, "sparse_bind(%s): point %d axis %d coordinate %g outside [%g, %g]",
                            name ? name : "", p, a, c, grid->origin[a],
                            grid->origin[a] + grid->h[a] * (double)(grid->shape[a] - 1));
            int64_t b = (int64_t)std::floor(xi);
            b = std::min<int64_t>(b, grid->shape[a] - 2);
            base[(size_t)p * nd + a] = b;
            f[a] = xi - (double)b;
        }
        for (int c = 0; c < nc; ++c) {
            double ww = 1.0;
            for (int a = 0; a < nd; ++a) ww *= ((c >> a) & 1) ? f[a] : (1.0 - f[a]);
            w[(size_t)p * nc + c] = ww;
        }
    }
    fdw_sparse *s = new fdw_sparse();
    s->grid = grid;
    s->name = name ? name : "";
    s->npoint = npoint;
    s->nt = nt;
    s->data = ddata;
    s->r = 2;
    s->ncorner = nc;
    s->base.swap(base);
    s->w.swap(w);
    grid->refs++;
    *out = s;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_sparse_bind_precomputed(fdw_grid *grid, const char *name, int npoint, int nt, int r,
                                const int64_t *gridpoints, const double *coeffs, float *ddata, fdw_sparse **out) {
    FDW_GUARD_BEGIN
    if (!grid || !out) return fail(FDW_ERR_ARG, "sparse_bind_precomputed: NULL grid/out");
    if (npoint < 0 || nt < 0) return fail(FDW_ERR_ARG, "sparse_bind_precomputed: negative npoint/nt");
    if (r < 1 || r > FDW_MAX_SUPPORT)
        return fail(FDW_ERR_ARG, "sparse_bind_precomputed: r = %d outside [1, %d]", r, FDW_MAX_SUPPORT);
    if (npoint > 0 && (!gridpoints || !coeffs || !ddata))
        return fail(FDW_ERR_ARG, "sparse_bind_precomputed: NULL gridpoints/coeffs/data");
    if (npoint > 0 && nt < 1) return fail(FDW_ERR_ARG, "sparse_bind_precomputed: nt must be >= 1");
    const int nd = grid->ndim;
    int nc = 1;
    for (int a = 0; a < nd; ++a) nc *= r;
    std::vector<int64_t> base((size_t)npoint * nd);
    std::vector<double> w((size_t)npoint * nc);
    for (int p = 0; p < npoint; ++p) {
        for (int a = 0; a < nd; ++a) {
            const int64_t b = gridpoints[(size_t)p * nd + a];
            if (b < 0 || b + r - 1 > grid->shape[a] - 1)
                return fail(FDW_ERR_DOMAIN, "sparse_bind_precomputed(%s): point %d axis %d support [%lld, %lld] outside [0, %lld]",
                            name ? name : "", p, a, (long long)b, (long long)(b + r - 1), (long long)(grid->shape[a] - 1));
            base[(size_t)p * nd + a] = b;
        }
        for (int c = 0; c < nc; ++c) {
            double ww = 1.0;
            int rest = c;
            for (int a = 0; a < nd; ++a) {
                ww *= coeffs[((size_t)p * nd + a) * r + rest % r];
                rest /= r;
            }
            w[(size_t)p * nc + c] = ww;
        }
    }
    fdw_sparse *s = new fdw_sparse();
    s->grid = grid;
    s->name = name ? name : "";
    s->npoint = npoint;
    s->nt = nt;
    s->data = ddata;
    s->r = r;
    s->ncorner = nc;
    s->base.swap(base);
    s->w.swap(w);
    grid->refs++;
    *out = s;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_sparse_destroy(fdw_sparse *s) {
    if (!s) return FDW_OK;
    if (s->refs > 0) return fail(FDW_ERR_STATE, "sparse_destroy: used by %d operators", s->refs);
    s->grid->refs--;
    delete s;
    return FDW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Operator construction helpers
// ---------------------------------------------------------------------------
static void drop_apply_graph(fdw_op *op) {
    if (op->graph_exec) (void)hipGraphExecDestroy(op->graph_exec);
    if (op->graph) (void)hipGraphDestroy(op->graph);
    op->graph_exec = nullptr;
    op->graph = nullptr;
    op->graph_key.clear();
}

static void release_device(fdw_op *op) {
    drop_apply_graph(op);
    for (hipEvent_t &e : op->graph_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
    if (op->graph_stream) (void)hipStreamDestroy(op->graph_stream);
    op->graph_stream = nullptr;
    if (op->d_eta) (void)hipFree(op->d_eta);
    if (op->d_stage) (void)hipFree(op->d_stage);
    if (op->d_fsrc) (void)hipFree(op->d_fsrc);
    op->d_fsrc = nullptr;
    if (op->d_tb) (void)hipFree(op->d_tb);
    op->d_tb = nullptr;
    if (op->d_src_base) (void)hipFree(op->d_src_base);
    if (op->d_rec_base) (void)hipFree(op->d_rec_base);
    if (op->d_src_w) (void)hipFree(op->d_src_w);
    if (op->d_rec_w) (void)hipFree(op->d_rec_w);
    if (op->d_src_idx) (void)hipFree(op->d_src_idx);
    if (op->d_rec_idx) (void)hipFree(op->d_rec_idx);
    op->d_src_idx = op->d_rec_idx = nullptr;
    if (op->d_src_tgt) (void)hipFree(op->d_src_tgt);
    if (op->d_src_goff) (void)hipFree(op->d_src_goff);
    if (op->d_src_gp) (void)hipFree(op->d_src_gp);
    if (op->d_src_gw) (void)hipFree(op->d_src_gw);
    if (op->d_src_gd) (void)hipFree(op->d_src_gd);
    op->d_src_tgt = nullptr;
    op->d_src_goff = op->d_src_gp = nullptr;
    op->d_src_gw = op->d_src_gd = nullptr;
    op->src_ntarget = 0;
    for (hipEvent_t e : op->ev_pool) (void)hipEventDestroy(e);
    op->ev_pool.clear();
    for (hipEvent_t e : op->ev_step) (void)hipEventDestroy(e);
    for (hipEvent_t e : op->ev_interp) (void)hipEventDestroy(e);
    op->ev_step.clear();
    op->ev_interp.clear();
    if (op->side) (void)hipStreamDestroy(op->side);
    op->side = nullptr;
    op->d_eta = op->d_stage = op->d_src_w = op->d_rec_w = nullptr;
    op->d_src_base = op->d_rec_base = nullptr;
}

// element offset of grid point (x, y, z) (2D: y ignored, idx[1] is z)
static int64_t element_offset(const fdw_op *op, const int64_t *idx) {
    if (op->ndim == 3) return op->geom.off0 + idx[2] * op->geom.sz + idx[1] * op->geom.sy + idx[0];
    return op->geom.off0 + idx[1] * op->geom.sz + idx[0];
}

static int upload_sparse(fdw_op *op, const fdw_sparse *s, double scale, int64_t **d_base, float **d_w, int **d_idx) {
    const int nc = s->ncorner;
    std::vector<int64_t> off(s->npoint);
    std::vector<float> w((size_t)s->npoint * nc);
    std::vector<int> idx((size_t)std::max(1, s->npoint) * 3, 0);
    for (int p = 0; p < s->npoint; ++p) {
        const int64_t *b = &s->base[(size_t)p * op->ndim];
        idx[(size_t)p * 3 + 0] = (int)b[0];
        idx[(size_t)p * 3 + 1] = op->ndim == 3 ? (int)b[1] : 0;
        idx[(size_t)p * 3 + 2] = (int)b[op->ndim - 1];
        off[p] = element_offset(op, &s->base[(size_t)p * op->ndim]);
        for (int c = 0; c < nc; ++c) w[(size_t)p * nc + c] = (float)(scale * s->w[(size_t)p * nc + c]);
    }
    hipError_t e = hipMalloc((void **)d_base, sizeof(int64_t) * std::max(1, s->npoint));
    if (e != hipSuccess) return fail(FDW_ERR_NOMEM, "operator_create: hipMalloc sparse base: %s", hipGetErrorString(e));
    e = hipMalloc((void **)d_w, sizeof(float) * std::max<size_t>(1, w.size()));
    if (e != hipSuccess) return fail(FDW_ERR_NOMEM, "operator_create: hipMalloc sparse weights: %s", hipGetErrorString(e));
    e = hipMalloc((void **)d_idx, sizeof(int) * idx.size());
    if (e != hipSuccess) return fail(FDW_ERR_NOMEM, "operator_create: hipMalloc sparse indices: %s", hipGetErrorString(e));
    if (s->npoint > 0) {
        e = hipMemcpy(*d_base, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(*d_w, w.data(), sizeof(float) * w.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(*d_idx, idx.data(), sizeof(int) * idx.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail_hip(e, "operator_create: sparse upload");
    }
    return FDW_OK;
}

// Injection of many sparse points as a gather: every lane's target element
// (corner offsets as the kernels compute them: digit k of c in base r along
// axis k), sorted by target then lane, grouped per target, with the lane's
// point and weight (scaled as upload_sparse scales them) and the target's
// damping divisor 1 + a (the float sum corner_damp forms on the device).
constexpr int64_t kGatherMinLanes = 4096;
static int build_inject_gather(fdw_op *op, const fdw_sparse *s, double scale, const std::vector<float> &eta) {
    const int nc = s->ncorner, r = s->r;
    const int64_t lanes = (int64_t)s->npoint * nc;
    if (lanes < kGatherMinLanes || lanes > INT32_MAX) return FDW_OK;
    const int64_t st1 = op->ndim == 3 ? op->geom.sy : op->geom.sz, st2 = op->ndim == 3 ? op->geom.sz : 0;
    const int nx = op->geom.nx, ny = op->geom.ny;
    struct Lane {
        int64_t tgt;
        int lane;
        float d;
    };
    std::vector<Lane> tl((size_t)lanes);
    for (int p = 0; p < s->npoint; ++p) {
        const int64_t *b = &s->base[(size_t)p * op->ndim];
        const int64_t b0 = element_offset(op, b);
        for (int c = 0; c < nc; ++c) {
            const int j0 = c % r, j1 = (c / r) % r, j2 = c / (r * r);
            float a;
            if (op->ndim == 3)
                a = eta[(size_t)(b[0] + j0)] + eta[(size_t)(nx + b[1] + j1)] + eta[(size_t)(nx + ny + b[2] + j2)];
            else
                a = eta[(size_t)(b[0] + j0)] + eta[(size_t)(nx + ny + b[1] + j1)];
            tl[(size_t)p * nc + c] = {b0 + j0 + j1 * st1 + j2 * st2, p * nc + c, 1.0f + a};
        }
    }
    std::sort(tl.begin(), tl.end(),
              [](const Lane &x, const Lane &y) { return x.tgt != y.tgt ? x.tgt < y.tgt : x.lane < y.lane; });
    std::vector<int64_t> tgt;
    std::vector<int> goff, gp((size_t)lanes);
    std::vector<float> gw((size_t)lanes), gd;
    for (size_t k = 0; k < tl.size(); ++k) {
        if (k == 0 || tl[k].tgt != tl[k - 1].tgt) {
            tgt.push_back(tl[k].tgt);
            goff.push_back((int)k);
            gd.push_back(tl[k].d);
        }
        gp[k] = tl[k].lane / nc;
        gw[k] = (float)(scale * s->w[(size_t)tl[k].lane]);
    }
    goff.push_back((int)lanes);
    hipError_t e = hipMalloc((void **)&op->d_src_tgt, sizeof(int64_t) * tgt.size());
    if (e == hipSuccess) e = hipMalloc((void **)&op->d_src_goff, sizeof(int) * goff.size());
    if (e == hipSuccess) e = hipMalloc((void **)&op->d_src_gp, sizeof(int) * gp.size());
    if (e == hipSuccess) e = hipMalloc((void **)&op->d_src_gw, sizeof(float) * gw.size());
    if (e == hipSuccess) e = hipMalloc((void **)&op->d_src_gd, sizeof(float) * gd.size());
    if (e != hipSuccess) return fail(FDW_ERR_NOMEM, "operator_create: injection gather: %s", hipGetErrorString(e));
    e = hipMemcpy(op->d_src_tgt, tgt.data(), sizeof(int64_t) * tgt.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(op->d_src_goff, goff.data(), sizeof(int) * goff.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(op->d_src_gp, gp.data(), sizeof(int) * gp.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(op->d_src_gw, gw.data(), sizeof(float) * gw.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(op->d_src_gd, gd.data(), sizeof(float) * gd.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "operator_create: injection gather upload");
    op->src_ntarget = (int)tgt.size();
    return FDW_OK;
}

static int check_func(const char *what, const fdw_func *f, const fdw_grid *g, int so) {
    if (!f) return fail(FDW_ERR_ARG, "operator_create: %s is required", what);
    if (f->grid != g) return fail(FDW_ERR_ARG, "operator_create: %s is bound on another grid", what);
    if (f->so != so)
        return fail(FDW_ERR_LAYOUT, "operator_create: %s bound at space order %d, operator uses %d", what, f->so, so);
    return FDW_OK;
}

static int check_tfunc(const char *what, const fdw_tfunc *f, const fdw_grid *g, int so) {
    if (!f) return fail(FDW_ERR_ARG, "operator_create: %s is required", what);
    if (f->grid != g) return fail(FDW_ERR_ARG, "operator_create: %s is bound on another grid", what);
    if (f->so != so)
        return fail(FDW_ERR_LAYOUT, "operator_create: %s bound at space order %d, operator uses %d", what, f->so, so);
    return FDW_OK;
}

static void pick_variants(fdw_op *op) {
    // FDW_KERNEL=naive forces the one-thread-per-point kernels (A/B checks).
    const char *k = std::getenv("FDW_KERNEL");
    const bool naive = k && std::strcmp(k, "naive") == 0;
    // the 3D streaming kernels address a z-chunk of the padded layout with
    // byte offsets below 2^31 from a descriptor based R + 2 planes below it:
    // grids whose chunk of one plane, 2R + 5 planes, reaches 2 GiB take the
    // per-point kernels (2D: fields above 2 GiB)
    const int64_t plane_bytes = op->lay.pitch_x * op->lay.pitch_y * (int64_t)sizeof(float);
    const bool big_plane = op->ndim == 3 ? (int64_t)(2 * op->R + 5) * plane_bytes >= ((int64_t)1 << 31)
                                         : plane_bytes > ((int64_t)1 << 31);
    op->iso_v = naive || big_plane ? IsoVariant::Naive : IsoVariant::Stream;
    op->tti_v = naive || big_plane ? TtiVariant::Naive : TtiVariant::Stream;
    // the persistent kernel handles linear (2 x 2) sparse supports only
    // (FDW_PERSIST2D=0 keeps small 2D grids on the per-step kernels: checks of that path)
    const char *p2 = std::getenv("FDW_PERSIST2D");
    const bool persist_off = p2 && p2[0] == '0';
    const bool linear = (!op->d.src || op->d.src->r == 2) && (!op->d.rec || op->d.rec->r == 2);
    op->use_persist2d = !naive && !persist_off && linear && op->d.kind == FDW_ISO && op->ndim == 2 &&
                        op->d.mode == FDW_FORWARD &&
                        (int64_t)op->geom.nx * op->geom.nz * (int64_t)sizeof(float) <= kPersist2DMaxLds;
}

extern "C" {

int fdw_operator_create(const fdw_op_desc *desc, fdw_op **out) {
    FDW_GUARD_BEGIN
    if (!desc || !out) return fail(FDW_ERR_ARG, "operator_create: NULL desc/out");
    const fdw_op_desc &d = *desc;
    if (d.kind != FDW_ISO && d.kind != FDW_TTI) return fail(FDW_ERR_ARG, "operator_create: unknown kind %d", d.kind);
    if (!valid_so(d.space_order))
        return fail(FDW_ERR_ARG, "operator_create: space_order %d not even in [2,16]", d.space_order);
    if (!d.u) return fail(FDW_ERR_ARG, "operator_create: wavefield u/p is required");
    fdw_grid *g = d.u->grid;
    const int so = d.space_order;
    int st = check_tfunc("u/p", d.u, g, so);
    if (!st) st = check_func("m", d.m, g, so);
    if (st) return st;
    if (d.kind == FDW_TTI) {
        if ((st = check_tfunc("r", d.r, g, so))) return st;
        if ((st = check_func("eps", d.eps, g, so))) return st;
        if ((st = check_func("delta", d.delta, g, so))) return st;
        if ((st = check_func("theta", d.theta, g, so))) return st;
        if (g->ndim == 3 && (st = check_func("phi", d.phi, g, so))) return st;
        if (d.r == d.u) return fail(FDW_ERR_ARG, "operator_create: p and r must be distinct TimeFunctions");
        if (d.r->nslots != d.u->nslots) return fail(FDW_ERR_ARG, "operator_create: p and r must use the same slot count");
    } else if (d.r) {
        return fail(FDW_ERR_ARG, "operator_create: r must be NULL for the isotropic operator");
    }
    if (d.src && d.src->grid != g) return fail(FDW_ERR_ARG, "operator_create: src bound on another grid");
    if (d.rec && d.rec->grid != g) return fail(FDW_ERR_ARG, "operator_create: rec bound on another grid");
    if (!(d.dt > 0.0) || !std::isfinite(d.dt)) return fail(FDW_ERR_ARG, "operator_create: dt must be positive");
    if (!(d.vmax > 0.0) || !std::isfinite(d.vmax)) return fail(FDW_ERR_ARG, "operator_create: vmax must be positive");
    if (d.nbl < 0) return fail(FDW_ERR_ARG, "operator_create: nbl must be >= 0");
    const double rc = d.damp_rc == 0.0 ? 1e-3 : d.damp_rc;
    if (!(rc > 0.0 && rc < 1.0)) return fail(FDW_ERR_ARG, "operator_create: damp_rc must be in (0, 1)");
    if (d.mode != FDW_FORWARD && d.mode != FDW_ADJOINT) return fail(FDW_ERR_ARG, "operator_create: unknown mode %d", d.mode);
    if (d.mode == FDW_ADJOINT && d.kind != FDW_ISO)
        return fail(FDW_ERR_ARG, "operator_create: the adjoint mode is available for the isotropic operator only");
    const double eps_max = d.kind == FDW_TTI ? d.eps_max : 0.0;
    if (!(eps_max >= 0.0)) return fail(FDW_ERR_ARG, "operator_create: eps_max must be >= 0");
    const double dtmax = stable_dt_axes(d.kind, g->ndim, so, d.vmax, eps_max, g->h);
    if (d.dt > dtmax)
        return fail(FDW_ERR_UNSTABLE, "operator_create: dt = %g exceeds the stability bound %g", d.dt, dtmax);

    fdw_op *op = new fdw_op();
    op->d = d;
    op->d.damp_rc = rc;
    op->ndim = g->ndim;
    op->R = so / 2;
    compute_layout(g, so, &op->lay);
    const fdw_layout &L = op->lay;
    Geom &G = op->geom;
    G.nx = (int)g->shape[0];
    if (g->ndim == 3) {
        G.ny = (int)g->shape[1];
        G.nz = (int)g->shape[2];
        G.sy = L.pitch_x;
        G.sz = L.pitch_x * L.pitch_y;
    } else {
        G.ny = 1;
        G.nz = (int)g->shape[1];
        G.sy = 0;
        G.sz = L.pitch_x;
    }
    G.off0 = L.origin_offset;
    op->dt2 = (float)(d.dt * d.dt);

    // FD coefficients (double, rounded once)
    double w1[kMaxR + 1], w2[kMaxR + 1];
    taylor_weights(op->R, w1, w2);
    std::memset(&op->coefs, 0, sizeof(op->coefs));
    const int axis_of[3] = {0, g->ndim == 3 ? 1 : 2, 2};  // grid axis -> coefficient slot
    double c0 = 0.0;
    for (int a = 0; a < g->ndim; ++a) {
        const int slot = axis_of[a];
        const double h = g->h[a];
        for (int k = 0; k <= op->R; ++k) {
            op->coefs.w2[slot][k] = (float)(w2[k] / (h * h));
            op->coefs.w1[slot][k] = (float)(w1[k] / h);
        }
        c0 += w2[0] / (h * h);
    }
    op->coefs.c0 = (float)c0;

    // damping tables eta_a(i) * dt / 2 (quadratic profile inside the layer)
    const int64_t nx = G.nx, ny = G.ny, nz = G.nz;
    std::vector<float> eta((size_t)(nx + ny + nz), 0.0f);
    auto fill_axis = [&](float *dst, int64_t n, double h) {
        for (int64_t i = 0; i < n; ++i) {
            double v = 0.0;
            if (d.nbl > 0) {
                const int64_t dist = std::max<int64_t>({(int64_t)d.nbl - i, i - (n - 1 - d.nbl), 0});
                const double emax = 3.0 * d.vmax * std::log(1.0 / rc) / (2.0 * d.nbl * h);
                const double r = (double)dist / (double)d.nbl;
                v = emax * r * r * d.dt / 2.0;
            }
            dst[i] = (float)v;
        }
    };
    fill_axis(eta.data(), nx, g->h[0]);
    if (g->ndim == 3) {
        fill_axis(eta.data() + nx, ny, g->h[1]);
        fill_axis(eta.data() + nx + ny, nz, g->h[2]);
    } else {
        fill_axis(eta.data() + nx + ny, nz, g->h[1]);  // the single y entry stays 0
    }
    hipError_t e = hipMalloc((void **)&op->d_eta, sizeof(float) * eta.size());
    if (e != hipSuccess) {
        release_device(op);
        delete op;
        return fail(FDW_ERR_NOMEM, "operator_create: hipMalloc damping: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(op->d_eta, eta.data(), sizeof(float) * eta.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release_device(op);
        delete op;
        return fail_hip(e, "operator_create: damping upload");
    }

    // sparse preprocessing: element offsets and float weights
    if (d.src) {
        st = upload_sparse(op, d.src, d.dt * d.dt, &op->d_src_base, &op->d_src_w, &op->d_src_idx);
        if (!st) st = build_inject_gather(op, d.src, d.dt * d.dt, eta);
        if (!st && d.src->npoint <= kMaxFusedSrc && d.src->r == 2) {
            op->src_fused = true;
            FusedSrc &F = op->fsrc_template;
            std::memset(&F, 0, sizeof(F));
            F.n = d.src->npoint;
            for (int s = 0; s < F.n; ++s) {
                const int64_t *b = &d.src->base[(size_t)s * g->ndim];
                F.bx[s] = (int)b[0];
                F.by[s] = g->ndim == 3 ? (int)b[1] : 0;
                F.bz[s] = (int)b[g->ndim - 1];
                for (int c = 0; c < (1 << g->ndim); ++c)
                    F.w[s][c] = (float)(d.dt * d.dt * d.src->w[(size_t)s * (1 << g->ndim) + c]);
            }
            // the temporal-blocking kernel reads the record from device memory
            e = hipMalloc((void **)&op->d_fsrc, sizeof(FusedSrc));
            if (e == hipSuccess) e = hipMemcpy(op->d_fsrc, &F, sizeof(FusedSrc), hipMemcpyHostToDevice);
            if (e != hipSuccess) st = fail(FDW_ERR_NOMEM, "operator_create: fused sources: %s", hipGetErrorString(e));
        }
    }
    if (!st && d.rec) st = upload_sparse(op, d.rec, 1.0, &op->d_rec_base, &op->d_rec_w, &op->d_rec_idx);
    if (st) {
        release_device(op);
        delete op;
        return st;
    }

    // TTI stage buffers (zero halo: g vanishes outside the domain)
    if (d.kind == FDW_TTI) {
        const size_t bytes = sizeof(float) * (size_t)L.elems_per_slot * 2;
        e = hipMalloc((void **)&op->d_stage, bytes);
        if (e == hipSuccess) e = hipMemset(op->d_stage, 0, bytes);
        if (e != hipSuccess) {
            release_device(op);
            delete op;
            return fail(FDW_ERR_NOMEM, "operator_create: TTI stage buffers: %s", hipGetErrorString(e));
        }
    }

    // zero the halo of every wavefield slot
    std::vector<fdw_tfunc *> tfs{d.u};
    if (d.kind == FDW_TTI) tfs.push_back(d.r);
    for (fdw_tfunc *tf : tfs)
        for (int sl = 0; sl < tf->nslots; ++sl) {
            e = launch_zero_halo(op->ndim, G, op->R, L.pitch_x, L.pitch_y, L.planes,
                                 tf->d + (int64_t)sl * L.elems_per_slot, nullptr);
            if (e != hipSuccess) break;
        }
    // the null stream only: work of the caller's other streams is not waited for
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e != hipSuccess) {
        release_device(op);
        delete op;
        return fail_hip(e, "operator_create: zero halo");
    }

    pick_variants(op);
    // 2D isotropic grids too large for the LDS-resident kernel can advance K
    // steps per launch on overlapped patches (opt-in, FDW_TB=1: on one MI355X
    // the per-step kernel, served from the Infinity Cache, is faster at the
    // sizes measured); in-place two-slot storage, fused (or no) sources,
    // linear receivers
    {
        const char *tb = std::getenv("FDW_TB");
        const bool off = !(tb && tb[0] == '1') || op->iso_v == IsoVariant::Naive;
        op->use_tb2d = !off && d.kind == FDW_ISO && op->ndim == 2 && d.mode == FDW_FORWARD && !op->use_persist2d &&
                       d.u->nslots == 2 && (!d.src || d.src->npoint == 0 || op->src_fused) &&
                       (!d.rec || d.rec->npoint == 0 || d.rec->r == 2) && tb2d_shape(op->R).k > 0;
        if (op->use_tb2d) {
            const size_t bytes = sizeof(float) * (size_t)L.elems_per_slot * 2;
            hipError_t e2 = hipMalloc((void **)&op->d_tb, bytes);
            if (e2 == hipSuccess) e2 = hipMemset(op->d_tb, 0, bytes);
            if (e2 != hipSuccess) {
                release_device(op);
                delete op;
                return fail(FDW_ERR_NOMEM, "operator_create: level buffers: %s", hipGetErrorString(e2));
            }
        }
    }
    // 3D isotropic grids advance two steps per launch (temporal blocking,
    // FDW_TB3D=1; 0 keeps one launch per step); in-place two-slot storage,
    // fused (or no) sources, linear (or no) receivers, fields below 2 GiB
    {
        const char *tb = std::getenv("FDW_TB3D");
        const bool on = tb && tb[0] == '1';
        const bool small_fields = (L.elems_per_slot * (int64_t)sizeof(float)) < ((int64_t)1 << 31);
        op->use_tb3d = on && d.kind == FDW_ISO && op->ndim == 3 && d.mode == FDW_FORWARD &&
                       op->iso_v == IsoVariant::Stream && small_fields && d.u->nslots == 2 &&
                       (!d.src || d.src->npoint == 0 || op->src_fused) && (!d.rec || d.rec->npoint == 0 || d.rec->r == 2);
        if (op->use_tb3d) {
            const size_t bytes = sizeof(float) * (size_t)L.elems_per_slot * 2;
            hipError_t e2 = hipMalloc((void **)&op->d_tb, bytes);
            if (e2 == hipSuccess) e2 = hipMemset(op->d_tb, 0, bytes);
            if (e2 != hipSuccess) {
                release_device(op);
                delete op;
                return fail(FDW_ERR_NOMEM, "operator_create: temporal-blocking buffers: %s", hipGetErrorString(e2));
            }
        }
    }
    // Receiver sampling of step t reads level t+1, which the stencil of step
    // t + S (S = slots) overwrites: it can run on a second stream, overlapped with
    // the next stencil launches, ordered by events (opt-in, FDW_OVERLAP_INTERP=1:
    // the cross-stream waits cost more than the overlap saves on one MI355X).
    {
        const char *ov = std::getenv("FDW_OVERLAP_INTERP");
        op->overlap_interp = op->ndim == 3 && d.rec && d.rec->npoint >= 1024 && ov && ov[0] == '1';
        if (op->overlap_interp) {
            const int ring = d.u->nslots + 1;
            hipError_t e2 = hipStreamCreateWithFlags(&op->side, hipStreamNonBlocking);
            for (int i = 0; e2 == hipSuccess && i < ring; ++i) {
                hipEvent_t a = nullptr, b = nullptr;
                e2 = hipEventCreateWithFlags(&a, hipEventDisableTiming);
                if (e2 == hipSuccess) e2 = hipEventCreateWithFlags(&b, hipEventDisableTiming);
                if (a) op->ev_step.push_back(a);
                if (b) op->ev_interp.push_back(b);
            }
            if (e2 != hipSuccess) {
                release_device(op);
                delete op;
                return fail_hip(e2, "operator_create: side stream");
            }
        }
    }
    // reference counts keep bound handles alive while the operator exists
    d.u->refs++;
    if (d.r) d.r->refs++;
    for (fdw_func *f : {d.m, d.eps, d.delta, d.theta, d.phi})
        if (f) f->refs++;
    if (d.src) d.src->refs++;
    if (d.rec) d.rec->refs++;
    *out = op;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_operator_destroy(fdw_op *op) {
    if (!op) return FDW_OK;
    const fdw_op_desc &d = op->d;
    d.u->refs--;
    if (d.r) d.r->refs--;
    for (fdw_func *f : {d.m, d.eps, d.delta, d.theta, d.phi})
        if (f) f->refs--;
    if (d.src) d.src->refs--;
    if (d.rec) d.rec->refs--;
    release_device(op);
    delete op;
    return FDW_OK;
}

// Injection / interpolation argument templates of an operator (field, row
// and sample pointers are filled per step).
static SparseArgs sparse_template(const fdw_op *op, const fdw_sparse *sp, bool rec) {
    const fdw_op_desc &d = op->d;
    SparseArgs a{};
    a.ndim = op->ndim;
    a.eta_x = op->d_eta;
    a.eta_y = op->d_eta + op->geom.nx;
    a.eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    a.npoint = sp ? sp->npoint : 0;
    a.r = sp ? sp->r : 2;
    a.ncorner = sp ? sp->ncorner : 1 << op->ndim;
    a.cstride[0] = 1;
    a.cstride[1] = op->ndim == 3 ? op->geom.sy : op->geom.sz;
    a.cstride[2] = op->ndim == 3 ? op->geom.sz : 0;
    if (rec) {
        a.damp_mode = d.mode == FDW_ADJOINT ? 2 : 0;
        a.idx = op->d_rec_idx;
        a.base = op->d_rec_base;
        a.w = op->d_rec_w;
        a.m = nullptr;
    } else {
        a.damp_mode = d.mode == FDW_ADJOINT ? 1 : 0;
        a.idx = op->d_src_idx;
        a.base = op->d_src_base;
        a.w = op->d_src_w;
        a.m = d.m->d;
        a.ntarget = op->src_ntarget;
        a.tgt = op->d_src_tgt;
        a.goff = op->d_src_goff;
        a.gp = op->d_src_gp;
        a.gw = op->d_src_gw;
        a.gd = op->d_src_gd;
    }
    return a;
}

// Does the operator sample its receivers inside its 3D streaming launches
// (extra workgroups reading the level the launch only reads)?
static bool samples_in_launch(const fdw_op *op) {
    const fdw_sparse *r = op->d.rec;
    return r && r->npoint > 0 && op->ndim == 3 && !op->overlap_interp && r->r == 2 &&
           (op->d.kind == FDW_ISO ? op->iso_v == IsoVariant::Stream : op->tti_v == TtiVariant::Stream);
}

// Stencil arguments of step t (level t + 1 from levels t and t - 1; level k
// in slot k mod nslots, so with two slots the new level overwrites t - 1).
static void iso_step_args(const fdw_op *op, int t, IsoArgs &a) {
    const fdw_op_desc &d = op->d;
    const int64_t E = op->lay.elems_per_slot;
    const int S = d.u->nslots;
    const int sc = t % S, sp = (t + S - 1) % S, sn = (t + 1) % S;
    a = IsoArgs{};
    a.g = op->geom;
    a.u_cur = d.u->d + sc * E;
    a.u_prev = d.u->d + sp * E;
    a.u_next = d.u->d + sn * E;
    a.m = d.m->d;
    a.eta_x = op->d_eta;
    a.eta_y = op->d_eta + op->geom.nx;
    a.eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    a.dt2 = op->dt2;
    a.c = op->coefs;
    if (op->src_fused && d.src && d.src->npoint > 0) {
        a.src = op->fsrc_template;
        a.src.q = d.src->data + (int64_t)t * d.src->npoint;
    }
    a.adjoint = d.mode == FDW_ADJOINT;
    a.save = nullptr;
    a.rec = nullptr;
    a.sampling = samples_in_launch(op) ? 1 : 0;
}

static void tti_step_args(const fdw_op *op, int t, TtiArgs &a, float *stage) {
    const fdw_op_desc &d = op->d;
    const int64_t E = op->lay.elems_per_slot;
    const int S = d.u->nslots;
    const int sc = t % S, sp = (t + S - 1) % S, sn = (t + 1) % S;
    a = TtiArgs{};
    a.g = op->geom;
    a.p_cur = d.u->d + sc * E;
    a.p_prev = d.u->d + sp * E;
    a.p_next = d.u->d + sn * E;
    a.r_cur = d.r->d + sc * E;
    a.r_prev = d.r->d + sp * E;
    a.r_next = d.r->d + sn * E;
    a.m = d.m->d;
    a.eps = d.eps->d;
    a.delta = d.delta->d;
    a.theta = d.theta->d;
    a.phi = d.phi ? d.phi->d : nullptr;
    a.gp = stage;
    a.gr = stage + E;
    a.eta_x = op->d_eta;
    a.eta_y = op->d_eta + op->geom.nx;
    a.eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    a.dt2 = op->dt2;
    a.c = op->coefs;
    if (op->src_fused && d.src && d.src->npoint > 0) {
        a.src = op->fsrc_template;
        a.src.q = d.src->data + (int64_t)t * d.src->npoint;
    }
    a.rec = nullptr;
}

// Arguments of the LDS-resident 2D isotropic kernel for one apply range.
static void persist2d_args(const fdw_op *op, int time_m, int time_M, Persist2DArgs &pa) {
    const fdw_op_desc &d = op->d;
    const int nsrc = d.src ? d.src->npoint : 0;
    const int nrec = d.rec ? d.rec->npoint : 0;
    pa = Persist2DArgs{};
    pa.g = op->geom;
    pa.u = d.u->d;
    pa.slot = op->lay.elems_per_slot;
    pa.nslots = d.u->nslots;
    pa.pitch_x = op->lay.pitch_x;
    pa.m = d.m->d;
    pa.eta_x = op->d_eta;
    pa.eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    pa.dt2 = op->dt2;
    pa.c = op->coefs;
    pa.time_m = time_m;
    pa.time_M = time_M;
    pa.nsrc = nsrc;
    pa.src_base = op->d_src_base;
    pa.src_w = op->d_src_w;
    pa.src_data = nsrc > 0 ? d.src->data : nullptr;
    pa.nrec = nrec;
    pa.rec_base = op->d_rec_base;
    pa.rec_w = op->d_rec_w;
    pa.rec_data = nrec > 0 ? d.rec->data : nullptr;
}

static int timing_event_pair(fdw_op *op, hipEvent_t *a, hipEvent_t *b) {
    while (op->ev_used + 2 > op->ev_pool.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return fail_hip(err, "timing: hipEventCreate");
        op->ev_pool.push_back(e);
    }
    *a = op->ev_pool[op->ev_used];
    *b = op->ev_pool[op->ev_used + 1];
    op->ev_used += 2;
    return FDW_OK;
}

// Events of the next stencil launch: runs of timing_every consecutive
// launches, the first carrying the start event and the last the stop event.
static int timing_next(fdw_op *op, LaunchEvents &ev) {
    if (!op->timing) return FDW_OK;
    if (!op->run_open) {
        int st = timing_event_pair(op, &op->run_start, &op->run_stop);
        if (st) return st;
        ev.start = op->run_start;
        op->run_open = true;
        op->run_len = 0;
    }
    if (++op->run_len == op->timing_every) {
        ev.stop = op->run_stop;
        op->run_open = false;
        op->acc_launches += op->run_len;
    }
    return FDW_OK;
}

// an apply that ends inside a run closes it after its last launch
static int timing_close(fdw_op *op, hipStream_t s) {
    if (!op->timing || !op->run_open) return FDW_OK;
    hipError_t e = hipEventRecord(op->run_stop, s);
    if (e != hipSuccess) return fail_hip(e, "operator_apply: timing event");
    op->run_open = false;
    op->acc_launches += op->run_len;
    return FDW_OK;
}

// Imaging condition along an adjoint apply: the factor of forward step t at
// s + (t - first) E, paired with adjoint level T - t, accumulated into grad.
struct ImageRun {
    const float *s;
    int first, T;
    float *grad;
};

// The apply loop.  stage: the TTI gradient buffers (gp | gr, elems_per_slot
// each); timed: the operator's kernel timing (which creates events) applies.
static int apply_impl(fdw_op *op, int time_m, int time_M, void *stream, float *stage, bool timed,
                      const ImageRun *img = nullptr) {
    if (!op) return fail(FDW_ERR_ARG, "operator_apply: NULL op");
    const fdw_op_desc &d = op->d;
    hipStream_t s = (hipStream_t)stream;
    if (time_M == -1) {
        int lim = -1;
        if (d.src && d.src->npoint > 0) lim = d.src->nt;
        if (d.rec && d.rec->npoint > 0) lim = lim < 0 ? d.rec->nt : std::min(lim, d.rec->nt);
        if (lim < 0) return fail(FDW_ERR_ARG, "operator_apply: time_M = -1 needs a source or receiver time axis");
        time_M = lim - 1;
    }
    if (time_m < 0 || time_M < time_m - 1)
        return fail(FDW_ERR_ARG, "operator_apply: invalid range time_m = %d, time_M = %d", time_m, time_M);
    if (d.src && d.src->npoint > 0 && time_M >= d.src->nt)
        return fail(FDW_ERR_ARG, "operator_apply: time_M = %d beyond the %d source samples", time_M, d.src->nt);
    if (d.rec && d.rec->npoint > 0 && time_M >= d.rec->nt)
        return fail(FDW_ERR_ARG, "operator_apply: time_M = %d beyond the %d receiver samples", time_M, d.rec->nt);
    const fdw_layout &L = op->lay;
    const int64_t E = L.elems_per_slot;
    const float *eta_x = op->d_eta, *eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    const int nsrc = d.src ? d.src->npoint : 0;
    const int nrec = d.rec ? d.rec->npoint : 0;
    timed = timed && op->timing;
    if (timed) op->last_stream = s;

    SparseArgs inj = sparse_template(op, d.src, false);
    SparseArgs itp = sparse_template(op, d.rec, true);

    // small 2D isotropic grids: the whole range in one persistent launch
    if (d.kind == FDW_ISO && op->ndim == 2 && op->use_persist2d && !op->save_buf && !op->isave_buf &&
        time_M >= time_m) {
        Persist2DArgs pa;
        persist2d_args(op, time_m, time_M, pa);
        LaunchEvents ev;
        int st = (timed ? timing_next(op, ev) : FDW_OK);
        if (st) return st;
        hipError_t e = launch_iso2d_persistent(op->R, pa, s, ev);
        if (e != hipSuccess) return fail_hip(e, "operator_apply: persistent 2D launch");
        return timed ? timing_close(op, s) : FDW_OK;
    }
    // 2D temporal blocking: passes of up to K steps, each reading its two input
    // levels from one pair of buffers and writing its two output levels to the
    // other; the pass count fixes which pair the first pass reads so that the
    // last pass writes the TimeFunction's slots (level k in slot k mod 2)
    if (op->use_tb2d && !op->save_buf && !op->isave_buf && time_M >= time_m) {
        const TB2DShape sh = tb2d_shape(op->R);
        const int N = time_M - time_m + 1, P = (N + sh.k - 1) / sh.k;
        float *tfb = d.u->d, *scb = op->d_tb;
        float *X = tfb, *Y = scb;
        if (P % 2 == 1) {
            hipError_t e = hipMemcpyAsync(scb, tfb, sizeof(float) * 2 * (size_t)E, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail_hip(e, "operator_apply: level copy");
            X = scb;
            Y = tfb;
        }
        for (int t0 = time_m; t0 <= time_M; t0 += sh.k) {
            const int n = std::min(sh.k, time_M - t0 + 1);
            TB2DArgs a{};
            a.g = op->geom;
            a.in_prev = X + (int64_t)((t0 + 1) % 2) * E;  // level t0 - 1
            a.in_cur = X + (int64_t)(t0 % 2) * E;
            a.out_prev = Y + (int64_t)((t0 + n + 1) % 2) * E;  // level t0 + n - 1
            a.out_cur = Y + (int64_t)((t0 + n) % 2) * E;
            a.m = d.m->d;
            a.eta_x = eta_x;
            a.eta_z = eta_z;
            a.dt2 = op->dt2;
            a.c = op->coefs;
            if (op->src_fused && nsrc > 0) {
                a.src = op->fsrc_template;
                a.src.q = d.src->data + (int64_t)t0 * nsrc;
                a.src_stride = nsrc;
            }
            a.nsteps = n;
            a.nrec = nrec;
            if (nrec > 0) {
                a.rec_idx = op->d_rec_idx;
                a.rec_w = op->d_rec_w;
                a.rec_rows = d.rec->data + (int64_t)t0 * nrec;
            }
            LaunchEvents ev;
            if (int st = (timed ? timing_next(op, ev) : FDW_OK)) return st;
            hipError_t e = launch_iso2d_tb(op->R, a, s, ev);
            if (e != hipSuccess) return fail_hip(e, "operator_apply: temporal-blocking launch");
            std::swap(X, Y);
        }
        return timed ? timing_close(op, s) : FDW_OK;
    }
    // 3D temporal blocking: pairs of steps, each pass reading levels t - 1, t
    // from one buffer pair and writing t + 1, t + 2 to the other, the pass
    // count fixing which pair the first pass reads so that the last writes
    // the TimeFunction's slots; receivers of a pass are sampled inside the
    // next pass, those of the last pass by their own launches; an odd last
    // step runs the per-step kernel below
    if (op->use_tb3d && !op->save_buf && !op->isave_buf && time_M - time_m + 1 >= 2) {
        const int P = (time_M - time_m + 1) / 2;
        float *A = d.u->d, *B = op->d_tb;
        if (P % 2 == 1) {
            hipError_t e = hipMemcpyAsync(op->d_tb, d.u->d, sizeof(float) * 2 * (size_t)E, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail_hip(e, "operator_apply: level copy");
            std::swap(A, B);
        }
        for (int k = 0; k < P; ++k) {
            const int t = time_m + 2 * k;
            TB3DArgs a{};
            a.f.g = op->geom;
            a.f.in_prev = A + (int64_t)((t + 1) % 2) * E;  // level t - 1
            a.f.in_cur = A + (int64_t)(t % 2) * E;
            a.f.out_prev = B + (int64_t)((t + 1) % 2) * E;  // level t + 1
            a.f.out_cur = B + (int64_t)(t % 2) * E;         // level t + 2
            a.f.m = d.m->d;
            a.f.eta_x = op->d_eta;
            a.f.eta_y = op->d_eta + op->geom.nx;
            a.f.eta_z = eta_z;
            a.f.dt2 = op->dt2;
            a.c = op->coefs;
            a.fsrc = op->src_fused && nsrc > 0 ? op->d_fsrc : nullptr;
            if (nsrc > 0) {
                a.q1 = d.src->data + (int64_t)t * nsrc;
                a.q2 = d.src->data + (int64_t)(t + 1) * nsrc;
            }
            if (nrec > 0 && t > time_m) {  // rows t - 2, t - 1 from levels t - 1, t
                a.rec[0] = itp;
                a.rec[0].field = const_cast<float *>(a.f.in_prev);
                a.rec[0].rec_row = d.rec->data + (int64_t)(t - 2) * nrec;
                a.rec[1] = itp;
                a.rec[1].field = const_cast<float *>(a.f.in_cur);
                a.rec[1].rec_row = d.rec->data + (int64_t)(t - 1) * nrec;
            }
            LaunchEvents ev;
            if (int st = (timed ? timing_next(op, ev) : FDW_OK)) return st;
            hipError_t e = launch_iso3d_tb2(op->R, a, s, ev);
            if (e != hipSuccess) return fail_hip(e, "operator_apply: temporal-blocking launch");
            std::swap(A, B);
        }
        const int tl = time_m + 2 * P - 2;  // the last pass computed levels tl + 1, tl + 2
        if (nrec > 0) {
            for (int r = 0; r < 2; ++r) {
                itp.field = d.u->d + (int64_t)((tl + 1 + r) % 2) * E;
                itp.rec_row = d.rec->data + (int64_t)(tl + r) * nrec;
                hipError_t e = launch_interp(itp, s);
                if (e != hipSuccess) return fail_hip(e, "operator_apply: interp launch");
            }
        }
        time_m += 2 * P;
        if (time_m > time_M) return timed ? timing_close(op, s) : FDW_OK;
    }
    const int S_ring = d.u->nslots + 1;
    // the 3D streaming kernels sample the receivers of step t - 1 inside the
    // launch of step t (extra workgroups reading level t); the last step of the
    // apply is sampled by its own launch after the loop
    const bool fuse_interp = nrec > 0 && op->ndim == 3 && !op->overlap_interp && interp_linear(itp) &&
                             (d.kind == FDW_ISO ? op->iso_v == IsoVariant::Stream : op->tti_v == TtiVariant::Stream);
    // saved level k occupies `fields` slots of the buffer (isotropic: u;
    // TTI: p then r)
    const int fields = d.kind == FDW_TTI ? 2 : 1;
    // the 3D streaming kernels store a step's imaging factor, and image the
    // centre level of an adjoint step, themselves (the factor needs the final
    // new level: fused sources only); elsewhere standalone kernels follow the
    // step
    const bool stream3d = op->ndim == 3 && d.kind == FDW_ISO && op->iso_v == IsoVariant::Stream;
    const bool fuse_isave = stream3d && (op->src_fused || nsrc == 0);
    const float inv_dt2 = (float)(1.0 / (d.dt * d.dt));
    auto image_args = [&]() {
        ImageArgs ia{};
        ia.g = op->geom;
        ia.eta_x = op->d_eta;
        ia.eta_y = op->d_eta + op->geom.nx;
        ia.eta_z = eta_z;
        ia.inv_dt2 = inv_dt2;
        return ia;
    };
    // the initial level 0 is no step's output: an apply from time 0 stores it
    if (op->save_buf && time_m == 0 && time_M >= time_m && op->save_first <= 0 && op->save_first % op->save_every == 0 &&
        -op->save_first / op->save_every < op->save_nlevels) {
        float *dst = op->save_buf + (int64_t)(-op->save_first / op->save_every) * fields * E;
        hipError_t e = hipMemcpyAsync(dst, d.u->d, sizeof(float) * (size_t)E, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess && d.kind == FDW_TTI)
            e = hipMemcpyAsync(dst + E, d.r->d, sizeof(float) * (size_t)E, hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) return fail_hip(e, "operator_apply: save copy of level 0");
    }
    for (int t = time_m; t <= time_M; ++t) {
        // the stencil of step t overwrites the slot of level t + 1 - S, which
        // the (overlapped) receiver sampling of step t - S reads
        if (op->overlap_interp && nrec > 0 && t - d.u->nslots >= time_m) {
            hipError_t er = hipStreamWaitEvent(s, op->ev_interp[(t - d.u->nslots) % S_ring], 0);
            if (er != hipSuccess) return fail_hip(er, "operator_apply: hipStreamWaitEvent");
        }
        const int sn = (t + 1) % d.u->nslots;
        LaunchEvents ev;
        if (int st = (timed ? timing_next(op, ev) : FDW_OK)) return st;
        hipError_t e;
        float *next_field;
        const float *cur_field = nullptr, *prev_field = nullptr;
        float *save_dst = nullptr;
        float *isave_dst = nullptr;
        if (op->isave_buf && t >= op->isave_first && t - op->isave_first < op->isave_n)
            isave_dst = op->isave_buf + (int64_t)(t - op->isave_first) * E;
        {
            const int L = t + 1;
            if (op->save_buf && L >= op->save_first && (L - op->save_first) % op->save_every == 0 &&
                (L - op->save_first) / op->save_every < op->save_nlevels)
                save_dst = op->save_buf + (int64_t)((L - op->save_first) / op->save_every) * fields * E;
        }
        if (d.kind == FDW_ISO) {
            IsoArgs a;
            iso_step_args(op, t, a);
            SparseArgs prev_itp = itp;
            a.rec = nullptr;
            if (fuse_interp && t > time_m) {
                prev_itp.field = const_cast<float *>(a.u_cur);  // level t, read-only in this launch
                prev_itp.rec_row = d.rec->data + (int64_t)(t - 1) * nrec;
                a.rec = &prev_itp;
            }
            if (save_dst && (op->src_fused || nsrc == 0)) a.save = save_dst;
            if (isave_dst && fuse_isave) a.isave = isave_dst;
            if (img && stream3d && t > time_m) {  // centre level t pairs with forward step T - t
                a.img_s = img->s + (int64_t)(img->T - t - img->first) * E;
                a.grad = img->grad;
                a.inv_dt2 = inv_dt2;
            }
            e = launch_iso(op->ndim, op->R, op->iso_v, a, s, ev);
            next_field = a.u_next;
            cur_field = a.u_cur;
            prev_field = a.u_prev;
        } else {
            TtiArgs a;
            tti_step_args(op, t, a, stage);
            SparseArgs prev_itp = itp;
            a.rec = nullptr;
            if (fuse_interp && t > time_m) {
                prev_itp.field = const_cast<float *>(a.p_cur);  // level t, read-only in this launch
                prev_itp.rec_row = d.rec->data + (int64_t)(t - 1) * nrec;
                a.rec = &prev_itp;
            }
            if (save_dst && (op->src_fused || nsrc == 0)) {
                a.save_p = save_dst;
                a.save_r = save_dst + E;
            }
            e = launch_tti(op->ndim, op->R, op->tti_v, a, s, ev);
            next_field = a.p_next;
        }
        if (e != hipSuccess) return fail_hip(e, "operator_apply: stencil launch");
        if (nsrc > 0 && !op->src_fused) {
            inj.q_row = d.src->data + (int64_t)t * nsrc;
            inj.field = next_field;
            if ((e = launch_inject(inj, s)) != hipSuccess) return fail_hip(e, "operator_apply: inject launch");
            if (d.kind == FDW_TTI) {
                inj.field = d.r->d + sn * E;
                if ((e = launch_inject(inj, s)) != hipSuccess) return fail_hip(e, "operator_apply: inject launch");
            }
        }
        if (save_dst && !(op->src_fused || nsrc == 0)) {
            e = hipMemcpyAsync(save_dst, next_field, sizeof(float) * (size_t)E, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess && d.kind == FDW_TTI)
                e = hipMemcpyAsync(save_dst + E, d.r->d + sn * E, sizeof(float) * (size_t)E, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return fail_hip(e, "operator_apply: save copy");
        }
        if (isave_dst && !fuse_isave) {
            ImageArgs ia = image_args();
            ia.u_next = next_field;
            ia.u_cur = cur_field;
            ia.u_prev = prev_field;
            ia.s_out = isave_dst;
            if ((e = launch_imaging_factor(op->ndim, ia, s)) != hipSuccess)
                return fail_hip(e, "operator_apply: imaging factor launch");
        }
        // imaging of the new level: here for the steps that do not fuse it,
        // after the last step for those that do
        if (img && (!stream3d || t == time_M)) {
            ImageArgs ia = image_args();
            ia.nu = next_field;
            ia.s_in = img->s + (int64_t)(img->T - 1 - t - img->first) * E;
            ia.grad = img->grad;
            if ((e = launch_image_update(op->ndim, ia, s)) != hipSuccess)
                return fail_hip(e, "gradient_apply: imaging launch");
        }
        if (nrec > 0 && (!fuse_interp || t == time_M)) {
            itp.field = next_field;
            itp.rec_row = d.rec->data + (int64_t)t * nrec;
            if (op->overlap_interp) {
                hipEvent_t es = op->ev_step[t % S_ring], ei = op->ev_interp[t % S_ring];
                hipError_t er = hipEventRecord(es, s);
                if (er == hipSuccess) er = hipStreamWaitEvent(op->side, es, 0);
                if (er != hipSuccess) return fail_hip(er, "operator_apply: side-stream ordering");
                if ((e = launch_interp(itp, op->side)) != hipSuccess) return fail_hip(e, "operator_apply: interp launch");
                if ((er = hipEventRecord(ei, op->side)) != hipSuccess) return fail_hip(er, "operator_apply: hipEventRecord");
            } else if ((e = launch_interp(itp, s)) != hipSuccess) {
                return fail_hip(e, "operator_apply: interp launch");
            }
        }
    }
    if (int st = timed ? timing_close(op, s) : FDW_OK) return st;
    // the caller's stream covers every receiver sample of this apply
    if (op->overlap_interp && nrec > 0 && time_M >= time_m) {
        const int last = std::max(time_m, time_M - d.u->nslots + 1);
        for (int t = last; t <= time_M; ++t) {
            hipError_t er = hipStreamWaitEvent(s, op->ev_interp[t % S_ring], 0);
            if (er != hipSuccess) return fail_hip(er, "operator_apply: hipStreamWaitEvent");
        }
    }
    return FDW_OK;
}


// The launch sequence of an apply depends only on its range and the
// operator's settings (every buffer is bound at creation, and the kernels read
// the data, sources included, at run time).  An apply whose range and settings
// repeat those of the previous call is captured into a hipGraph on a private
// stream and instantiated; the next calls with that key replay it, ordered
// after the caller's stream and before its later work by two events.  Not
// with kernel timing on (events around launches), receiver sampling on a
// second stream, or FDW_APPLY_GRAPH=0.
static int apply_graphed(fdw_op *op, int time_m, int time_M, hipStream_t s) {
    const std::vector<int64_t> key = {time_m,
                                      time_M,
                                      (int64_t)(intptr_t)op->save_buf,
                                      op->save_nlevels,
                                      op->save_every,
                                      op->save_first,
                                      (int64_t)(intptr_t)op->isave_buf,
                                      op->isave_n,
                                      op->isave_first};
    if (!(op->graph_exec && key == op->graph_key)) {
        if (key != op->graph_seen) {  // first time: launch directly
            op->graph_seen = key;
            return apply_impl(op, time_m, time_M, s, op->d_stage, false);
        }
        drop_apply_graph(op);
        hipError_t e = hipSuccess;
        if (!op->graph_stream) e = hipStreamCreateWithFlags(&op->graph_stream, hipStreamNonBlocking);
        for (hipEvent_t &ev : op->graph_ev)
            if (e == hipSuccess && !ev) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return fail_hip(e, "operator_apply: graph stream");
        e = hipStreamBeginCapture(op->graph_stream, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail_hip(e, "operator_apply: hipStreamBeginCapture");
        const int st = apply_impl(op, time_m, time_M, op->graph_stream, op->d_stage, false);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(op->graph_stream, &g);
        if (st != FDW_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return st != FDW_OK ? st : fail_hip(e, "operator_apply: graph capture");
        }
        e = hipGraphInstantiate(&op->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            op->graph_exec = nullptr;
            return fail_hip(e, "operator_apply: hipGraphInstantiate");
        }
        op->graph = g;
        op->graph_key = key;
        op->graph_builds++;
    }
    hipError_t e = hipEventRecord(op->graph_ev[0], s);
    if (e == hipSuccess) e = hipStreamWaitEvent(op->graph_stream, op->graph_ev[0], 0);
    if (e == hipSuccess) e = hipGraphLaunch(op->graph_exec, op->graph_stream);
    if (e == hipSuccess) e = hipEventRecord(op->graph_ev[1], op->graph_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, op->graph_ev[1], 0);
    if (e != hipSuccess) return fail_hip(e, "operator_apply: graph replay");
    op->graph_replays++;
    return FDW_OK;
}

int fdw_operator_apply(fdw_op *op, int time_m, int time_M, void *stream) {
    FDW_GUARD_BEGIN
    if (!op) return fail(FDW_ERR_ARG, "operator_apply: NULL op");
    static const bool graphs = [] {
        const char *e = std::getenv("FDW_APPLY_GRAPH");
        return !(e && e[0] == '0');
    }();
    if (graphs && !op->timing && !op->overlap_interp && time_m >= 0 && time_M >= time_m)
        return apply_graphed(op, time_m, time_M, (hipStream_t)stream);
    return apply_impl(op, time_m, time_M, stream, op->d_stage, true);
    FDW_GUARD_END
}

int fdw_operator_graph_stats(const fdw_op *op, int64_t *builds, int64_t *replays) {
    if (!op) return fail(FDW_ERR_ARG, "graph_stats: NULL op");
    if (builds) *builds = op->graph_builds;
    if (replays) *replays = op->graph_replays;
    return FDW_OK;
}

int fdw_operator_set_save(fdw_op *op, float *buf, int64_t nlevels, int every, int first_level) {
    if (!op) return fail(FDW_ERR_ARG, "set_save: NULL op");
    if (buf && (every < 1 || nlevels < 0)) return fail(FDW_ERR_ARG, "set_save: every must be >= 1 and nlevels >= 0");
    op->save_buf = buf;
    op->save_nlevels = buf ? nlevels : 0;
    op->save_every = buf ? every : 1;
    op->save_first = buf ? first_level : 0;
    return FDW_OK;
}

int fdw_operator_set_imaging_save(fdw_op *op, float *buf, int64_t nsteps, int first_step) {
    FDW_GUARD_BEGIN
    if (!op) return fail(FDW_ERR_ARG, "set_imaging_save: NULL op");
    if (!buf) {
        op->isave_buf = nullptr;
        op->isave_n = 0;
        op->isave_first = 0;
        return FDW_OK;
    }
    if (op->d.kind != FDW_ISO || op->d.mode != FDW_FORWARD)
        return fail(FDW_ERR_ARG, "set_imaging_save: isotropic forward operators only");
    if (op->d.u->nslots < 3)
        return fail(FDW_ERR_ARG, "set_imaging_save: the wavefield needs three time slots (has %d)", op->d.u->nslots);
    if (nsteps < 1 || first_step < 0)
        return fail(FDW_ERR_ARG, "set_imaging_save: nsteps must be >= 1 and first_step >= 0");
    op->isave_buf = buf;
    op->isave_n = nsteps;
    op->isave_first = first_step;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_gradient_apply(fdw_op *adj, int time_m, int time_M, int nt, const float *imaging, int first_step,
                       int64_t nsteps, float *grad, void *stream) {
    FDW_GUARD_BEGIN
    if (!adj || !imaging || !grad) return fail(FDW_ERR_ARG, "gradient_apply: NULL argument");
    if (adj->d.kind != FDW_ISO || adj->d.mode != FDW_ADJOINT)
        return fail(FDW_ERR_ARG, "gradient_apply: isotropic adjoint operators only");
    if (time_m < 0 || time_M >= nt || nt < 1)
        return fail(FDW_ERR_ARG, "gradient_apply: steps %d .. %d outside 0 .. nt - 1 = %d", time_m, time_M, nt - 1);
    if (time_M < time_m) return FDW_OK;
    // adjoint step tau pairs its new level with forward step nt - 1 - tau
    if (nt - 1 - time_M < first_step || nt - 1 - time_m >= first_step + nsteps)
        return fail(FDW_ERR_ARG,
                    "gradient_apply: forward steps %d .. %d not all among the %lld imaging factors from step %d",
                    nt - 1 - time_M, nt - 1 - time_m, (long long)nsteps, first_step);
    const ImageRun run{imaging, first_step, nt, grad};
    return apply_impl(adj, time_m, time_M, stream, adj->d_stage, true, &run);
    FDW_GUARD_END
}

int fdw_gradient_accumulate(fdw_op *op, const float *nu, const float *u_next, const float *u_cur,
                            const float *u_prev, float *grad, void *stream) {
    if (!op || !nu || !u_next || !u_cur || !u_prev || !grad) return fail(FDW_ERR_ARG, "gradient_accumulate: NULL argument");
    if (op->d.kind != FDW_ISO) return fail(FDW_ERR_ARG, "gradient_accumulate: isotropic operators only");
    GradArgs a{};
    a.g = op->geom;
    a.nu = nu;
    a.u_next = u_next;
    a.u_cur = u_cur;
    a.u_prev = u_prev;
    a.grad = grad;
    a.eta_x = op->d_eta;
    a.eta_y = op->d_eta + op->geom.nx;
    a.eta_z = op->d_eta + op->geom.nx + op->geom.ny;
    a.inv_dt2 = (float)(1.0 / (op->d.dt * op->d.dt));
    hipError_t e = launch_gradient(op->ndim, a, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "gradient_accumulate: launch");
    return FDW_OK;
}

int fdw_bandwidth_probe(int kind, float *dst, const float *a, const float *b, float s, int64_t n, void *stream) {
    if (!dst || !a || (kind == 1 && !b)) return fail(FDW_ERR_ARG, "bandwidth_probe: NULL buffer");
    if (kind != 0 && kind != 1) return fail(FDW_ERR_ARG, "bandwidth_probe: kind must be 0 (copy) or 1 (triad)");
    if (n < 0 || n % 4 != 0) return fail(FDW_ERR_ARG, "bandwidth_probe: n = %lld is not a multiple of 4", (long long)n);
    if (((uintptr_t)dst | (uintptr_t)a | (uintptr_t)b) % 16 != 0)
        return fail(FDW_ERR_ARG, "bandwidth_probe: buffers must be 16-byte aligned");
    hipError_t e = launch_bandwidth_probe(kind, dst, a, b, s, n, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "bandwidth_probe: launch");
    return FDW_OK;
}

int fdw_sync(fdw_op *op) {
    if (!op) return fail(FDW_ERR_ARG, "sync: NULL op");
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail_hip(e, "sync");
    return FDW_OK;
}

int fdw_operator_set_timing(fdw_op *op, int enable) {
    if (!op) return fail(FDW_ERR_ARG, "set_timing: NULL op");
    if (enable < 0) return fail(FDW_ERR_ARG, "set_timing: negative sampling interval %d", enable);
    op->timing = enable != 0;
    op->timing_every = enable > 0 ? enable : 1;
    op->run_open = false;
    op->run_len = 0;
    op->ev_used = 0;
    op->acc_ms = 0.0;
    op->acc_launches = 0;
    return FDW_OK;
}

int fdw_operator_kernel_time(fdw_op *op, double *total_ms, int64_t *launches, int reset) {
    if (!op || !total_ms || !launches) return fail(FDW_ERR_ARG, "kernel_time: NULL argument");
    double sum = op->acc_ms;
    for (size_t i = 0; i + 1 < op->ev_used; i += 2) {
        hipError_t e = hipEventSynchronize(op->ev_pool[i + 1]);
        if (e != hipSuccess) return fail_hip(e, "kernel_time: hipEventSynchronize");
        float ms = 0.0f;
        e = hipEventElapsedTime(&ms, op->ev_pool[i], op->ev_pool[i + 1]);
        if (e != hipSuccess) return fail_hip(e, "kernel_time: hipEventElapsedTime");
        sum += ms;
    }
    // fold the measured pairs so the pool can be reused
    op->acc_ms = sum;
    op->ev_used = 0;
    *total_ms = sum;
    *launches = op->acc_launches;
    if (reset) {
        op->acc_ms = 0.0;
        op->acc_launches = 0;
    }
    return FDW_OK;
}

int fdw_operator_describe(const fdw_op *op, char *buf, int buflen, double *alg_bytes_per_point) {
    if (!op || !buf || buflen <= 0) return fail(FDW_ERR_ARG, "describe: NULL argument");
    const bool iso = op->d.kind == FDW_ISO;
    char tbname[96];
    if (op->use_tb2d) {
        const TB2DShape sh = tb2d_shape(op->R);
        snprintf(tbname, sizeof(tbname), "iso2d_tb (temporal blocking, %d steps per launch, tile %dx%d)", sh.k, sh.ix,
                 sh.iz);
    }
    const char *name = iso ? (op->use_persist2d ? "iso2d_persistent (LDS-resident, one launch per apply)"
                              : op->use_tb2d    ? tbname
                              : op->use_tb3d    ? tb3d_kernel_name(op->geom, op->R)
                                                : iso_kernel_name(op->ndim, op->R, op->iso_v, op->geom,
                                                                  samples_in_launch(op)))
                           : tti_kernel_name(op->ndim, op->R, op->tti_v, op->geom);
    snprintf(buf, (size_t)buflen, "%s so=%d R=%d ndim=%d src=%s nsrc=%d nrec=%d", name, op->d.space_order, op->R,
             op->ndim, op->src_fused ? "fused" : "kernel", op->d.src ? op->d.src->npoint : 0,
             op->d.rec ? op->d.rec->npoint : 0);
    // algorithmic HBM bytes per point per step: iso reads u^n, u^n-1, m and
    // writes u^n+1; TTI reads p, r at two levels and m, eps, delta, theta(, phi)
    // and writes p, r.
    // A temporal-blocking launch does two steps' work: 32 B per point.
    if (alg_bytes_per_point)
        *alg_bytes_per_point = iso ? (op->use_tb3d ? 32.0 : 16.0) : (op->ndim == 3 ? 44.0 : 40.0);
    return FDW_OK;
}

}  // extern "C"

int64_t fdw::operator_stage_floats(const fdw_op *op) {
    return op && op->d.kind == FDW_TTI ? 2 * op->lay.elems_per_slot : 0;
}

int fdw::operator_apply_stage(fdw_op *op, int time_m, int time_M, void *stream, float *stage) {
    FDW_GUARD_BEGIN
    if (!op) return fail(FDW_ERR_ARG, "operator_apply: NULL op");
    return apply_impl(op, time_m, time_M, stream, stage, false);
    FDW_GUARD_END
}

// ---------------------------------------------------------------------------
// Fused multi-shot steps: several operators of one geometry advance together,
// one launch per stage and step for all of them (shot index as a grid
// dimension).  Per-shot, per-step records are packed on the host into a pinned
// buffer, copied to the device once per call, and the launch sequence of a
// call is captured once in a hipGraph and replayed while the shot count,
// step count and receiver width stay the same.
// ---------------------------------------------------------------------------
struct fdw_batch {
    char *h_stage = nullptr;  // pinned host records
    char *d_stage = nullptr;  // device records
    size_t cap = 0;
    hipEvent_t ev_copy = nullptr;
    bool copy_pending = false;
    // cached graph of the last launch sequence
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<int64_t> key;
    hipStream_t graph_stream = nullptr;
    int64_t graph_replays = 0, graph_builds = 0;
};

static void batch_drop_graph(fdw_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->key.clear();
}

static size_t align256(size_t n) { return (n + 255) / 256 * 256; }

extern "C" {

int fdw_batch_create(fdw_batch **out) {
    FDW_GUARD_BEGIN
    if (!out) return fail(FDW_ERR_ARG, "batch_create: NULL out");
    fdw_batch *b = new fdw_batch();
    hipError_t e = hipEventCreateWithFlags(&b->ev_copy, hipEventDisableTiming);
    if (e != hipSuccess) {
        delete b;
        return fail_hip(e, "batch_create: hipEventCreate");
    }
    *out = b;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_batch_destroy(fdw_batch *b) {
    if (!b) return FDW_OK;
    if (b->copy_pending) (void)hipEventSynchronize(b->ev_copy);
    batch_drop_graph(b);
    if (b->h_stage) (void)hipHostFree(b->h_stage);
    if (b->d_stage) (void)hipFree(b->d_stage);
    if (b->ev_copy) (void)hipEventDestroy(b->ev_copy);
    delete b;
    return FDW_OK;
}

int fdw_batch_apply(fdw_batch *b, fdw_op *const *ops, int n, const int *time_m, const int *time_M, void *stream) {
    FDW_GUARD_BEGIN
    if (!b || !ops || !time_m || !time_M || n < 1) return fail(FDW_ERR_ARG, "batch_apply: NULL argument or n < 1");
    const fdw_op *o0 = ops[0];
    if (!o0) return fail(FDW_ERR_ARG, "batch_apply: NULL op");
    const int kind = o0->d.kind, ndim = o0->ndim, R = o0->R;
    // A single 3D shot runs the single-shot kernels, which take the operator
    // and its field pointers as kernel arguments (the multi-shot kernels read
    // them from a record: 2.6 % slower at space order 16, up to 12 % for the
    // isotropic step); the results are the same bit for bit.  Only the checks
    // of the batch's own contract apply (forward, no saving, range, sparse
    // time axes): what only the multi-shot kernels need (fused sources, linear
    // receivers, fields below 4 GiB) does not.
    if (n == 1 && ndim == 3) {
        const fdw_op_desc &d = o0->d;
        if (d.mode != FDW_FORWARD || o0->save_buf)
            return fail(FDW_ERR_ARG, "batch_apply: op 0: forward operators without level saving only");
        if (time_m[0] < 0 || time_M[0] < time_m[0] - 1)
            return fail(FDW_ERR_ARG, "batch_apply: op 0: invalid range %d..%d", time_m[0], time_M[0]);
        const int nsrc = d.src ? d.src->npoint : 0, nrec = d.rec ? d.rec->npoint : 0;
        if ((nsrc > 0 && time_M[0] >= d.src->nt) || (nrec > 0 && time_M[0] >= d.rec->nt))
            return fail(FDW_ERR_ARG, "batch_apply: op 0: time_M = %d beyond the sparse time axis", time_M[0]);
        if (time_M[0] < time_m[0]) return FDW_OK;
        return fdw_operator_apply(ops[0], time_m[0], time_M[0], stream);
    }
    int K = 0;
    int64_t max_rec = 0;  // the most receivers of any shot
    for (int i = 0; i < n; ++i) {
        const fdw_op *op = ops[i];
        if (!op) return fail(FDW_ERR_ARG, "batch_apply: NULL op %d", i);
        const fdw_op_desc &d = op->d;
        const Geom &g = op->geom, &g0 = o0->geom;
        if (d.kind != kind || op->ndim != ndim || op->R != R || g.nx != g0.nx || g.ny != g0.ny || g.nz != g0.nz ||
            g.sy != g0.sy || g.sz != g0.sz || g.off0 != g0.off0)
            return fail(FDW_ERR_ARG, "batch_apply: op %d differs from op 0 in kind, space order or geometry", i);
        if (d.mode != FDW_FORWARD || op->save_buf)
            return fail(FDW_ERR_ARG, "batch_apply: op %d: forward operators without level saving only", i);
        if (ndim == 3 && (kind == FDW_ISO ? op->iso_v != IsoVariant::Stream : op->tti_v != TtiVariant::Stream))
            return fail(FDW_ERR_ARG, "batch_apply: op %d: 3D operators need the streaming kernels", i);
        if (ndim == 3 && kind == FDW_ISO && iso_wide_fields(g))
            return fail(FDW_ERR_ARG, "batch_apply: op %d: fields of 4 GiB or more are applied one shot at a time", i);
        const int nsrc = d.src ? d.src->npoint : 0, nrec = d.rec ? d.rec->npoint : 0;
        if (nsrc > 0 && !op->src_fused)
            return fail(FDW_ERR_ARG, "batch_apply: op %d: at most %d sources with linear weights per shot", i,
                        kMaxFusedSrc);
        if (nrec > 0 && (d.rec->r != 2))
            return fail(FDW_ERR_ARG, "batch_apply: op %d: receivers need linear weights", i);
        if (time_m[i] < 0 || time_M[i] < time_m[i] - 1)
            return fail(FDW_ERR_ARG, "batch_apply: op %d: invalid range %d..%d", i, time_m[i], time_M[i]);
        if ((nsrc > 0 && time_M[i] >= d.src->nt) || (nrec > 0 && time_M[i] >= d.rec->nt))
            return fail(FDW_ERR_ARG, "batch_apply: op %d: time_M = %d beyond the sparse time axis", i, time_M[i]);
        K = std::max(K, time_M[i] - time_m[i] + 1);
        max_rec = std::max<int64_t>(max_rec, nrec);
    }
    if (K == 0) return FDW_OK;
    hipStream_t s = (hipStream_t)stream;
    // 3D: receivers of step t are sampled in the launch of step t + 1, so one
    // more launch samples the last step; 2D: a sampling launch after each step
    const int nl = (ndim == 3 && max_rec > 0) ? K + 1 : K;
    const size_t r1 = kind == FDW_ISO ? iso_multi_record_bytes(ndim) : tti_multi_record_bytes(ndim, 1);
    const size_t r2 = (kind == FDW_TTI && ndim == 3) ? tti_multi_record_bytes(3, 2) : 0;
    const size_t rs = ndim == 2 ? sizeof(SparseArgs) : 0;
    const size_t off2 = align256(r1 * n), offs = off2 + align256(r2 * n);
    const size_t step_bytes = offs + align256(rs * n);
    // 2D isotropic grids small enough for the LDS-resident kernel: one
    // workgroup per shot runs its whole range in one launch, with the kernel
    // body fdw_operator_apply uses (so the same bits)
    bool persist = ndim == 2 && kind == FDW_ISO;
    for (int i = 0; i < n; ++i) persist = persist && ops[i]->use_persist2d;
    const size_t total = persist ? sizeof(Persist2DArgs) * (size_t)n : step_bytes * (size_t)nl;
    if (b->copy_pending) {
        hipError_t e = hipEventSynchronize(b->ev_copy);
        if (e != hipSuccess) return fail_hip(e, "batch_apply: waiting for the previous record copy");
        b->copy_pending = false;
    }
    if (total > b->cap) {
        // the device buffer may still be read by launched work on its stream
        if (b->d_stage) {
            hipError_t e = hipStreamSynchronize(b->graph_stream ? b->graph_stream : s);
            if (e != hipSuccess) return fail_hip(e, "batch_apply: hipStreamSynchronize");
        }
        batch_drop_graph(b);
        if (b->h_stage) (void)hipHostFree(b->h_stage);
        if (b->d_stage) (void)hipFree(b->d_stage);
        b->h_stage = b->d_stage = nullptr;
        b->cap = 0;
        const size_t cap = std::max(total, (size_t)1 << 20);
        hipError_t e = hipHostMalloc((void **)&b->h_stage, cap, hipHostMallocDefault);
        if (e == hipSuccess) e = hipMalloc((void **)&b->d_stage, cap);
        if (e != hipSuccess) return fail(FDW_ERR_NOMEM, "batch_apply: record buffers: %s", hipGetErrorString(e));
        b->cap = cap;
    }
    if (persist) {
        auto *pa = reinterpret_cast<Persist2DArgs *>(b->h_stage);
        for (int i = 0; i < n; ++i) persist2d_args(ops[i], time_m[i], time_M[i], pa[i]);
        hipError_t e = hipMemcpyAsync(b->d_stage, b->h_stage, total, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventRecord(b->ev_copy, s);
        if (e != hipSuccess) return fail_hip(e, "batch_apply: record upload");
        b->copy_pending = true;
        e = launch_iso2d_persistent_multi(R, o0->geom, reinterpret_cast<const Persist2DArgs *>(b->d_stage), n, s);
        if (e != hipSuccess) return fail_hip(e, "batch_apply: persistent 2D launch");
        return FDW_OK;
    }
    // pack the records of every launch
    std::memset(b->h_stage, 0, total);
    for (int k = 0; k < nl; ++k) {
        char *base = b->h_stage + (size_t)k * step_bytes;
        for (int i = 0; i < n; ++i) {
            const fdw_op *op = ops[i];
            const fdw_op_desc &d = op->d;
            const int cnt = time_M[i] - time_m[i] + 1;
            const int t = time_m[i] + std::min(k, std::max(cnt - 1, 0));
            const bool live = k < cnt;
            const int nrec = d.rec ? d.rec->npoint : 0;
            const int64_t E = op->lay.elems_per_slot;
            const int S = d.u->nslots;
            SparseArgs rec{};
            if (nrec > 0) {
                rec = sparse_template(op, d.rec, true);
                if (ndim == 3) {
                    // launch k samples row t - 1 from level t = time_m + k (its slot is
                    // read-only in that launch)
                    if (k >= 1 && k <= cnt) {
                        const int lv = time_m[i] + k;
                        rec.field = d.u->d + (int64_t)(lv % S) * E;
                        rec.rec_row = d.rec->data + (int64_t)(lv - 1) * nrec;
                    } else {
                        rec.npoint = 0;
                    }
                } else {
                    if (live) {
                        rec.field = d.u->d + (int64_t)((t + 1) % S) * E;
                        rec.rec_row = d.rec->data + (int64_t)t * nrec;
                    } else {
                        rec.npoint = 0;
                    }
                }
            }
            const SparseArgs none{};
            if (kind == FDW_ISO) {
                IsoArgs a;
                iso_step_args(op, t, a);
                multi_pack_iso(ndim, a, live, ndim == 3 ? rec : none, base + r1 * i);
            } else {
                TtiArgs a;
                tti_step_args(op, t, a, op->d_stage);
                multi_pack_tti(ndim, a, live, ndim == 3 ? rec : none, base + r1 * i, r2 ? base + off2 + r2 * i : nullptr);
            }
            if (ndim == 2) std::memcpy(base + offs + rs * i, &rec, sizeof(rec));
        }
    }
    hipError_t e = hipMemcpyAsync(b->d_stage, b->h_stage, total, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventRecord(b->ev_copy, s);
    if (e != hipSuccess) return fail_hip(e, "batch_apply: record upload");
    b->copy_pending = true;

    auto launches = [&](hipStream_t st) -> hipError_t {
        for (int k = 0; k < nl; ++k) {
            const char *base = b->d_stage + (size_t)k * step_bytes;
            const int64_t rl = ndim == 3 ? max_rec : 0;
            hipError_t er = kind == FDW_ISO ? launch_iso_multi(ndim, R, o0->geom, base, n, rl, st)
                                            : launch_tti_multi(ndim, R, o0->geom, base, r2 ? base + off2 : nullptr, n,
                                                               rl, st);
            if (er != hipSuccess) return er;
            if (ndim == 2 && max_rec > 0) {
                er = launch_interp_multi(reinterpret_cast<const SparseArgs *>(base + offs), n, max_rec, st);
                if (er != hipSuccess) return er;
            }
        }
        return hipSuccess;
    };
    const char *g_env = std::getenv("FDW_BATCH_GRAPH");
    const bool use_graph = s != nullptr && !(g_env && g_env[0] == '0');
    if (!use_graph) {
        e = launches(s);
        if (e != hipSuccess) return fail_hip(e, "batch_apply: launch");
        return FDW_OK;
    }
    const std::vector<int64_t> key = {kind, ndim, R, o0->geom.nx, o0->geom.ny, o0->geom.nz, o0->geom.sy, o0->geom.sz,
                                      o0->geom.off0, n, nl, max_rec, (int64_t)step_bytes, (int64_t)(intptr_t)b->d_stage,
                                      (int64_t)(intptr_t)s};
    if (!b->exec || key != b->key) {
        batch_drop_graph(b);
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return fail_hip(e, "batch_apply: hipStreamBeginCapture");
        hipError_t el = launches(s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail_hip(el != hipSuccess ? el : e, "batch_apply: graph capture");
        }
        e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            b->exec = nullptr;
            return fail_hip(e, "batch_apply: hipGraphInstantiate");
        }
        b->graph = g;
        b->key = key;
        b->graph_stream = s;
        b->graph_builds++;
    }
    e = hipGraphLaunch(b->exec, s);
    if (e != hipSuccess) return fail_hip(e, "batch_apply: hipGraphLaunch");
    b->graph_replays++;
    return FDW_OK;
    FDW_GUARD_END
}

int fdw_batch_stats(const fdw_batch *b, int64_t *graph_builds, int64_t *graph_launches) {
    if (!b) return fail(FDW_ERR_ARG, "batch_stats: NULL batch");
    if (graph_builds) *graph_builds = b->graph_builds;
    if (graph_launches) *graph_launches = b->graph_replays;
    return FDW_OK;
}

}  // extern "C"
