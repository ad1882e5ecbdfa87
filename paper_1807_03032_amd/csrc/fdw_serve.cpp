// Shot server: continuous batching of forward-modelling requests on one GPU.
//
// Requests of any kind (isotropic / TTI), dimension, grid size, space order
// and step count are queued; a scheduling round (fdw_server_progress)
//   1. retires shots whose last chunk has completed on the device (their
//      receiver traces are already copied to host memory) and returns their
//      device memory to the server's pool;
//   2. admits queued requests, in arrival order, whose device footprint fits
//      in what the budget has left (a request that does not fit lets later,
//      smaller ones pass);
//   3. advances every bucket -- the running shots of one (kind, geometry,
//      space order) -- by one chunk of steps with fused multi-shot launches
//      (fdw_batch_apply: one launch per stage and step for all shots of the
//      bucket, the launch sequence captured in a hipGraph and replayed), each
//      bucket on its own stream so the buckets' work overlaps on the device.
// Shots join and leave buckets between chunks; up to two chunks per bucket
// are in flight so the device does not wait for the host between chunks.
//
// Everything here is host orchestration over the public C ABI (fdw.h); every
// step of every shot runs in the library's HIP kernels.
#include "fdw.h"
#include "fdw_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <set>
#include <string>
#include <vector>

namespace {

// messages go to the library's thread-local error (fdw_last_error)
int sfail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    return fdw::set_error(code, buf);
}

int sfail_hip(hipError_t e, const char *where) {
    return sfail(FDW_ERR_DEVICE, "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
}

// propagate a library error with its message
int lib_fail(int st, const char *where) { return sfail(st, "%s: %s", where, fdw_last_error()); }

struct Shot;

// A shot of at least this many grid points fills the chip alone (a 200^3
// step already gives thousands of workgroups).
constexpr int64_t kLargePoints = (int64_t)1 << 22;

// Host time one progress call may spend admitting requests.
constexpr double kAdmitSliceSeconds = 0.004;

// One chunk of a bucket in flight: its completion event and the shots whose
// last step it contains.
struct Chunk {
    hipEvent_t ev = nullptr;
    int batch = 0;
    std::vector<Shot *> finishing;
};

struct Bucket {
    std::string key;
    bool large = false;  // one shot fills the chip (see kLargePoints)
    int64_t chunks_launched = 0;
    hipStream_t stream = nullptr;
    fdw_batch *batch[2] = {nullptr, nullptr};
    int next_batch = 0;
    int chunk_steps = 1;
    std::vector<Shot *> active;
    std::deque<Chunk> inflight;
    std::vector<hipEvent_t> free_events;
};

struct Shot {
    int64_t ticket = 0;
    fdw_shot_desc d{};  // borrowed host arrays until admission
    int64_t footprint = 0;
    int state = FDW_SHOT_QUEUED;
    double t_submit = 0, t_admit = 0, t_done = 0;
    int t_next = 0;
    // device objects while admitted
    fdw_grid *grid = nullptr;
    fdw_layout lay{};
    fdw_func *fn[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // m, eps, delta, theta, phi
    fdw_tfunc *tf[2] = {nullptr, nullptr};                            // u or p, r
    fdw_sparse *src = nullptr, *rec = nullptr;
    fdw_op *op = nullptr;
    std::vector<std::pair<void *, size_t>> dev;  // pool allocations
    float *d_field[2] = {nullptr, nullptr};
    float *d_src = nullptr, *d_rec = nullptr;
    // results (pinned host memory)
    float *h_rec = nullptr;
    float *h_field = nullptr;  // padded last level of u / p when kept
    bool released = false;     // results fetched; freed with the graveyard
    std::string error;         // why the shot failed (admission or a refused chunk)
};

}  // namespace

struct fdw_server {
    int64_t budget = 0, used = 0, pool_bytes = 0;
    int chunk_target_us = 20000;
    int nstreams = 1;
    std::vector<hipStream_t> streams;
    hipStream_t upload = nullptr;  // model uploads of admissions
    int next_stream = 0;
    std::vector<Bucket *> large_order;  // large buckets in creation order
    int64_t next_ticket = 1;
    std::deque<Shot *> queue;
    std::map<int64_t, std::unique_ptr<Shot>> shots;
    std::map<std::string, std::unique_ptr<Bucket>> buckets;
    std::multimap<size_t, void *> pool;  // free device blocks by size
    std::vector<Shot *> graveyard;       // retired shots whose library objects await destruction
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    int64_t chunks = 0, admitted = 0, completed = 0;
    double admit_s = 0, launch_s = 0;  // host time in admissions / chunk enqueueing

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

// ---------------------------------------------------------------- memory
int pool_alloc(fdw_server *sv, size_t bytes, void **out) {
    bytes = (bytes + 255) / 256 * 256;
    auto it = sv->pool.find(bytes);
    if (it != sv->pool.end()) {
        *out = it->second;
        sv->pool.erase(it);
        sv->pool_bytes -= (int64_t)bytes;
        return FDW_OK;
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return sfail(FDW_ERR_NOMEM, "server: hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    return FDW_OK;
}

void pool_release(fdw_server *sv, void *p, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    sv->pool.emplace(bytes, p);
    sv->pool_bytes += (int64_t)bytes;
}

// hipFree waits for the device; only called when the server is idle or
// memory is short.
void pool_trim(fdw_server *sv) {
    for (auto &kv : sv->pool) (void)hipFree(kv.second);
    sv->pool.clear();
    sv->pool_bytes = 0;
}

void destroy_objects(Shot *s) {
    if (s->op) fdw_operator_destroy(s->op);
    s->op = nullptr;
    if (s->src) fdw_sparse_destroy(s->src);
    if (s->rec) fdw_sparse_destroy(s->rec);
    s->src = s->rec = nullptr;
    for (auto &t : s->tf)
        if (t) {
            fdw_timefunction_destroy(t);
            t = nullptr;
        }
    for (auto &f : s->fn)
        if (f) {
            fdw_function_destroy(f);
            f = nullptr;
        }
    if (s->grid) fdw_grid_destroy(s->grid);
    s->grid = nullptr;
}

// Library objects and pinned buffers of retired shots are freed only here
// (hipFree / hipHostFree wait for the device), when the server is idle or
// short of memory, and at destruction.
void flush_graveyard(fdw_server *sv) {
    for (Shot *s : sv->graveyard) {
        destroy_objects(s);
        if (s->released) {
            if (s->h_rec) (void)hipHostFree(s->h_rec);
            if (s->h_field) (void)hipHostFree(s->h_field);
            s->h_rec = s->h_field = nullptr;
            sv->shots.erase(s->ticket);
        }
    }
    sv->graveyard.clear();
}

// ------------------------------------------------------------- footprint
struct Sizes {
    int64_t E = 0;
    int nwave = 0, nparam = 0, nstage = 0;
    int64_t sparse = 0, tables = 0;
};

int shot_sizes(const fdw_shot_desc *d, Sizes *z) {
    if (!d) return sfail(FDW_ERR_ARG, "server: NULL shot description");
    if (d->kind != FDW_ISO && d->kind != FDW_TTI) return sfail(FDW_ERR_ARG, "server: kind must be FDW_ISO or FDW_TTI");
    if (d->ndim != 2 && d->ndim != 3) return sfail(FDW_ERR_ARG, "server: ndim must be 2 or 3");
    if (d->nt < 1 || d->nsrc < 0 || d->nrec < 0) return sfail(FDW_ERR_ARG, "server: nt >= 1, nsrc, nrec >= 0");
    fdw_grid *g = nullptr;
    int st = fdw_grid_create(d->ndim, d->shape, d->extent, d->origin, &g);
    if (st) return lib_fail(st, "server: grid");
    fdw_layout L{};
    st = fdw_field_layout(g, d->space_order, &L);
    fdw_grid_destroy(g);
    if (st) return lib_fail(st, "server: layout");
    z->E = L.elems_per_slot;
    const bool tti = d->kind == FDW_TTI;
    z->nwave = tti ? 4 : 2;                          // two slots (in-place leapfrog) per wavefield
    z->nparam = tti ? (d->ndim == 3 ? 5 : 4) : 1;    // m (, eps, delta, theta, phi)
    z->nstage = tti ? 2 : 0;                         // TTI rotated-gradient buffers
    z->sparse = (int64_t)d->nt * (d->nsrc + d->nrec);
    int64_t axes = 0;
    for (int a = 0; a < d->ndim; ++a) axes += d->shape[a];
    z->tables = axes + (int64_t)(d->nsrc + d->nrec) * (2 + (1 << d->ndim) + 3);
    return FDW_OK;
}

int64_t footprint_bytes(const Sizes &z) {
    return 4 * ((int64_t)(z.nwave + z.nparam + z.nstage) * z.E + z.sparse + z.tables) + 64 * 256;
}

// ------------------------------------------------------------- admission
// Shots of one kind, grid and space order share a bucket (fused launches).  A
// shot that fills the GPU alone gains nothing from fusion (the multi-shot
// kernels read the operator from a record and are slower), so it gets a
// bucket of its own and runs the single-shot kernels.
std::string bucket_key(const fdw_shot_desc &d, int64_t ticket) {
    int64_t npts = 1;
    for (int a = 0; a < d.ndim; ++a) npts *= d.shape[a];
    char buf[256];
    snprintf(buf, sizeof(buf), "%d/%d/%lldx%lldx%lld/so%d/h%.9g,%.9g,%.9g/%lld", d.kind, d.ndim,
             (long long)d.shape[0], (long long)d.shape[1], (long long)(d.ndim == 3 ? d.shape[2] : 1), d.space_order,
             d.extent[0] / (double)(d.shape[0] - 1), d.extent[1] / (double)(d.shape[1] - 1),
             d.ndim == 3 ? d.extent[2] / (double)(d.shape[2] - 1) : 0.0,
             (long long)(npts >= kLargePoints ? ticket : 0));
    return buf;
}

fdw::Geom layout_geom(const fdw_layout &L, int ndim) {
    fdw::Geom g{};
    g.nx = (int)L.shape[0];
    g.ny = ndim == 3 ? (int)L.shape[1] : 1;
    g.nz = ndim == 3 ? (int)L.shape[2] : (int)L.shape[1];
    g.sy = ndim == 3 ? L.pitch_x : 0;
    g.sz = ndim == 3 ? L.pitch_x * L.pitch_y : L.pitch_x;
    g.off0 = L.origin_offset;
    return g;
}

// logical host array (x fastest) -> padded device slot: one contiguous copy
// into a device staging buffer, then a scatter kernel into the layout
int upload_field(const fdw_layout &L, int ndim, const float *host, float *staging, float *dev, hipStream_t s) {
    const fdw::Geom g = layout_geom(L, ndim);
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    hipError_t e = hipMemcpyAsync(staging, host, n * sizeof(float), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = fdw::launch_pad_copy(g, staging, dev, s);
    if (e != hipSuccess) return sfail_hip(e, "server: model upload");
    return FDW_OK;
}

int admit(fdw_server *sv, Shot *s) {
    const fdw_shot_desc &d = s->d;
    Sizes z;
    int st = shot_sizes(&d, &z);
    if (st) return st;
    const std::string key = bucket_key(d, s->ticket);
    auto bit = sv->buckets.find(key);
    Bucket *b = nullptr;
    if (bit == sv->buckets.end()) {
        auto nb = std::make_unique<Bucket>();
        nb->key = key;
        int64_t npts = 1;
        for (int a = 0; a < d.ndim; ++a) npts *= d.shape[a];
        // Shots that fill the chip alone gain nothing from running beside each
        // other (they only compete for the caches): large buckets advance one at
        // a time, in creation order, on stream 0; small ones share the other
        // streams and fill the gaps.
        nb->large = npts >= kLargePoints;
        nb->stream = nb->large ? sv->streams[0] : sv->streams[sv->nstreams > 1 ? 1 + sv->next_stream++ % (sv->nstreams - 1) : 0];
        for (auto &bt : nb->batch) {
            st = fdw_batch_create(&bt);
            if (st) return lib_fail(st, "server: batch");
        }
        // chunk length: about chunk_target_us of device time for one shot
        const double pts_per_us = d.kind == FDW_TTI ? 40e3 : 250e3;
        const double step_us = (double)npts / pts_per_us + 4.0;
        nb->chunk_steps = (int)std::min(1000.0, std::max(8.0, sv->chunk_target_us / step_us));
        b = nb.get();
        if (b->large) sv->large_order.push_back(b);
        sv->buckets.emplace(key, std::move(nb));
    } else {
        b = bit->second.get();
    }
    hipStream_t hs = sv->upload;
    auto alloc = [&](size_t bytes, void **p) -> int {
        int r = pool_alloc(sv, bytes, p);
        if (!r) s->dev.emplace_back(*p, bytes);
        return r;
    };
    auto fail_admit = [&](int code) {
        for (auto &pb : s->dev) pool_release(sv, pb.first, pb.second);
        s->dev.clear();
        destroy_objects(s);
        if (s->h_rec) (void)hipHostFree(s->h_rec);
        if (s->h_field) (void)hipHostFree(s->h_field);
        s->h_rec = s->h_field = nullptr;
        return code;
    };
    st = fdw_grid_create(d.ndim, d.shape, d.extent, d.origin, &s->grid);
    if (st) return fail_admit(lib_fail(st, "server: grid"));
    fdw_field_layout(s->grid, d.space_order, &s->lay);
    const int64_t E = z.E;
    const bool tti = d.kind == FDW_TTI;
    static const char *wname[2] = {"u", "r"};
    for (int w = 0; w < (tti ? 2 : 1); ++w) {
        void *p = nullptr;
        if ((st = alloc(sizeof(float) * 2 * E, &p))) return fail_admit(st);
        s->d_field[w] = (float *)p;
        hipError_t e = hipMemsetAsync(p, 0, sizeof(float) * 2 * E, hs);
        if (e != hipSuccess) return fail_admit(sfail_hip(e, "server: wavefield clear"));
        st = fdw_timefunction_bind(s->grid, tti && w == 0 ? "p" : wname[w], (float *)p, 2 * E, d.space_order, 2, 2,
                                   &s->tf[w]);
        if (st) return fail_admit(lib_fail(st, "server: wavefield"));
    }
    const float *params[5] = {d.m, d.eps, d.delta, d.theta, d.phi};
    static const char *pname[5] = {"m", "eps", "delta", "theta", "phi"};
    size_t nlog = 1;
    for (int a = 0; a < d.ndim; ++a) nlog *= (size_t)d.shape[a];
    void *staging = nullptr;
    if ((st = pool_alloc(sv, sizeof(float) * nlog, &staging))) return fail_admit(st);
    struct StagingGuard {  // back to the pool once the uploads are done
        fdw_server *sv;
        void *p;
        size_t n;
        ~StagingGuard() { pool_release(sv, p, n); }
    } guard{sv, staging, sizeof(float) * nlog};
    for (int k = 0; k < z.nparam; ++k) {
        if (!params[k]) return fail_admit(sfail(FDW_ERR_ARG, "server: ticket %lld: %s missing", (long long)s->ticket, pname[k]));
        void *p = nullptr;
        if ((st = alloc(sizeof(float) * E, &p))) return fail_admit(st);
        // m = 1 outside the domain keeps 1/m finite (never read); others 0
        const uint32_t fill = k == 0 ? 0x3f800000u : 0u;
        hipError_t e = hipMemsetD32Async((hipDeviceptr_t)p, (int)fill, (size_t)E, hs);
        if (e != hipSuccess) return fail_admit(sfail_hip(e, "server: parameter fill"));
        if ((st = upload_field(s->lay, d.ndim, params[k], (float *)staging, (float *)p, hs))) return fail_admit(st);
        // the staging buffer is reused by the next field
        hipError_t es = hipStreamSynchronize(hs);
        if (es != hipSuccess) return fail_admit(sfail_hip(es, "server: upload"));
        st = fdw_function_bind(s->grid, pname[k], (float *)p, E, d.space_order, &s->fn[k]);
        if (st) return fail_admit(lib_fail(st, "server: parameter"));
    }
    if (d.nsrc > 0) {
        void *p = nullptr;
        if ((st = alloc(sizeof(float) * (size_t)d.nt * d.nsrc, &p))) return fail_admit(st);
        s->d_src = (float *)p;
        hipError_t e = hipMemcpyAsync(p, d.src, sizeof(float) * (size_t)d.nt * d.nsrc, hipMemcpyHostToDevice, hs);
        if (e != hipSuccess) return fail_admit(sfail_hip(e, "server: source upload"));
        st = fdw_sparse_bind(s->grid, "src", d.nsrc, d.nt, d.src_coords, s->d_src, &s->src);
        if (st) return fail_admit(lib_fail(st, "server: sources"));
    }
    if (d.nrec > 0) {
        void *p = nullptr;
        if ((st = alloc(sizeof(float) * (size_t)d.nt * d.nrec, &p))) return fail_admit(st);
        s->d_rec = (float *)p;
        st = fdw_sparse_bind(s->grid, "rec", d.nrec, d.nt, d.rec_coords, s->d_rec, &s->rec);
        if (st) return fail_admit(lib_fail(st, "server: receivers"));
        hipError_t e = hipHostMalloc((void **)&s->h_rec, sizeof(float) * (size_t)d.nt * d.nrec, hipHostMallocDefault);
        if (e != hipSuccess) return fail_admit(sfail(FDW_ERR_NOMEM, "server: pinned trace buffer"));
    }
    if (d.keep_field) {
        hipError_t e = hipHostMalloc((void **)&s->h_field, sizeof(float) * (size_t)E, hipHostMallocDefault);
        if (e != hipSuccess) return fail_admit(sfail(FDW_ERR_NOMEM, "server: pinned field buffer"));
    }
    fdw_op_desc od{};
    od.kind = d.kind;
    od.space_order = d.space_order;
    od.dt = d.dt;
    od.nbl = d.nbl;
    od.damp_rc = d.damp_rc;
    od.vmax = d.vmax;
    od.eps_max = d.eps_max;
    od.u = s->tf[0];
    od.r = s->tf[1];
    od.m = s->fn[0];
    od.eps = s->fn[1];
    od.delta = s->fn[2];
    od.theta = s->fn[3];
    od.phi = s->fn[4];
    od.src = s->src;
    od.rec = s->rec;
    od.mode = FDW_FORWARD;
    // uploads and clears complete before the shot's first chunk is enqueued
    // (the operator's own set-up completes inside fdw_operator_create)
    hipError_t e = hipStreamSynchronize(hs);
    if (e != hipSuccess) return fail_admit(sfail_hip(e, "server: upload"));
    st = fdw_operator_create(&od, &s->op);
    if (st) return fail_admit(lib_fail(st, "server: operator"));
    s->footprint = footprint_bytes(z);
    s->state = FDW_SHOT_RUNNING;
    s->t_admit = sv->now();
    s->t_next = 0;
    b->active.push_back(s);
    sv->used += s->footprint;
    sv->admitted++;
    return FDW_OK;
}

void retire(fdw_server *sv, Shot *s) {
    for (auto &pb : s->dev) pool_release(sv, pb.first, pb.second);
    s->dev.clear();
    s->d_field[0] = s->d_field[1] = nullptr;
    s->d_src = s->d_rec = nullptr;
    sv->used -= s->footprint;
    s->state = FDW_SHOT_DONE;
    s->t_done = sv->now();
    sv->completed++;
    sv->graveyard.push_back(s);
}

// A running shot whose chunk the library refuses: it fails alone, its device
// blocks go back to the pool once the bucket's chunks in flight (which may
// still read them) have completed.
void fail_running(fdw_server *sv, Bucket *b, const std::string &why) {
    for (Chunk &c : b->inflight) (void)hipEventSynchronize(c.ev);
    for (Shot *s : b->active) {
        for (auto &pb : s->dev) pool_release(sv, pb.first, pb.second);
        s->dev.clear();
        s->d_field[0] = s->d_field[1] = nullptr;
        s->d_src = s->d_rec = nullptr;
        sv->used -= s->footprint;
        s->state = FDW_SHOT_FAILED;
        s->error = why;
        s->t_done = sv->now();
        sv->graveyard.push_back(s);
    }
    b->active.clear();
}

// enqueue one chunk of a bucket
int launch_chunk(fdw_server *sv, Bucket *b) {
    const int n = (int)b->active.size();
    std::vector<fdw_op *> ops(n);
    std::vector<int> tm(n), tM(n);
    Chunk c;
    std::vector<Shot *> keep;
    for (int i = 0; i < n; ++i) {
        Shot *s = b->active[i];
        ops[i] = s->op;
        tm[i] = s->t_next;
        tM[i] = std::min(s->t_next + b->chunk_steps, s->d.nt) - 1;
    }
    c.batch = b->next_batch;
    b->next_batch ^= 1;
    int st = fdw_batch_apply(b->batch[c.batch], ops.data(), n, tm.data(), tM.data(), b->stream);
    if (st == FDW_ERR_DEVICE) return lib_fail(st, "server: chunk");
    if (st) {  // refused before any launch: these shots fail, the others go on
        fail_running(sv, b, std::string("server: chunk refused: ") + fdw_last_error());
        b->next_batch = c.batch;
        return FDW_OK;
    }
    for (int i = 0; i < n; ++i) {
        Shot *s = b->active[i];
        s->t_next = tM[i] + 1;
        if (s->t_next >= s->d.nt) {
            const fdw_shot_desc &d = s->d;
            hipError_t e = hipSuccess;
            if (d.nrec > 0)
                e = hipMemcpyAsync(s->h_rec, s->d_rec, sizeof(float) * (size_t)d.nt * d.nrec, hipMemcpyDeviceToHost,
                                   b->stream);
            if (e == hipSuccess && s->h_field)  // level nt lives in slot nt mod 2
                e = hipMemcpyAsync(s->h_field, s->d_field[0] + (int64_t)(d.nt % 2) * s->lay.elems_per_slot,
                                   sizeof(float) * (size_t)s->lay.elems_per_slot, hipMemcpyDeviceToHost, b->stream);
            if (e != hipSuccess) return sfail_hip(e, "server: result copy");
            c.finishing.push_back(s);
        } else {
            keep.push_back(s);
        }
    }
    b->active.swap(keep);
    if (b->free_events.empty()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return sfail_hip(e, "server: hipEventCreate");
        b->free_events.push_back(ev);
    }
    c.ev = b->free_events.back();
    b->free_events.pop_back();
    hipError_t e = hipEventRecord(c.ev, b->stream);
    if (e != hipSuccess) return sfail_hip(e, "server: hipEventRecord");
    b->inflight.push_back(std::move(c));
    b->chunks_launched++;
    sv->chunks++;
    return FDW_OK;
}

}  // namespace

extern "C" {

int fdw_server_footprint(const fdw_shot_desc *d, int64_t *bytes) {
    if (!bytes) return sfail(FDW_ERR_ARG, "server_footprint: NULL bytes");
    Sizes z;
    int st = shot_sizes(d, &z);
    if (st) return st;
    *bytes = footprint_bytes(z);
    return FDW_OK;
}

int fdw_server_create(int64_t budget_bytes, int chunk_target_us, int nstreams, fdw_server **out) {
    if (!out || nstreams < 1 || nstreams > 16 || chunk_target_us < 0)
        return sfail(FDW_ERR_ARG, "server_create: NULL out, nstreams outside 1..16 or negative chunk target");
    fdw_server *sv = new (std::nothrow) fdw_server();
    if (!sv) return sfail(FDW_ERR_NOMEM, "server_create: host allocation");
    if (budget_bytes <= 0) {
        size_t fr = 0, tot = 0;
        hipError_t e = hipMemGetInfo(&fr, &tot);
        if (e != hipSuccess) {
            delete sv;
            return sfail_hip(e, "server_create: hipMemGetInfo");
        }
        budget_bytes = (int64_t)(0.8 * (double)fr);
    }
    sv->budget = budget_bytes;
    sv->chunk_target_us = chunk_target_us > 0 ? chunk_target_us : 20000;
    sv->nstreams = nstreams;
    for (int i = 0; i <= nstreams; ++i) {
        hipStream_t s;
        hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e != hipSuccess) {
            for (hipStream_t x : sv->streams) (void)hipStreamDestroy(x);
            if (sv->upload) (void)hipStreamDestroy(sv->upload);
            delete sv;
            return sfail_hip(e, "server_create: hipStreamCreate");
        }
        if (i == nstreams)
            sv->upload = s;
        else
            sv->streams.push_back(s);
    }
    *out = sv;
    return FDW_OK;
}

int fdw_server_submit(fdw_server *sv, const fdw_shot_desc *d, int64_t *ticket) {
    if (!sv || !d || !ticket) return sfail(FDW_ERR_ARG, "server_submit: NULL argument");
    Sizes z;
    int st = shot_sizes(d, &z);
    if (st) return st;
    if (!d->m || (d->nsrc > 0 && (!d->src_coords || !d->src)) || (d->nrec > 0 && !d->rec_coords))
        return sfail(FDW_ERR_ARG, "server_submit: missing model, source or receiver arrays");
    if (d->nsrc > 4) return sfail(FDW_ERR_ARG, "server_submit: at most 4 sources per shot");
    const int64_t fp = footprint_bytes(z);
    if (fp > sv->budget)
        return sfail(FDW_ERR_NOMEM, "server_submit: footprint %lld bytes exceeds the budget %lld", (long long)fp,
                     (long long)sv->budget);
    auto s = std::make_unique<Shot>();
    s->ticket = sv->next_ticket++;
    s->d = *d;
    s->footprint = fp;
    s->t_submit = sv->now();
    sv->queue.push_back(s.get());
    *ticket = s->ticket;
    sv->shots.emplace(s->ticket, std::move(s));
    return FDW_OK;
}

int fdw_server_progress(fdw_server *sv, int *queued, int *running) {
    if (!sv) return sfail(FDW_ERR_ARG, "server_progress: NULL server");
    // 1. completed chunks
    for (auto &kv : sv->buckets) {
        Bucket *b = kv.second.get();
        while (!b->inflight.empty()) {
            Chunk &c = b->inflight.front();
            hipError_t e = hipEventQuery(c.ev);
            if (e == hipErrorNotReady) break;
            if (e != hipSuccess) return sfail_hip(e, "server_progress: chunk");
            for (Shot *s : c.finishing) retire(sv, s);
            b->free_events.push_back(c.ev);
            b->inflight.pop_front();
        }
    }
    // a large bucket holds one shot: drop it once that shot's work is done
    for (auto it = sv->buckets.begin(); it != sv->buckets.end();) {
        Bucket *b = it->second.get();
        if (b->large && b->active.empty() && b->inflight.empty()) {
            for (hipEvent_t e : b->free_events) (void)hipEventDestroy(e);
            for (fdw_batch *bt : b->batch) fdw_batch_destroy(bt);
            sv->large_order.erase(std::remove(sv->large_order.begin(), sv->large_order.end(), b),
                                  sv->large_order.end());
            it = sv->buckets.erase(it);
        } else {
            ++it;
        }
    }
    // 2. admissions, in arrival order; requests that do not fit wait.  At most
    // a few milliseconds of host work per call: the chunks of what is already
    // admitted are launched below, so the GPU starts on the first requests of
    // a burst while the later ones are still being uploaded.
    const double t_adm = sv->now();
    bool sliced = false;  // queued requests left unexamined for lack of time
    for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        if (sv->now() - t_adm > kAdmitSliceSeconds) {
            sliced = true;
            break;
        }
        Shot *s = *it;
        if (sv->used + s->footprint > sv->budget) {
            ++it;
            continue;
        }
        const double ta = sv->now();
        int st = admit(sv, s);
        sv->admit_s += sv->now() - ta;
        if (st == FDW_ERR_NOMEM && (!sv->pool.empty() || !sv->graveyard.empty())) {
            // free cached blocks and retired objects, then try once more
            for (auto &kv : sv->buckets)
                for (Chunk &c : kv.second->inflight) (void)hipEventSynchronize(c.ev);
            flush_graveyard(sv);
            pool_trim(sv);
            st = admit(sv, s);
        }
        if (st == FDW_ERR_NOMEM && sv->used > 0) {  // may fit once running shots retire
            ++it;
            continue;
        }
        if (st == FDW_ERR_DEVICE) return st;
        if (st) {  // cannot be served: fail this request, keep serving the others
            s->state = FDW_SHOT_FAILED;
            s->error = fdw_last_error();
            s->t_done = sv->now();
        }
        it = sv->queue.erase(it);
    }
    // 3. next chunk of every bucket with running shots (two chunks in flight);
    // of the large buckets only the oldest one with running shots.  While
    // admissions are cut short, a bucket that has not started yet waits for
    // the queued requests of its own shape, so that they share its launches.
    std::set<std::string> pending_keys;
    if (sliced)
        for (Shot *q : sv->queue) pending_keys.insert(bucket_key(q->d, q->ticket));
    Bucket *large_now = nullptr;
    for (Bucket *b : sv->large_order)
        if (!b->active.empty()) {
            large_now = b;
            break;
        }
    int nrun = 0;
    for (auto &kv : sv->buckets) {
        Bucket *b = kv.second.get();
        const bool gather = b->inflight.empty() && b->chunks_launched == 0 && pending_keys.count(b->key) > 0;
        if (!b->active.empty() && b->inflight.size() < 2 && (!b->large || b == large_now) && !gather) {
            const double tl = sv->now();
            int st = launch_chunk(sv, b);
            sv->launch_s += sv->now() - tl;
            if (st) return st;
        }
        nrun += (int)b->active.size();
        for (Chunk &c : b->inflight) nrun += (int)c.finishing.size();
    }
    if (nrun == 0 && sv->queue.empty()) flush_graveyard(sv);
    if (queued) *queued = (int)sv->queue.size();
    if (running) *running = nrun;
    return FDW_OK;
}

int fdw_server_info(fdw_server *sv, int64_t ticket, fdw_shot_info *out) {
    if (!sv || !out) return sfail(FDW_ERR_ARG, "server_info: NULL argument");
    auto it = sv->shots.find(ticket);
    if (it == sv->shots.end() || it->second->released)
        return sfail(FDW_ERR_ARG, "server_info: unknown or released ticket %lld", (long long)ticket);
    const Shot *s = it->second.get();
    out->state = s->state;
    out->footprint = s->footprint;
    out->t_submit = s->t_submit;
    out->t_admit = s->t_admit;
    out->t_done = s->t_done;
    out->steps_done = s->state == FDW_SHOT_DONE ? s->d.nt : (s->state == FDW_SHOT_RUNNING ? s->t_next : 0);
    return FDW_OK;
}

int fdw_server_fetch(fdw_server *sv, int64_t ticket, float *rec_host, float *field_host) {
    if (!sv) return sfail(FDW_ERR_ARG, "server_fetch: NULL server");
    auto it = sv->shots.find(ticket);
    if (it == sv->shots.end()) return sfail(FDW_ERR_ARG, "server_fetch: unknown ticket %lld", (long long)ticket);
    Shot *s = it->second.get();
    if (s->state == FDW_SHOT_FAILED)
        return sfail(FDW_ERR_STATE, "server_fetch: ticket %lld failed: %s", (long long)ticket,
                     s->error.c_str());
    if (s->state != FDW_SHOT_DONE) return sfail(FDW_ERR_STATE, "server_fetch: ticket %lld not finished", (long long)ticket);
    if (s->released) return sfail(FDW_ERR_STATE, "server_fetch: ticket %lld was released", (long long)ticket);
    const fdw_shot_desc &d = s->d;
    if (rec_host && d.nrec > 0) std::memcpy(rec_host, s->h_rec, sizeof(float) * (size_t)d.nt * d.nrec);
    if (field_host) {
        if (!s->h_field) return sfail(FDW_ERR_STATE, "server_fetch: ticket %lld kept no field", (long long)ticket);
        const fdw_layout &L = s->lay;
        const int64_t nx = L.shape[0], ny = d.ndim == 3 ? L.shape[1] : 1, nz = d.ndim == 3 ? L.shape[2] : L.shape[1];
        for (int64_t z = 0; z < nz; ++z)
            for (int64_t y = 0; y < ny; ++y) {
                const float *src = s->h_field + L.origin_offset + z * L.pitch_x * (d.ndim == 3 ? L.pitch_y : 1) +
                                   y * L.pitch_x;
                std::memcpy(field_host + (z * ny + y) * nx, src, sizeof(float) * (size_t)nx);
            }
    }
    return FDW_OK;
}

int fdw_server_release(fdw_server *sv, int64_t ticket) {
    if (!sv) return sfail(FDW_ERR_ARG, "server_release: NULL server");
    auto it = sv->shots.find(ticket);
    if (it == sv->shots.end()) return sfail(FDW_ERR_ARG, "server_release: unknown ticket %lld", (long long)ticket);
    Shot *s = it->second.get();
    if (s->state != FDW_SHOT_DONE && s->state != FDW_SHOT_FAILED)
        return sfail(FDW_ERR_STATE, "server_release: ticket %lld not finished", (long long)ticket);
    if (s->released) return sfail(FDW_ERR_STATE, "server_release: ticket %lld already released", (long long)ticket);
    s->released = true;
    // freeing now would wait for the device: the graveyard frees it later
    if (std::find(sv->graveyard.begin(), sv->graveyard.end(), s) == sv->graveyard.end()) {
        if (s->h_rec) (void)hipHostFree(s->h_rec);
        if (s->h_field) (void)hipHostFree(s->h_field);
        sv->shots.erase(it);
    }
    return FDW_OK;
}

int fdw_server_stats(fdw_server *sv, fdw_server_stats_t *out) {
    if (!sv || !out) return sfail(FDW_ERR_ARG, "server_stats: NULL argument");
    out->budget = sv->budget;
    out->used = sv->used;
    out->pool_bytes = sv->pool_bytes;
    out->chunks = sv->chunks;
    out->admitted = sv->admitted;
    out->completed = sv->completed;
    out->buckets = (int64_t)sv->buckets.size();
    int64_t builds = 0, launches = 0;
    for (auto &kv : sv->buckets)
        for (fdw_batch *bt : kv.second->batch) {
            int64_t gb = 0, gl = 0;
            if (bt && !fdw_batch_stats(bt, &gb, &gl)) {
                builds += gb;
                launches += gl;
            }
        }
    out->graph_builds = builds;
    out->graph_launches = launches;
    out->now = sv->now();
    out->admit_seconds = sv->admit_s;
    out->launch_seconds = sv->launch_s;
    return FDW_OK;
}

int fdw_server_destroy(fdw_server *sv) {
    if (!sv) return FDW_OK;
    for (hipStream_t s : sv->streams) (void)hipStreamSynchronize(s);
    (void)hipStreamSynchronize(sv->upload);
    for (auto &kv : sv->buckets) {
        Bucket *b = kv.second.get();
        for (Chunk &c : b->inflight) {
            for (Shot *s : c.finishing) retire(sv, s);
            b->free_events.push_back(c.ev);
        }
        b->inflight.clear();
        for (Shot *s : b->active) retire(sv, s);
        b->active.clear();
        for (hipEvent_t e : b->free_events) (void)hipEventDestroy(e);
        for (fdw_batch *bt : b->batch) fdw_batch_destroy(bt);
    }
    flush_graveyard(sv);
    for (auto &kv : sv->shots) {
        Shot *s = kv.second.get();
        if (s->h_rec) (void)hipHostFree(s->h_rec);
        if (s->h_field) (void)hipHostFree(s->h_field);
        s->h_rec = s->h_field = nullptr;
    }
    pool_trim(sv);
    for (hipStream_t s : sv->streams) (void)hipStreamDestroy(s);
    (void)hipStreamDestroy(sv->upload);
    delete sv;
    return FDW_OK;
}

}  // extern "C"
