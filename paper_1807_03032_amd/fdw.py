"""Python binding of the fdw C ABI (include/fdw.h).

Argument marshalling only: every step of the operators (stencil, injection,
interpolation) runs in the HIP kernels of libfdw.so.  PyTorch supplies device
memory (tensors) and streams; numpy arrays are moved in and out of the padded
field layout with plain tensor copies.

The functions keep the C names (fdw_grid_create, ..., fdw_operator_apply) and
raise FdwError on a negative status, carrying fdw_last_error().  Loading fails
loudly when the HIP library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libfdw.so")

FDW_OK = 0
FDW_ERR_ARG = -1
FDW_ERR_DOMAIN = -2
FDW_ERR_UNSTABLE = -3
FDW_ERR_LAYOUT = -4
FDW_ERR_DEVICE = -5
FDW_ERR_NOMEM = -6
FDW_ERR_STATE = -7
FDW_ISO = 0
FDW_TTI = 1
FDW_FORWARD = 0
FDW_ADJOINT = 1
FDW_X_OFFSET = 32

# every symbol include/fdw.h declares
EXPORTS = (
    "fdw_grid_create", "fdw_grid_destroy", "fdw_field_layout", "fdw_function_bind", "fdw_function_destroy",
    "fdw_timefunction_bind", "fdw_timefunction_destroy", "fdw_sparse_bind", "fdw_sparse_destroy",
    "fdw_operator_create", "fdw_operator_apply", "fdw_sync", "fdw_operator_destroy",
    "fdw_operator_set_timing", "fdw_operator_kernel_time", "fdw_operator_describe", "fdw_stable_dt",
    "fdw_last_error", "fdw_version", "fdw_operator_set_save", "fdw_gradient_accumulate",
    "fdw_sparse_bind_precomputed", "fdw_batch_create", "fdw_batch_apply", "fdw_batch_stats", "fdw_batch_destroy",
    "fdw_server_create", "fdw_server_footprint", "fdw_server_submit", "fdw_server_progress", "fdw_server_info",
    "fdw_server_fetch", "fdw_server_release", "fdw_server_stats", "fdw_server_destroy", "fdw_bandwidth_probe",
    "fdw_operator_apply_noalloc", "fdw_operator_set_imaging_save", "fdw_gradient_apply", "fdw_operator_graph_stats",
)
FDW_SHOT_QUEUED, FDW_SHOT_RUNNING, FDW_SHOT_DONE, FDW_SHOT_FAILED = 0, 1, 2, 3


class FdwError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fdw status {code}: {msg}")
        self.code = code


class fdw_layout(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("halo", ctypes.c_int), ("shape", ctypes.c_int64 * 3),
                ("pitch_x", ctypes.c_int64), ("pitch_y", ctypes.c_int64), ("planes", ctypes.c_int64),
                ("origin_offset", ctypes.c_int64), ("elems_per_slot", ctypes.c_int64),
                ("alignment_bytes", ctypes.c_int)]


class fdw_op_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("space_order", ctypes.c_int), ("dt", ctypes.c_double),
                ("nbl", ctypes.c_int), ("damp_rc", ctypes.c_double), ("vmax", ctypes.c_double),
                ("eps_max", ctypes.c_double), ("u", ctypes.c_void_p), ("r", ctypes.c_void_p),
                ("m", ctypes.c_void_p), ("eps", ctypes.c_void_p), ("delta", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("phi", ctypes.c_void_p), ("src", ctypes.c_void_p),
                ("rec", ctypes.c_void_p), ("mode", ctypes.c_int)]


class fdw_shot_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("ndim", ctypes.c_int), ("shape", ctypes.c_int64 * 3),
                ("extent", ctypes.c_double * 3), ("origin", ctypes.c_double * 3), ("space_order", ctypes.c_int),
                ("nt", ctypes.c_int), ("dt", ctypes.c_double), ("nbl", ctypes.c_int), ("damp_rc", ctypes.c_double),
                ("vmax", ctypes.c_double), ("eps_max", ctypes.c_double), ("m", ctypes.c_void_p),
                ("eps", ctypes.c_void_p), ("delta", ctypes.c_void_p), ("theta", ctypes.c_void_p),
                ("phi", ctypes.c_void_p), ("nsrc", ctypes.c_int), ("src_coords", ctypes.c_void_p),
                ("src", ctypes.c_void_p), ("nrec", ctypes.c_int), ("rec_coords", ctypes.c_void_p),
                ("keep_field", ctypes.c_int)]


class fdw_shot_info(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int), ("steps_done", ctypes.c_int), ("footprint", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class fdw_server_stats_t(ctypes.Structure):
    _fields_ = [("budget", ctypes.c_int64), ("used", ctypes.c_int64), ("pool_bytes", ctypes.c_int64),
                ("chunks", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("buckets", ctypes.c_int64), ("graph_builds", ctypes.c_int64), ("graph_launches", ctypes.c_int64),
                ("now", ctypes.c_double), ("admit_seconds", ctypes.c_double), ("launch_seconds", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libfdw.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"HIP library {path} is missing: run paper_1807_03032_amd.build first")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
    pvp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "fdw_grid_create": (i32, [i32, ctypes.POINTER(i64), ctypes.POINTER(dbl), ctypes.POINTER(dbl), pvp]),
        "fdw_grid_destroy": (i32, [vp]),
        "fdw_field_layout": (i32, [vp, i32, ctypes.POINTER(fdw_layout)]),
        "fdw_function_bind": (i32, [vp, ctypes.c_char_p, vp, i64, i32, pvp]),
        "fdw_function_destroy": (i32, [vp]),
        "fdw_timefunction_bind": (i32, [vp, ctypes.c_char_p, vp, i64, i32, i32, i32, pvp]),
        "fdw_timefunction_destroy": (i32, [vp]),
        "fdw_sparse_bind": (i32, [vp, ctypes.c_char_p, i32, i32, ctypes.POINTER(dbl), vp, pvp]),
        "fdw_sparse_bind_precomputed": (i32, [vp, ctypes.c_char_p, i32, i32, i32, ctypes.POINTER(ctypes.c_int64),
                                              ctypes.POINTER(dbl), vp, pvp]),
        "fdw_sparse_destroy": (i32, [vp]),
        "fdw_operator_create": (i32, [ctypes.POINTER(fdw_op_desc), pvp]),
        "fdw_operator_apply": (i32, [vp, i32, i32, vp]),
        "fdw_operator_apply_noalloc": (i32, [vp, i32, i32, vp]),
        "fdw_sync": (i32, [vp]),
        "fdw_operator_destroy": (i32, [vp]),
        "fdw_operator_set_timing": (i32, [vp, i32]),
        "fdw_operator_kernel_time": (i32, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64), i32]),
        "fdw_operator_describe": (i32, [vp, ctypes.c_char_p, i32, ctypes.POINTER(dbl)]),
        "fdw_stable_dt": (dbl, [i32, i32, i32, dbl, dbl, dbl]),
        "fdw_operator_set_save": (i32, [vp, vp, i64, i32, i32]),
        "fdw_gradient_accumulate": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "fdw_operator_set_imaging_save": (i32, [vp, vp, i64, i32]),
        "fdw_operator_graph_stats": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "fdw_gradient_apply": (i32, [vp, i32, i32, i32, vp, i32, i64, vp, vp]),
        "fdw_batch_create": (i32, [pvp]),
        "fdw_batch_apply": (i32, [vp, ctypes.POINTER(vp), i32, ctypes.POINTER(i32), ctypes.POINTER(i32), vp]),
        "fdw_batch_stats": (i32, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "fdw_batch_destroy": (i32, [vp]),
        "fdw_server_create": (i32, [i64, i32, i32, pvp]),
        "fdw_server_footprint": (i32, [ctypes.POINTER(fdw_shot_desc), ctypes.POINTER(i64)]),
        "fdw_server_submit": (i32, [vp, ctypes.POINTER(fdw_shot_desc), ctypes.POINTER(i64)]),
        "fdw_server_progress": (i32, [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "fdw_server_info": (i32, [vp, i64, ctypes.POINTER(fdw_shot_info)]),
        "fdw_server_fetch": (i32, [vp, i64, vp, vp]),
        "fdw_server_release": (i32, [vp, i64]),
        "fdw_server_stats": (i32, [vp, ctypes.POINTER(fdw_server_stats_t)]),
        "fdw_server_destroy": (i32, [vp]),
        "fdw_bandwidth_probe": (i32, [i32, vp, vp, vp, ctypes.c_float, i64, vp]),
        "fdw_last_error": (ctypes.c_char_p, []),
        "fdw_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _chk(st: int):
    if st != FDW_OK:
        raise FdwError(st, load().fdw_last_error().decode())


def fdw_last_error() -> str:
    return load().fdw_last_error().decode()


def fdw_version() -> str:
    return load().fdw_version().decode()


def fdw_bandwidth_probe(kind: int, dst: int, a: int, b: int, s: float, n: int, stream: int = 0) -> None:
    """One launch of the copy (kind 0) or triad (kind 1) probe on device pointers."""
    _chk(load().fdw_bandwidth_probe(kind, dst, a, b or None, s, n, stream or None))


def fdw_stable_dt(kind: int, ndim: int, space_order: int, vmax: float, eps_max: float, hmin: float) -> float:
    return load().fdw_stable_dt(kind, ndim, space_order, vmax, eps_max, hmin)


def fdw_grid_create(shape, extent, origin=None) -> int:
    nd = len(shape)
    sh = (ctypes.c_int64 * 3)(*[int(s) for s in shape], *([1] * (3 - nd)))
    ex = (ctypes.c_double * 3)(*[float(e) for e in extent], *([0.0] * (3 - nd)))
    org = (ctypes.c_double * 3)(*[float(o) for o in origin], *([0.0] * (3 - nd))) if origin is not None else None
    out = ctypes.c_void_p()
    _chk(load().fdw_grid_create(nd, sh, ex, org, ctypes.byref(out)))
    return out.value


def fdw_grid_destroy(g):
    _chk(load().fdw_grid_destroy(g))


def fdw_field_layout(g, space_order: int) -> fdw_layout:
    lay = fdw_layout()
    _chk(load().fdw_field_layout(g, space_order, ctypes.byref(lay)))
    return lay


def fdw_function_bind(g, name: str, dptr: int, nelem: int, space_order: int) -> int:
    out = ctypes.c_void_p()
    _chk(load().fdw_function_bind(g, name.encode(), dptr, nelem, space_order, ctypes.byref(out)))
    return out.value


def fdw_function_destroy(f):
    _chk(load().fdw_function_destroy(f))


def fdw_timefunction_bind(g, name: str, dptr: int, nelem: int, space_order: int, time_order: int = 2,
                          nslots: int = 3) -> int:
    out = ctypes.c_void_p()
    _chk(load().fdw_timefunction_bind(g, name.encode(), dptr, nelem, space_order, time_order, nslots,
                                      ctypes.byref(out)))
    return out.value


def fdw_timefunction_destroy(f):
    _chk(load().fdw_timefunction_destroy(f))


def fdw_sparse_bind(g, name: str, coords: np.ndarray, nt: int, ddata: Optional[int]) -> int:
    c = np.ascontiguousarray(coords, dtype=np.float64)
    npoint = c.shape[0] if c.size else 0
    out = ctypes.c_void_p()
    cp = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if npoint else None
    _chk(load().fdw_sparse_bind(g, name.encode(), npoint, nt, cp, ddata, ctypes.byref(out)))
    return out.value


def fdw_sparse_bind_precomputed(g, name: str, gridpoints: np.ndarray, coeffs: np.ndarray, nt: int,
                                ddata: Optional[int]) -> int:
    """gridpoints [npoint][ndim] first support index per axis, coeffs
    [npoint][ndim][r] per-axis coefficients."""
    gp = np.ascontiguousarray(gridpoints, dtype=np.int64)
    cf = np.ascontiguousarray(coeffs, dtype=np.float64)
    npoint = gp.shape[0] if gp.size else 0
    r = cf.shape[-1] if cf.ndim == 3 else 0
    if npoint and (cf.ndim != 3 or cf.shape[:2] != gp.shape):
        raise ValueError(f"coeffs shape {cf.shape} does not match gridpoints {gp.shape}")
    out = ctypes.c_void_p()
    gptr = gp.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if npoint else None
    cptr = cf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if npoint else None
    _chk(load().fdw_sparse_bind_precomputed(g, name.encode(), npoint, nt, r if npoint else 2, gptr, cptr, ddata,
                                            ctypes.byref(out)))
    return out.value


def fdw_sparse_destroy(s):
    _chk(load().fdw_sparse_destroy(s))


def fdw_operator_create(desc: fdw_op_desc) -> int:
    out = ctypes.c_void_p()
    _chk(load().fdw_operator_create(ctypes.byref(desc), ctypes.byref(out)))
    return out.value


def fdw_operator_apply(op, time_m: int, time_M: int, stream: Optional[int] = None):
    _chk(load().fdw_operator_apply(op, time_m, time_M, stream))


def fdw_operator_apply_noalloc(op, time_m: int, time_M: int, stream: Optional[int] = None):
    _chk(load().fdw_operator_apply_noalloc(op, time_m, time_M, stream))


def fdw_sync(op):
    _chk(load().fdw_sync(op))


def fdw_operator_destroy(op):
    _chk(load().fdw_operator_destroy(op))


def fdw_operator_set_save(op, buf: Optional[int], nlevels: int = 0, every: int = 1, first_level: int = 0):
    _chk(load().fdw_operator_set_save(op, buf, nlevels, every, first_level))


def fdw_gradient_accumulate(op, nu: int, u_next: int, u_cur: int, u_prev: int, grad: int,
                            stream: Optional[int] = None):
    _chk(load().fdw_gradient_accumulate(op, nu, u_next, u_cur, u_prev, grad, stream))


def fdw_operator_graph_stats(op):
    """(graphs built, graph replays) of the operator's applies."""
    b, r = ctypes.c_int64(0), ctypes.c_int64(0)
    _chk(load().fdw_operator_graph_stats(op, ctypes.byref(b), ctypes.byref(r)))
    return b.value, r.value


def fdw_operator_set_imaging_save(op, buf: Optional[int], nsteps: int = 0, first_step: int = 0):
    _chk(load().fdw_operator_set_imaging_save(op, buf, nsteps, first_step))


def fdw_gradient_apply(adj, time_m: int, time_M: int, nt: int, imaging: int, first_step: int, nsteps: int,
                       grad: int, stream: Optional[int] = None):
    _chk(load().fdw_gradient_apply(adj, time_m, time_M, nt, imaging, first_step, nsteps, grad, stream))


def fdw_operator_set_timing(op, enable):
    """enable: False/0 off, True/1 each launch bracketed alone, k > 1 runs of k consecutive launches."""
    _chk(load().fdw_operator_set_timing(op, int(enable)))


def fdw_operator_kernel_time(op, reset: bool = True):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _chk(load().fdw_operator_kernel_time(op, ctypes.byref(ms), ctypes.byref(n), int(reset)))
    return ms.value, n.value


def fdw_operator_describe(op):
    buf = ctypes.create_string_buffer(512)
    b = ctypes.c_double()
    _chk(load().fdw_operator_describe(op, buf, 512, ctypes.byref(b)))
    return buf.value.decode(), b.value


# ---------------------------------------------------------------------------
# Padded-layout marshalling (torch tensors <-> logical numpy arrays)
# ---------------------------------------------------------------------------
def slot_view(flat, lay: fdw_layout, slot: int = 0):
    """Logical-domain view (numpy order: (nz, ny, nx) or (nz, nx)) of one slot."""
    E = lay.elems_per_slot
    R = lay.halo
    base = flat[slot * E:(slot + 1) * E]
    if lay.ndim == 3:
        v = base.view(lay.planes, lay.pitch_y, lay.pitch_x)
        nx, ny, nz = lay.shape[0], lay.shape[1], lay.shape[2]
        return v[R:R + nz, R:R + ny, FDW_X_OFFSET:FDW_X_OFFSET + nx]
    v = base.view(lay.pitch_y, lay.pitch_x)
    nx, nz = lay.shape[0], lay.shape[1]
    return v[R:R + nz, FDW_X_OFFSET:FDW_X_OFFSET + nx]


def alloc_field(lay: fdw_layout, nslots: int, device):
    """Zero-filled float32 tensor for nslots slots of this layout (256-byte aligned)."""
    import torch

    t = torch.zeros(nslots * lay.elems_per_slot, dtype=torch.float32, device=device)
    assert t.data_ptr() % 256 == 0
    return t


def upload(flat, lay: fdw_layout, slot: int, arr: np.ndarray):
    import torch

    v = slot_view(flat, lay, slot)
    v.copy_(torch.from_numpy(np.ascontiguousarray(arr, dtype=np.float32)))


def download(flat, lay: fdw_layout, slot: int) -> np.ndarray:
    return slot_view(flat, lay, slot).to("cpu").numpy().astype(np.float64)


class Shot:
    """One problem (paper_1807_03032_amd.workloads.Problem) bound on the GPU.

    Owns the torch tensors and the fdw handles; `apply` enqueues steps on the
    current torch stream; `fields()` / `traces()` fetch results.
    """

    def __init__(self, prob, device="cuda:0", u_init=None, nslots: int = 3):
        import torch

        self.prob = prob
        self.device = torch.device(device)
        kind = FDW_TTI if prob.kind == "tti" else FDW_ISO
        self.kind = kind
        self.handles = []
        self.grid = fdw_grid_create(prob.shape, prob.extent, prob.origin)
        self.lay = fdw_field_layout(self.grid, prob.so)
        E = self.lay.elems_per_slot
        self.wave = {}
        names = ["u"] if kind == FDW_ISO else ["p", "r"]
        self.tf = {}
        self.nslots = nslots
        for nm in names:
            t = alloc_field(self.lay, nslots, self.device)
            self.wave[nm] = t
            self.tf[nm] = fdw_timefunction_bind(self.grid, nm, t.data_ptr(), t.numel(), prob.so, 2, nslots)
        if u_init:
            for nm, (prev, cur) in u_init.items():
                upload(self.wave[nm], self.lay, nslots - 1, prev)  # level -1
                upload(self.wave[nm], self.lay, 0, cur)
        self.par = {}
        self.fn = {}
        for nm, arr in prob.fields.items():
            t = alloc_field(self.lay, 1, self.device)
            if nm == "m":
                t.fill_(1.0)  # keep 1/m finite outside the domain (never read)
            upload(t, self.lay, 0, arr)
            self.par[nm] = t
            self.fn[nm] = fdw_function_bind(self.grid, nm, t.data_ptr(), E, prob.so)
        nt = prob.nt
        self.src_data = torch.from_numpy(np.ascontiguousarray(prob.src, dtype=np.float32)).to(self.device)
        src_ptr = self.src_data.data_ptr() if self.src_data.numel() else None
        if getattr(prob, "src_pre", None) is not None:
            self.src = fdw_sparse_bind_precomputed(self.grid, "src", *prob.src_pre, nt, src_ptr)
        else:
            self.src = fdw_sparse_bind(self.grid, "src", prob.src_coords, nt, src_ptr)
        nrec = prob.rec_coords.shape[0]
        self.rec_data = torch.zeros((nt, max(nrec, 0)), dtype=torch.float32, device=self.device)
        rec_ptr = self.rec_data.data_ptr() if nrec else None
        if getattr(prob, "rec_pre", None) is not None:
            self.rec = fdw_sparse_bind_precomputed(self.grid, "rec", *prob.rec_pre, nt, rec_ptr)
        else:
            self.rec = fdw_sparse_bind(self.grid, "rec", prob.rec_coords, nt, rec_ptr)
        d = fdw_op_desc()
        d.kind = kind
        d.space_order = prob.so
        d.dt = prob.dt
        d.nbl = prob.nbl
        d.damp_rc = prob.rc
        d.vmax = prob.vmax
        d.eps_max = prob.eps_max
        d.u = self.tf[names[0]]
        d.r = self.tf["r"] if kind == FDW_TTI else None
        d.m = self.fn["m"]
        if kind == FDW_TTI:
            d.eps, d.delta, d.theta = self.fn["eps"], self.fn["delta"], self.fn["theta"]
            d.phi = self.fn.get("phi")
        d.src = self.src if prob.src_coords.size else None
        d.rec = self.rec if nrec else None
        self.op = fdw_operator_create(d)

    def apply(self, time_m: int = 0, time_M: Optional[int] = None, stream=None):
        import torch

        if time_M is None:
            time_M = self.prob.nt - 1
        s = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        fdw_operator_apply(self.op, time_m, time_M, s)

    def fields(self, t_last: int):
        """Levels t_last and t_last+1 of every wavefield as numpy float64."""
        import torch

        torch.cuda.synchronize(self.device)
        out = {}
        for nm, t in self.wave.items():
            S = self.nslots
            out[nm] = (download(t, self.lay, t_last % S), download(t, self.lay, (t_last + 1) % S))
        return out

    def traces(self) -> np.ndarray:
        import torch

        torch.cuda.synchronize(self.device)
        return self.rec_data.to("cpu").numpy().astype(np.float64)

    def close(self):
        if getattr(self, "op", None):
            fdw_operator_destroy(self.op)
            self.op = None
            fdw_sparse_destroy(self.src)
            fdw_sparse_destroy(self.rec)
            for h in list(self.tf.values()):
                fdw_timefunction_destroy(h)
            for h in list(self.fn.values()):
                fdw_function_destroy(h)
            fdw_grid_destroy(self.grid)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- batches
def fdw_batch_create() -> int:
    out = ctypes.c_void_p()
    _chk(load().fdw_batch_create(ctypes.byref(out)))
    return out.value


def fdw_batch_apply(b, ops, time_m, time_M, stream=None):
    n = len(ops)
    arr = (ctypes.c_void_p * n)(*ops)
    tm = (ctypes.c_int * n)(*[int(t) for t in time_m])
    tM = (ctypes.c_int * n)(*[int(t) for t in time_M])
    _chk(load().fdw_batch_apply(b, arr, n, tm, tM, stream))


def fdw_batch_stats(b):
    gb, gl = ctypes.c_int64(), ctypes.c_int64()
    _chk(load().fdw_batch_stats(b, ctypes.byref(gb), ctypes.byref(gl)))
    return gb.value, gl.value


def fdw_batch_destroy(b):
    _chk(load().fdw_batch_destroy(b))


# ----------------------------------------------------------------- server
def shot_desc(prob, keep_field: bool = False):
    """fdw_shot_desc of a workloads.Problem plus the numpy arrays it borrows
    (keep them alive until the shot is admitted)."""
    kind = FDW_TTI if prob.kind == "tti" else FDW_ISO
    d = fdw_shot_desc()
    nd = prob.ndim
    d.kind, d.ndim = kind, nd
    for a in range(3):
        d.shape[a] = int(prob.shape[a]) if a < nd else 1
        d.extent[a] = float(prob.extent[a]) if a < nd else 0.0
        d.origin[a] = float(prob.origin[a]) if a < nd else 0.0
    d.space_order, d.nt, d.dt, d.nbl = prob.so, prob.nt, prob.dt, prob.nbl
    d.damp_rc, d.vmax, d.eps_max = prob.rc, prob.vmax, prob.eps_max
    keep = []

    def f32p(a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        keep.append(a)
        return a.ctypes.data

    def f64p(a):
        a = np.ascontiguousarray(a, dtype=np.float64)
        keep.append(a)
        return a.ctypes.data

    d.m = f32p(prob.fields["m"])
    if kind == FDW_TTI:
        d.eps, d.delta, d.theta = (f32p(prob.fields[k]) for k in ("eps", "delta", "theta"))
        d.phi = f32p(prob.fields["phi"]) if nd == 3 else None
    d.nsrc = prob.src_coords.shape[0]
    if d.nsrc:
        d.src_coords = f64p(prob.src_coords)
        d.src = f32p(prob.src)
    d.nrec = prob.rec_coords.shape[0]
    if d.nrec:
        d.rec_coords = f64p(prob.rec_coords)
    d.keep_field = 1 if keep_field else 0
    return d, keep


class Server:
    """Thin wrapper of the fdw_server C ABI."""

    def __init__(self, budget_bytes: int = 0, chunk_target_us: int = 0, nstreams: int = 4):
        out = ctypes.c_void_p()
        _chk(load().fdw_server_create(int(budget_bytes), int(chunk_target_us), int(nstreams), ctypes.byref(out)))
        self.h = out.value
        self.borrowed = {}
        self.meta = {}

    @staticmethod
    def footprint(prob) -> int:
        d, _ = shot_desc(prob)
        out = ctypes.c_int64()
        _chk(load().fdw_server_footprint(ctypes.byref(d), ctypes.byref(out)))
        return out.value

    def submit(self, prob, keep_field: bool = False) -> int:
        d, keep = shot_desc(prob, keep_field)
        t = ctypes.c_int64()
        _chk(load().fdw_server_submit(self.h, ctypes.byref(d), ctypes.byref(t)))
        self.borrowed[t.value] = keep
        self.meta[t.value] = (prob.nt, prob.rec_coords.shape[0], prob.array_shape)
        return t.value

    def progress(self):
        q, r = ctypes.c_int(), ctypes.c_int()
        _chk(load().fdw_server_progress(self.h, ctypes.byref(q), ctypes.byref(r)))
        # host arrays of admitted shots are no longer borrowed
        for t in [t for t in self.borrowed if self.info(t).state != FDW_SHOT_QUEUED]:
            del self.borrowed[t]
        return q.value, r.value

    def info(self, ticket: int) -> fdw_shot_info:
        out = fdw_shot_info()
        _chk(load().fdw_server_info(self.h, int(ticket), ctypes.byref(out)))
        return out

    def fetch(self, ticket: int, field: bool = False):
        nt, nrec, ash = self.meta[ticket]
        rec = np.zeros((nt, nrec), dtype=np.float32)
        fld = np.zeros(ash, dtype=np.float32) if field else None
        _chk(load().fdw_server_fetch(self.h, int(ticket), rec.ctypes.data if nrec else None,
                                     fld.ctypes.data if field else None))
        return rec, fld

    def release(self, ticket: int):
        _chk(load().fdw_server_release(self.h, int(ticket)))
        self.meta.pop(ticket, None)

    def stats(self) -> dict:
        out = fdw_server_stats_t()
        _chk(load().fdw_server_stats(self.h, ctypes.byref(out)))
        return {k: getattr(out, k) for k, _ in out._fields_}

    def close(self):
        if self.h:
            _chk(load().fdw_server_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
