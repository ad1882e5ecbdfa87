"""FP64 CPU oracle for the finite-difference wave-equation operators.

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check in
``__graft_entry__.py`` and by the CPU-baseline leg of ``bench.py``.  The HIP
product path never imports, links or calls anything here, and shares no code
with it.

This module is a thin ctypes wrapper over ``fdw_oracle.c`` (plain C, OpenMP
over the outermost axis, no blocking).  Arrays are numpy float64 in logical
layout with the FIRST axis fastest, i.e. a numpy array of shape
``(nz, ny, nx)`` for a 3D grid with axes (x, y, z), ``(nz, nx)`` for 2D
(x, z) and ``(nx,)`` for 1D.

Paper: arXiv 1807.03032, Section 3 (symbolic API: eq. WE, Listings fd-1..fd-3,
eq. interp, Listing finject) and Section 7.2 (test-case setup).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_DOMAIN, ERR_NOMEM = 0, -1, -2, -3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math: IEEE FP64 throughout)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
             "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_long * 3), ("h", ctypes.c_double * 3),
                ("o", ctypes.c_double * 3), ("so", ctypes.c_int), ("dt", ctypes.c_double),
                ("nbl", ctypes.c_int), ("vmax", ctypes.c_double), ("rc", ctypes.c_double),
                ("periodic", ctypes.c_int)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
    return _lib


class OracleError(RuntimeError):
    pass


def _check(st, what):
    if st != OK:
        raise OracleError(f"{what}: oracle status {st}")


_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


class Grid:
    """Grid description (Section 3.1: Grid(shape, extent, origin)).

    shape/extent/origin are given in axis order (x,), (x, z) or (x, y, z);
    spacing h_a = extent_a / (shape_a - 1).
    """

    def __init__(self, shape, extent, origin=None, so=4, dt=1.0, nbl=0, vmax=0.0, rc=1e-3,
                 periodic=False):
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.extent = tuple(float(e) for e in extent)
        self.origin = tuple(float(o) for o in (origin if origin is not None else (0.0,) * self.ndim))
        self.spacing = tuple(e / (s - 1) for e, s in zip(self.extent, self.shape))
        self.so, self.dt, self.nbl, self.vmax, self.rc = int(so), float(dt), int(nbl), float(vmax), float(rc)
        self.periodic = bool(periodic)

    @property
    def array_shape(self):
        """numpy shape of a logical field: reversed axis order, first axis fastest."""
        return tuple(reversed(self.shape))

    def c(self):
        g = _Grid()
        g.ndim = self.ndim
        for a in range(3):
            g.n[a] = self.shape[a] if a < self.ndim else 1
            g.h[a] = self.spacing[a] if a < self.ndim else 1.0
            g.o[a] = self.origin[a] if a < self.ndim else 0.0
        g.so, g.dt, g.nbl, g.vmax, g.rc = self.so, self.dt, self.nbl, self.vmax, self.rc
        g.periodic = int(self.periodic)
        return g


def _field(grid, a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if a.shape != grid.array_shape:
        raise ValueError(f"field shape {a.shape} != {grid.array_shape}")
    return a


def num_threads() -> int:
    """OpenMP threads the oracle's loops use."""
    return int(_load().or_num_threads())


def fd_weights(so: int, deriv: int) -> np.ndarray:
    """Weights w[0..R] of the centred stencil of order so for d^deriv/dx^deriv."""
    w = np.zeros(so // 2 + 1)
    _check(_load().or_fd_weights(ctypes.c_int(so), ctypes.c_int(deriv), _ptr(w)), "fd_weights")
    return w


def laplacian(grid: Grid, u) -> np.ndarray:
    u = _field(grid, u)
    out = np.empty_like(u)
    g = grid.c()
    _check(_load().or_laplacian(ctypes.byref(g), _ptr(u), _ptr(out)), "laplacian")
    return out


def deriv1(grid: Grid, axis: int, u) -> np.ndarray:
    u = _field(grid, u)
    out = np.empty_like(u)
    g = grid.c()
    _check(_load().or_deriv1(ctypes.byref(g), ctypes.c_int(axis), _ptr(u), _ptr(out)), "deriv1")
    return out


def damping(grid: Grid) -> np.ndarray:
    out = np.empty(grid.array_shape)
    g = grid.c()
    _check(_load().or_damping(ctypes.byref(g), _ptr(out)), "damping")
    return out


def _coords(grid, c):
    c = np.ascontiguousarray(np.asarray(c, dtype=np.float64).reshape(-1, grid.ndim))
    return c


def sparse_setup(grid: Grid, coords):
    c = _coords(grid, coords)
    n = c.shape[0]
    base = np.zeros((n, grid.ndim), dtype=np.int64)
    w = np.zeros((n, 1 << grid.ndim))
    g = grid.c()
    st = _load().or_sparse_setup(ctypes.byref(g), ctypes.c_int(n), _ptr(c),
                                 base.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _ptr(w))
    _check(st, "sparse_setup")
    return base, w


def interp(grid: Grid, coords, u) -> np.ndarray:
    c = _coords(grid, coords)
    u = _field(grid, u)
    out = np.zeros(c.shape[0])
    g = grid.c()
    _check(_load().or_interp(ctypes.byref(g), ctypes.c_int(c.shape[0]), _ptr(c), _ptr(u), _ptr(out)),
           "interp")
    return out


def inject(grid: Grid, coords, q, u, scale=1.0, m=None) -> np.ndarray:
    """Returns a copy of u with scale*w*q/m scattered in (m=None: divisor 1)."""
    c = _coords(grid, coords)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    u = _field(grid, u).copy()
    mm = _field(grid, m) if m is not None else None
    g = grid.c()
    _check(_load().or_inject(ctypes.byref(g), ctypes.c_int(c.shape[0]), _ptr(c), _ptr(q),
                             ctypes.c_double(scale), _ptr(mm), _ptr(u)), "inject")
    return u


def _pre(grid, gridpoints, coeffs):
    gp = np.ascontiguousarray(np.asarray(gridpoints, dtype=np.int64).reshape(-1, grid.ndim))
    cf = np.ascontiguousarray(np.asarray(coeffs, dtype=np.float64))
    if cf.ndim != 3 or cf.shape[:2] != gp.shape:
        raise ValueError(f"coeffs shape {cf.shape} does not match gridpoints {gp.shape}")
    return gp, cf, int(cf.shape[2])


def _lptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_long)) if a is not None else None


def interp_pre(grid: Grid, gridpoints, coeffs, u) -> np.ndarray:
    """Precomputed sparse points: out[p] = sum over the r^d support points."""
    gp, cf, r = _pre(grid, gridpoints, coeffs)
    u = _field(grid, u)
    out = np.zeros(gp.shape[0])
    g = grid.c()
    _check(_load().or_interp_pre(ctypes.byref(g), ctypes.c_int(gp.shape[0]), ctypes.c_int(r), _lptr(gp), _ptr(cf),
                                 _ptr(u), _ptr(out)), "interp_pre")
    return out


def inject_pre(grid: Grid, gridpoints, coeffs, q, u, scale=1.0, m=None) -> np.ndarray:
    gp, cf, r = _pre(grid, gridpoints, coeffs)
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(-1)
    u = _field(grid, u).copy()
    mm = _field(grid, m) if m is not None else None
    g = grid.c()
    _check(_load().or_inject_pre(ctypes.byref(g), ctypes.c_int(gp.shape[0]), ctypes.c_int(r), _lptr(gp), _ptr(cf),
                                 _ptr(q), ctypes.c_double(scale), _ptr(mm), _ptr(u)), "inject_pre")
    return u


def iso_run_pre(grid: Grid, m, nt: int, src_pre, src, rec_pre, u_prev=None, u_cur=None, time_m: int = 0,
                time_M: int | None = None):
    """iso_run with precomputed sparse points: src_pre / rec_pre are
    (gridpoints, coeffs) pairs or None."""
    if time_M is None:
        time_M = nt - 1
    m = _field(grid, m)
    up = _field(grid, u_prev).copy() if u_prev is not None else np.zeros(grid.array_shape)
    uc = _field(grid, u_cur).copy() if u_cur is not None else np.zeros(grid.array_shape)
    ns, sr, sgp, scf, sd = 0, 1, None, None, None
    if src_pre is not None:
        sgp, scf, sr = _pre(grid, *src_pre)
        ns = sgp.shape[0]
        sd = np.ascontiguousarray(src, dtype=np.float64)
        if sd.shape != (nt, ns):
            raise ValueError(f"src data shape {sd.shape} != {(nt, ns)}")
    nr, rr, rgp, rcf = 0, 1, None, None
    if rec_pre is not None:
        rgp, rcf, rr = _pre(grid, *rec_pre)
        nr = rgp.shape[0]
    rec = np.zeros((nt, nr))
    g = grid.c()
    st = _load().or_iso_run_pre(ctypes.byref(g), _ptr(m), ctypes.c_int(time_m), ctypes.c_int(time_M), _ptr(up),
                                _ptr(uc), ctypes.c_int(ns), ctypes.c_int(sr), _lptr(sgp), _ptr(scf), _ptr(sd),
                                ctypes.c_int(nr), ctypes.c_int(rr), _lptr(rgp), _ptr(rcf),
                                _ptr(rec) if nr else None)
    _check(st, "iso_run_pre")
    return up, uc, rec


def rotated_h(grid: Grid, theta, phi, u) -> np.ndarray:
    u = _field(grid, u)
    th = _field(grid, theta)
    ph = _field(grid, phi) if grid.ndim == 3 else None
    out = np.empty_like(u)
    g = grid.c()
    _check(_load().or_rotated_h(ctypes.byref(g), _ptr(th), _ptr(ph), _ptr(u), _ptr(out)), "rotated_h")
    return out


def _sparse_args(grid, coords, data, nt, name):
    if coords is None or len(np.asarray(coords).reshape(-1)) == 0:
        return 0, None, None
    c = _coords(grid, coords)
    if data is None:
        return c.shape[0], c, None
    d = np.ascontiguousarray(data, dtype=np.float64)
    if d.shape != (nt, c.shape[0]):
        raise ValueError(f"{name} data shape {d.shape} != {(nt, c.shape[0])}")
    return c.shape[0], c, d


def iso_run(grid: Grid, m, nt: int, u_prev=None, u_cur=None, src_coords=None, src=None,
            rec_coords=None, time_m: int = 0, time_M: int | None = None):
    """Run the isotropic operator for steps time_m..time_M (default 0..nt-1).

    Returns (u_prev, u_cur, rec) = (level time_M, level time_M+1, rec[nt][nrec]).
    """
    if time_M is None:
        time_M = nt - 1
    m = _field(grid, m)
    up = _field(grid, u_prev).copy() if u_prev is not None else np.zeros(grid.array_shape)
    uc = _field(grid, u_cur).copy() if u_cur is not None else np.zeros(grid.array_shape)
    ns, sc, sd = _sparse_args(grid, src_coords, src, nt, "src")
    if ns and sd is None:
        raise ValueError("src data required with src_coords")
    nr, rc, _ = _sparse_args(grid, rec_coords, None, nt, "rec")
    rec = np.zeros((nt, nr))
    g = grid.c()
    st = _load().or_iso_run(ctypes.byref(g), _ptr(m), ctypes.c_int(time_m), ctypes.c_int(time_M),
                            _ptr(up), _ptr(uc), ctypes.c_int(ns), _ptr(sc), _ptr(sd), ctypes.c_int(nr),
                            _ptr(rc), _ptr(rec) if nr else None)
    _check(st, "iso_run")
    return up, uc, rec


def tti_run(grid: Grid, m, eps, delta, theta, phi, nt: int, p_prev=None, p_cur=None, r_prev=None,
            r_cur=None, src_coords=None, src=None, rec_coords=None, time_m: int = 0,
            time_M: int | None = None):
    """Run the TTI operator; returns (p_prev, p_cur, r_prev, r_cur, rec)."""
    if time_M is None:
        time_M = nt - 1
    m, eps, delta, theta = (_field(grid, a) for a in (m, eps, delta, theta))
    phi = _field(grid, phi) if grid.ndim == 3 else None
    z = lambda a: _field(grid, a).copy() if a is not None else np.zeros(grid.array_shape)  # noqa: E731
    pp, pc, rp, rcur = z(p_prev), z(p_cur), z(r_prev), z(r_cur)
    ns, sc, sd = _sparse_args(grid, src_coords, src, nt, "src")
    if ns and sd is None:
        raise ValueError("src data required with src_coords")
    nr, rc, _ = _sparse_args(grid, rec_coords, None, nt, "rec")
    rec = np.zeros((nt, nr))
    g = grid.c()
    st = _load().or_tti_run(ctypes.byref(g), _ptr(m), _ptr(eps), _ptr(delta), _ptr(theta), _ptr(phi),
                            ctypes.c_int(time_m), ctypes.c_int(time_M), _ptr(pp), _ptr(pc), _ptr(rp),
                            _ptr(rcur), ctypes.c_int(ns), _ptr(sc), _ptr(sd), ctypes.c_int(nr), _ptr(rc),
                            _ptr(rec) if nr else None)
    _check(st, "tti_run")
    return pp, pc, rp, rcur, rec


def iso_adjoint(grid: Grid, m, nt: int, src_coords, rec_coords, resid) -> np.ndarray:
    """Transpose of the source-to-receiver map of iso_run (zero initial levels):
    resid [nt][nrec] -> [nt][nsrc]."""
    m = _field(grid, m)
    sc, rc = _coords(grid, src_coords), _coords(grid, rec_coords)
    d = np.ascontiguousarray(resid, dtype=np.float64)
    assert d.shape == (nt, rc.shape[0])
    out = np.zeros((nt, sc.shape[0]))
    g = grid.c()
    _check(_load().or_iso_adjoint(ctypes.byref(g), _ptr(m), ctypes.c_int(nt), ctypes.c_int(sc.shape[0]), _ptr(sc),
                                  ctypes.c_int(rc.shape[0]), _ptr(rc), _ptr(d), _ptr(out)), "iso_adjoint")
    return out


def iso_gradient(grid: Grid, m, nt: int, src_coords, src, rec_coords, resid) -> np.ndarray:
    """d/dm of sum_t <resid[t], rec[t]> for the forward run of iso_run."""
    m = _field(grid, m)
    sc, rc = _coords(grid, src_coords), _coords(grid, rec_coords)
    q = np.ascontiguousarray(src, dtype=np.float64)
    d = np.ascontiguousarray(resid, dtype=np.float64)
    assert q.shape == (nt, sc.shape[0]) and d.shape == (nt, rc.shape[0])
    out = np.zeros(grid.array_shape)
    g = grid.c()
    _check(_load().or_iso_gradient(ctypes.byref(g), _ptr(m), ctypes.c_int(nt), ctypes.c_int(sc.shape[0]), _ptr(sc),
                                   _ptr(q), ctypes.c_int(rc.shape[0]), _ptr(rc), _ptr(d), _ptr(out)),
           "iso_gradient")
    return out
