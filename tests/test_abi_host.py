"""CPU tests of the C ABI: the library loads and exports every symbol that
include/fdw.h declares, and the host-side validation, layout arithmetic and
stability bound behave as documented.  No call here reaches the device: every
error path tested returns before any HIP runtime call, and pointers passed in
are never dereferenced on the host."""
import math
import os
import re

import numpy as np
import pytest

from paper_1807_03032_amd import fdw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdw.h")


@pytest.fixture(scope="module", autouse=True)
def lib():
    if not os.path.exists(fdw.LIB_PATH):
        from paper_1807_03032_amd import build
        build.build()
    return fdw.load()


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdw_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    syms = declared_symbols()
    assert len(syms) >= 19
    assert set(syms) == set(fdw.EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


def test_version_and_empty_error():
    assert "fdw" in fdw.fdw_version()


def test_grid_validation():
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_grid_create((10,), (1.0,))
    assert e.value.code == fdw.FDW_ERR_ARG
    with pytest.raises(fdw.FdwError):
        fdw.fdw_grid_create((1, 10), (1.0, 1.0))
    with pytest.raises(fdw.FdwError):
        fdw.fdw_grid_create((10, 10), (0.0, 1.0))
    g = fdw.fdw_grid_create((10, 12, 14), (90.0, 110.0, 130.0), (1.0, 2.0, 3.0))
    fdw.fdw_grid_destroy(g)


@pytest.mark.parametrize("shape,so", [((101, 101), 4), ((256, 256, 256), 8), ((37, 29, 23), 12), ((5, 3), 16)])
def test_layout_arithmetic(shape, so):
    g = fdw.fdw_grid_create(shape, tuple(10.0 * (s - 1) for s in shape))
    lay = fdw.fdw_field_layout(g, so)
    R = so // 2
    assert lay.halo == R
    assert lay.pitch_x % 32 == 0 and lay.pitch_x >= fdw.FDW_X_OFFSET + shape[0] + R
    if len(shape) == 3:
        assert lay.pitch_y == shape[1] + 2 * R and lay.planes == shape[2] + 2 * R
        assert lay.origin_offset == (R * lay.pitch_y + R) * lay.pitch_x + fdw.FDW_X_OFFSET
    else:
        assert lay.pitch_y == shape[1] + 2 * R and lay.planes == 1
        assert lay.origin_offset == R * lay.pitch_x + fdw.FDW_X_OFFSET
    assert lay.elems_per_slot == lay.pitch_x * lay.pitch_y * lay.planes
    assert (lay.origin_offset * 4) % 128 == 0  # logical x = 0 is 128-byte aligned
    with pytest.raises(fdw.FdwError):
        fdw.fdw_field_layout(g, 3)
    with pytest.raises(fdw.FdwError):
        fdw.fdw_field_layout(g, 18)
    fdw.fdw_grid_destroy(g)


@pytest.mark.parametrize("so,lam", [(2, 4.0), (4, 16 / 3), (8, None), (16, None)])
def test_stable_dt(so, lam):
    """dt_max = 2 / (v sqrt(d lambda_so) / h), lambda_so the largest symbol of
    -d2/dx2 (at the Nyquist wavenumber): 4 for so = 2, 16/3 for so = 4."""
    if lam is None:
        import brute
        w = brute.taylor_w2(so // 2)
        lam = float(-(w[0] + 2 * sum(w[k] * (-1) ** k for k in range(1, so // 2 + 1))))
    dt = fdw.fdw_stable_dt(fdw.FDW_ISO, 3, so, 2000.0, 0.0, 10.0)
    assert abs(dt - 2 * 10.0 / (2000.0 * math.sqrt(3 * lam))) < 1e-12 * dt
    dtt = fdw.fdw_stable_dt(fdw.FDW_TTI, 3, so, 2000.0, 0.3, 10.0)
    assert abs(dtt - dt / math.sqrt(1.6)) < 1e-12 * dt
    assert fdw.fdw_stable_dt(fdw.FDW_ISO, 3, 5, 2000.0, 0.0, 10.0) < 0


def test_bind_validation_without_device():
    g = fdw.fdw_grid_create((20, 18, 16), (190.0, 170.0, 150.0))
    lay = fdw.fdw_field_layout(g, 8)
    fake = 0x7F0000000000  # never dereferenced by the host code
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_function_bind(g, "m", fake + 4, lay.elems_per_slot, 8)
    assert e.value.code == fdw.FDW_ERR_LAYOUT
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_function_bind(g, "m", fake, lay.elems_per_slot - 1, 8)
    assert e.value.code == fdw.FDW_ERR_LAYOUT
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_timefunction_bind(g, "u", fake, 2 * lay.elems_per_slot, 8)
    assert e.value.code == fdw.FDW_ERR_LAYOUT
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_timefunction_bind(g, "u", fake, 3 * lay.elems_per_slot, 8, time_order=1)
    assert e.value.code == fdw.FDW_ERR_ARG
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_timefunction_bind(g, "u", fake, 4 * lay.elems_per_slot, 8, nslots=4)
    assert e.value.code == fdw.FDW_ERR_ARG
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_timefunction_bind(g, "u", fake, 2 * lay.elems_per_slot - 1, 8, nslots=2)
    assert e.value.code == fdw.FDW_ERR_LAYOUT
    t2 = fdw.fdw_timefunction_bind(g, "u", fake, 2 * lay.elems_per_slot, 8, nslots=2)
    fdw.fdw_timefunction_destroy(t2)
    f = fdw.fdw_function_bind(g, "m", fake, lay.elems_per_slot, 8)
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_grid_destroy(g)  # still referenced
    assert e.value.code == fdw.FDW_ERR_STATE
    fdw.fdw_function_destroy(f)
    fdw.fdw_grid_destroy(g)


def test_sparse_domain_check():
    g = fdw.fdw_grid_create((11, 11), (100.0, 100.0), (5.0, 0.0))
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_sparse_bind(g, "src", np.array([[4.9, 50.0]]), 10, 0x7F0000000000)
    assert e.value.code == fdw.FDW_ERR_DOMAIN
    assert "outside" in fdw.fdw_last_error()
    s = fdw.fdw_sparse_bind(g, "src", np.array([[105.0, 100.0], [5.0, 0.0]]), 10, 0x7F0000000000)
    fdw.fdw_sparse_destroy(s)
    fdw.fdw_grid_destroy(g)


def _desc(kind, so, dt, u=None, r=None, m=None, **kw):
    d = fdw.fdw_op_desc()
    d.kind, d.space_order, d.dt, d.nbl, d.vmax = kind, so, dt, 10, 2000.0
    d.u, d.r, d.m = u, r, m
    for k, v in kw.items():
        setattr(d, k, v)
    return d


def test_operator_create_validation_without_device():
    g = fdw.fdw_grid_create((20, 18, 16), (190.0, 170.0, 150.0))
    lay = fdw.fdw_field_layout(g, 8)
    fake = 0x7F0000000000
    E = lay.elems_per_slot
    u = fdw.fdw_timefunction_bind(g, "u", fake, 3 * E, 8)
    m = fdw.fdw_function_bind(g, "m", fake, E, 8)
    m4 = fdw.fdw_function_bind(g, "m4", fake, fdw.fdw_field_layout(g, 4).elems_per_slot, 4)
    dt_ok = 0.9 * fdw.fdw_stable_dt(fdw.FDW_ISO, 3, 8, 2000.0, 0.0, 10.0)

    def code(d):
        with pytest.raises(fdw.FdwError) as e:
            fdw.fdw_operator_create(d)
        return e.value.code

    assert code(_desc(fdw.FDW_ISO, 8, 1.2 * dt_ok / 0.9, u, None, m)) == fdw.FDW_ERR_UNSTABLE
    assert code(_desc(fdw.FDW_ISO, 8, dt_ok, u, None, None)) == fdw.FDW_ERR_ARG
    assert code(_desc(fdw.FDW_ISO, 8, dt_ok, u, None, m4)) == fdw.FDW_ERR_LAYOUT
    assert code(_desc(fdw.FDW_ISO, 6, dt_ok, u, None, m)) == fdw.FDW_ERR_LAYOUT
    assert code(_desc(fdw.FDW_ISO, 8, -1.0, u, None, m)) == fdw.FDW_ERR_ARG
    assert code(_desc(fdw.FDW_TTI, 8, dt_ok, u, None, m)) == fdw.FDW_ERR_ARG  # r missing
    assert code(_desc(7, 8, dt_ok, u, None, m)) == fdw.FDW_ERR_ARG
    for h in (u,):
        fdw.fdw_timefunction_destroy(h)
    fdw.fdw_function_destroy(m)
    fdw.fdw_function_destroy(m4)
    fdw.fdw_grid_destroy(g)


def test_binding_fails_loudly_without_library(tmp_path):
    import importlib
    mod = importlib.import_module("paper_1807_03032_amd.fdw")
    saved = mod._lib
    try:
        mod._lib = None
        with pytest.raises(ImportError):
            mod.load(str(tmp_path / "missing.so"))
    finally:
        mod._lib = saved


def test_precomputed_sparse_validation():
    g = fdw.fdw_grid_create((12, 10, 9), (110.0, 90.0, 80.0))
    fake = 0x7F0000000000
    gp = np.array([[3, 2, 1]], dtype=np.int64)
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_sparse_bind_precomputed(g, "s", gp, np.full((1, 3, 5), 0.2), 10, fake)  # r = 5 > max
    assert e.value.code == fdw.FDW_ERR_ARG
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_sparse_bind_precomputed(g, "s", np.array([[9, 2, 1]]), np.full((1, 3, 4), 0.25), 10, fake)
    assert e.value.code == fdw.FDW_ERR_DOMAIN  # x support 9..12 leaves the 12-point axis
    assert "outside" in fdw.fdw_last_error()
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_sparse_bind_precomputed(g, "s", np.array([[0, -1, 1]]), np.full((1, 3, 2), 0.5), 10, fake)
    assert e.value.code == fdw.FDW_ERR_DOMAIN
    s = fdw.fdw_sparse_bind_precomputed(g, "s", np.array([[8, 6, 5]]), np.full((1, 3, 4), 0.25), 10, fake)
    fdw.fdw_sparse_destroy(s)
    fdw.fdw_grid_destroy(g)


@pytest.mark.parametrize("kind,ndim,n,so", [("iso", 3, 64, 8), ("tti", 3, 48, 12), ("iso", 2, 201, 4), ("tti", 2, 97, 16)])
def test_server_footprint(kind, ndim, n, so):
    """Device bytes of a served shot: two slots per wavefield, the model
    parameters, TTI stage buffers, source / receiver samples and small tables."""
    from paper_1807_03032_amd import workloads as W
    prob = W.serve_problem(kind, ndim, n, so, 30, seed=1, nbl=10)
    got = fdw.Server.footprint(prob)
    g = fdw.fdw_grid_create(prob.shape, prob.extent)
    E = fdw.fdw_field_layout(g, so).elems_per_slot
    fdw.fdw_grid_destroy(g)
    slots = {"iso": 2 + 1, "tti": 4 + (5 if ndim == 3 else 4) + 2}[kind]
    nrec = prob.rec_coords.shape[0]
    floats = slots * E + 30 * (1 + nrec) + ndim * n + (1 + nrec) * (2 + 2 ** ndim + 3)
    assert got == 4 * floats + 64 * 256


def test_server_footprint_validation():
    from paper_1807_03032_amd import workloads as W
    prob = W.serve_problem("iso", 2, 50, 8, 10, seed=2, nbl=5)
    d, keep = fdw.shot_desc(prob)
    d.kind = 5
    import ctypes
    out = ctypes.c_int64()
    assert fdw.load().fdw_server_footprint(ctypes.byref(d), ctypes.byref(out)) == fdw.FDW_ERR_ARG
    d.kind, d.space_order = fdw.FDW_ISO, 7
    assert fdw.load().fdw_server_footprint(ctypes.byref(d), ctypes.byref(out)) == fdw.FDW_ERR_ARG
    assert "space order" in fdw.fdw_last_error() or "space_order" in fdw.fdw_last_error()


def test_bandwidth_probe_validation(lib):
    """Argument checks happen before any device call (no GPU needed)."""
    for args in ((2, 64, 64, 64, 16), (0, 0, 64, 64, 16), (1, 64, 64, 0, 16), (0, 64, 64, 64, 6),
                 (0, 68, 64, 64, 16), (1, 64, 64, 72, 16)):
        kind, dst, a, b, n = args
        with pytest.raises(fdw.FdwError) as e:
            fdw.fdw_bandwidth_probe(kind, dst, a, b, 1.0, n)
        assert e.value.code == fdw.FDW_ERR_ARG, args


def test_imaging_entry_points_validate_without_device(lib):
    """NULL operators and buffers are refused before any device call."""
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_operator_set_imaging_save(None, 256, 4, 0)
    assert e.value.code == fdw.FDW_ERR_ARG
    with pytest.raises(fdw.FdwError) as e:
        fdw.fdw_gradient_apply(None, 0, 3, 4, 256, 0, 4, 512)
    assert e.value.code == fdw.FDW_ERR_ARG
