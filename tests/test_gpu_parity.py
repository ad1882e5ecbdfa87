"""GPU parity: the HIP operators (called through the C ABI) against the FP64
oracle on identical seeded inputs.

Bar (written here, from the target accuracy of the operators): relative L2
error <= 1e-4, computed in FP64, separately for each of the last two time
levels of every wavefield over the domain and for the receiver traces.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1807_03032_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_1807_03032_amd import fdw
    fdw.load()
    return torch.device("cuda:0")


def gpu_run(prob, dev, splits=None, u_init=None, time_M=None, nslots=3):
    from paper_1807_03032_amd import fdw
    shot = fdw.Shot(prob, dev, u_init=u_init, nslots=nslots)
    try:
        if splits:
            lo = 0
            for hi in splits + [prob.nt - 1]:
                shot.apply(lo, hi)
                lo = hi + 1
        elif time_M == -1:
            shot.apply(0, -1)
        else:
            shot.apply(0, prob.nt - 1)
        f = shot.fields(prob.nt - 1)
        tr = shot.traces()
        desc = fdw.fdw_operator_describe(shot.op)[0]
    finally:
        shot.close()
    return f, tr, desc


def oracle_run(prob, u_init=None):
    g = oracle.Grid(prob.shape, prob.extent, prob.origin, so=prob.so, dt=prob.dt, nbl=prob.nbl, vmax=prob.vmax,
                    rc=prob.rc)
    f = prob.fields
    if prob.kind == "iso":
        ui = (u_init or {}).get("u", (None, None))
        up, uc, rec = oracle.iso_run(g, f["m"], prob.nt, ui[0], ui[1], src_coords=prob.src_coords, src=prob.src,
                                     rec_coords=prob.rec_coords)
        return {"u": (up, uc)}, rec
    pi = (u_init or {}).get("p", (None, None))
    ri = (u_init or {}).get("r", (None, None))
    pp, pc, rp, rc, rec = oracle.tti_run(g, f["m"], f["eps"], f["delta"], f["theta"], f.get("phi"), prob.nt, pi[0],
                                         pi[1], ri[0], ri[1], src_coords=prob.src_coords, src=prob.src,
                                         rec_coords=prob.rec_coords)
    return {"p": (pp, pc), "r": (rp, rc)}, rec


def check(prob, gf, gtr, of, otr, tol=TOL):
    errs = {}
    for nm, (ref_prev, ref_cur) in of.items():
        errs[f"{nm}_prev"] = rel_l2(gf[nm][0], ref_prev)
        errs[f"{nm}_cur"] = rel_l2(gf[nm][1], ref_cur)
    if otr.size:
        errs["rec"] = rel_l2(gtr, otr)
    say(prob.name, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= tol, (prob.name, k, v)
    for nm, (ref_prev, ref_cur) in of.items():
        assert np.linalg.norm(ref_cur) > 0, "degenerate case: reference field is zero"
    return errs


# ---------------------------------------------------------------- small grids
@pytest.mark.parametrize("so", [2, 4, 8, 12, 16])
@pytest.mark.parametrize("shape", [(67, 45), (37, 29, 23)])
def test_iso_small(torch_dev, shape, so):
    prob = W.small_problem("iso", shape, so, nt=40, seed=so, nsrc=2, nrec=16, nbl=4)
    say("iso", shape, so)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("so", [4, 8, 12, 16])
@pytest.mark.parametrize("shape", [(53, 41), (33, 27, 21)])
def test_tti_small(torch_dev, shape, so):
    prob = W.small_problem("tti", shape, so, nt=30, seed=50 + so, nsrc=1, nrec=12, nbl=4)
    say("tti", shape, so)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("so", [8, 12, 16])
def test_tti_multitile_full_grid(torch_dev, so):
    """150 x 70 x 90, 30 steps, every element compared: three 64-wide x-tiles,
    several y-tiles of both stages and several z-chunks, so the halo exchange
    between x-tiles, y-tiles and chunks of stage 1 and stage 2 is checked
    everywhere, not on samples."""
    prob = W.small_problem("tti", (150, 70, 90), so, nt=30, seed=300 + so, nsrc=2, nrec=40, nbl=6)
    say("tti multi-tile", prob.shape, so)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert "tti3d_stream" in desc, desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("shape", [(150, 70, 90), (91, 77)])
def test_tti_angles_full_turn(torch_dev, shape):
    """theta and phi drawn over [0, 2 pi): every sign of every component of
    the symmetry axis, through the hardware sine and cosine."""
    prob = W.small_problem("tti", shape, 12, nt=30, seed=321, nsrc=1, nrec=30, nbl=6,
                           angle_range=(0.0, 2.0 * np.pi))
    th = prob.fields["theta"]
    assert th.min() < 0.5 and th.max() > 5.5, (th.min(), th.max())
    say("tti full-turn angles", shape)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("shape,so,nt,splits", [((150, 70, 90), 8, 24, None), ((61, 53, 47), 4, 17, None),
                                                 ((100, 90, 120), 16, 10, None), ((133, 80, 71), 8, 23, [4, 11, 12]),
                                                 ((256, 256, 256), 8, 12, None)])
def test_tb3d_equals_per_step(torch_dev, monkeypatch, shape, so, nt, splits):
    """Two steps per launch (3D temporal blocking) against one launch per
    step, bit for bit: fields and traces, odd step counts (a last per-step
    launch) and applies split at odd points; several x/y tiles and z-chunks,
    sources and receivers anywhere.  The oracle bar on top."""
    prob = W.small_problem("iso", shape, so, nt=nt, seed=500 + so + nt, nsrc=2, nrec=40, nbl=6)
    say("tb3d", shape, so, nt, splits)
    monkeypatch.setenv("FDW_TB3D", "0")
    f0, t0, d0 = gpu_run(prob, torch_dev, nslots=2, splits=splits)
    monkeypatch.setenv("FDW_TB3D", "1")
    f1, t1, d1 = gpu_run(prob, torch_dev, nslots=2, splits=splits)
    assert "iso3d_tb2" in d1 and "iso3d_tb2" not in d0, (d0, d1)
    np.testing.assert_array_equal(f1["u"][1], f0["u"][1])
    np.testing.assert_array_equal(f1["u"][0], f0["u"][0])
    np.testing.assert_array_equal(t1, t0)
    if np.prod(shape) <= 2e6:
        of, otr = oracle_run(prob)
        check(prob, f1, t1, of, otr)


@pytest.mark.parametrize("kind", ["iso", "tti"])
def test_many_colliding_sources(torch_dev, kind):
    """More sources than the fused path holds (atomic injection), several in one cell."""
    shape = (41, 35, 30)
    ext = np.array([10.0 * (s - 1) for s in shape])
    rng = np.random.default_rng(3)
    pts = rng.uniform(0, 1, size=(6, 3)) * ext
    pts = np.concatenate([pts, np.repeat([[201.3, 170.7, 140.1]], 3, axis=0)])
    prob = W.small_problem(kind, shape, 8, nt=25, seed=9, src_at=pts, nrec=10)
    say("many sources", kind, prob.src.shape)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert "src=kernel" in desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("ndim", [2, 3])
def test_points_on_edges_and_corners(torch_dev, ndim):
    shape = (31, 26, 22)[:ndim]
    ext = [10.0 * (s - 1) for s in shape]
    corners = [list(ext), [0.0] * ndim, [ext[0], *([0.0] * (ndim - 1))], [0.0, *ext[1:]]]
    src = [list(ext), [0.0] * ndim]  # last node (clamped base) and origin
    prob = W.small_problem("iso", shape, 8, nt=30, seed=4, src_at=src, rec_coords=corners + [[e / 2 for e in ext]],
                           nbl=3)
    say("edges", ndim)
    gf, gtr, _ = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


def test_nonzero_initial_levels(torch_dev):
    prob = W.small_problem("tti", (29, 23, 19), 8, nt=20, seed=12, nrec=8)
    rng = np.random.default_rng(5)
    ash = prob.array_shape
    init = {"p": (rng.standard_normal(ash).astype(np.float32).astype(np.float64),
                  rng.standard_normal(ash).astype(np.float32).astype(np.float64)),
            "r": (rng.standard_normal(ash).astype(np.float32).astype(np.float64),
                  rng.standard_normal(ash).astype(np.float32).astype(np.float64))}
    say("nonzero initial levels")
    gf, gtr, _ = gpu_run(prob, torch_dev, u_init=init)
    of, otr = oracle_run(prob, u_init=init)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("kind", ["iso", "tti"])
def test_split_apply_is_identical(torch_dev, kind):
    prob = W.small_problem(kind, (35, 30, 26), 8, nt=24, seed=21, nrec=9)
    say("split apply", kind)
    f1, t1, _ = gpu_run(prob, torch_dev)
    f2, t2, _ = gpu_run(prob, torch_dev, splits=[0, 7, 15])
    f3, t3, _ = gpu_run(prob, torch_dev, time_M=-1)
    for nm in f1:
        np.testing.assert_array_equal(f1[nm][1], f2[nm][1])
        np.testing.assert_array_equal(f1[nm][0], f2[nm][0])
        np.testing.assert_array_equal(f1[nm][1], f3[nm][1])
    np.testing.assert_array_equal(t1, t2)
    np.testing.assert_array_equal(t1, t3)


def test_no_sparse_points(torch_dev):
    prob = W.small_problem("iso", (21, 19, 17), 4, nt=10, seed=2, src_at=np.zeros((0, 3)),
                           rec_coords=np.zeros((0, 3)))
    rng = np.random.default_rng(1)
    init = {"u": (np.zeros(prob.array_shape), rng.standard_normal(prob.array_shape).astype(np.float32).astype(float))}
    say("no sparse points")
    gf, gtr, _ = gpu_run(prob, torch_dev, u_init=init)
    of, otr = oracle_run(prob, u_init=init)
    check(prob, gf, gtr, of, otr)


# ---------------------------------------------------------- full-size configs
def test_config_2d_iso_101_full(torch_dev):
    """101 x 101, so = 4, 500 steps: full oracle run, every output compared."""
    prob = W.config_2d_iso_101()
    say(prob.name)
    gf, gtr, _ = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


def test_config_3d_iso_256_short_full_grid(torch_dev):
    """256^3, so = 8, first 40 steps on the full grid: every output compared."""
    prob = W.config_3d_iso_256(nt=40)
    say(prob.name, "nt=40")
    gf, gtr, _ = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


def _sampled_check(name, prob, gf, gtr):
    path = os.path.join(GOLDEN, f"full_{name}.npz")
    z = np.load(path)
    meta = json.loads(str(z["meta"]))
    assert meta["nt"] == prob.nt
    errs = {}
    for nm in gf:
        for tag, lv in (("prev", 0), ("cur", 1)):
            idx = z[f"{nm}_{tag}_idx"]
            ref = z[f"{nm}_{tag}_val"]
            got = gf[nm][lv].reshape(-1)[idx]
            errs[f"{nm}_{tag}"] = rel_l2(got, ref)
    errs["rec"] = rel_l2(gtr[:, z["rec_idx"]], z["rec_val"])
    say(name, "sampled", {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= TOL, (name, k, v)
    assert np.all(np.isfinite(gtr))


def test_config_3d_iso_256_full_sampled(torch_dev):
    """256^3, so = 8, all 1000 steps: sampled outputs against stored oracle values."""
    if not os.path.exists(os.path.join(GOLDEN, "full_3d_iso_256.npz")):
        pytest.skip("stored oracle samples not generated")
    prob = W.config_3d_iso_256()
    say(prob.name, "full")
    gf, gtr, _ = gpu_run(prob, torch_dev)
    _sampled_check("3d_iso_256", prob, gf, gtr)


def test_config_3d_tti_512_full_sampled(torch_dev):
    """512^3, so = 12, all 800 steps: sampled outputs against stored oracle values."""
    if not os.path.exists(os.path.join(GOLDEN, "full_3d_tti_512.npz")):
        pytest.skip("stored oracle samples not generated")
    prob = W.config_3d_tti_512()
    say(prob.name, "full")
    gf, gtr, _ = gpu_run(prob, torch_dev)
    _sampled_check("3d_tti_512", prob, gf, gtr)


def test_large_2d_grid_uses_per_step_kernel(torch_dev):
    """A 2D grid too large for the LDS-resident kernel (per-step launches)."""
    src = np.array([[1200.0, 900.0], [2500.5, 1700.25]])
    rec = np.concatenate([src + d for d in ([35.0, 0.0], [0.0, -42.5], [-27.3, 31.1], [12.0, 12.0])])
    prob = W.small_problem("iso", (401, 301), 8, nt=40, seed=31, src_at=src, rec_coords=rec, nbl=6)
    say("large 2D", prob.shape)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert "persistent" not in desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("kind,shape,so", [("iso", (401, 301), 4), ("iso", (130, 77), 12), ("iso", (257, 190), 14),
                                           ("iso", (70, 33), 8), ("iso", (97, 300), 2), ("tti", (401, 301), 4),
                                           ("tti", (130, 77), 12), ("tti", (203, 150), 16), ("tti", (70, 33), 8)])
def test_2d_streaming_equals_one_thread_per_point(torch_dev, monkeypatch, kind, shape, so):
    """2D grids too large for the LDS-resident kernel (or with it switched
    off; TTI always) run on the ring engine's flat mode, 64-column wavefronts
    streaming along z (ragged edges here; TTI angles over a full turn): the
    oracle's results, and the bits of the one-thread-per-point kernels
    (FDW_KERNEL=naive)."""
    src = np.array([[10.0 * (shape[0] // 3) + 3.3, 10.0 * (shape[1] // 2) - 4.1], [5.0, 10.0 * (shape[1] - 1)]])
    # receivers on the row of the first source (the wave reaches them in 40 steps)
    rec = np.array([[10.0 * k * (shape[0] - 1) / 11.0, 10.0 * (shape[1] // 2) + 13.7] for k in range(12)])
    prob = W.small_problem(kind, shape, so, nt=40, seed=34, src_at=src, rec_coords=rec, nbl=6,
                           angle_range=(0.0, 2.0 * np.pi))
    say("2d streaming", kind, shape, so)
    monkeypatch.setenv("FDW_PERSIST2D", "0")
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert f"{kind}2d_stream" in desc, desc
    monkeypatch.setenv("FDW_KERNEL", "naive")
    nf, ntr, ndesc = gpu_run(prob, torch_dev)
    assert "naive" in ndesc, ndesc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)
    for nm in gf:
        np.testing.assert_array_equal(gf[nm][1], nf[nm][1])
        np.testing.assert_array_equal(gf[nm][0], nf[nm][0])
    np.testing.assert_array_equal(gtr, ntr)


def test_small_2d_grid_uses_persistent_kernel(torch_dev):
    prob = W.small_problem("iso", (120, 95), 12, nt=60, seed=32, nsrc=6, nrec=30, nbl=8)
    say("persistent 2D", prob.shape)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert "persistent" in desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("kind,shape", [("iso", (35, 30, 26)), ("tti", (33, 28, 25)), ("iso", (60, 41)),
                                        ("tti", (48, 39))])
def test_one_thread_per_point_schedule(torch_dev, monkeypatch, kind, shape):
    """FDW_KERNEL=naive selects the one-thread-per-point kernels at operator
    creation; they must agree with the oracle as well."""
    monkeypatch.setenv("FDW_KERNEL", "naive")
    prob = W.small_problem(kind, shape, 8, nt=20, seed=33, nrec=10)
    say("naive schedule", kind, shape)
    gf, gtr, desc = gpu_run(prob, torch_dev)
    assert "naive" in desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("kind,shape,so", [("iso", (37, 29, 23), 8), ("tti", (33, 27, 21), 12), ("iso", (67, 45), 4),
                                           ("iso", (401, 301), 4)])
def test_inplace_two_slot_storage(torch_dev, kind, shape, so):
    """Two-slot (in-place leapfrog) storage gives the oracle's results, and the
    same bits as the three-slot modulo buffer."""
    if len(shape) == 2 and shape[0] > 300:
        src = np.array([[1200.0, 900.0]])
        prob = W.small_problem(kind, shape, so, nt=30, seed=41, src_at=src, rec_coords=src + 20.0)
    else:
        prob = W.small_problem(kind, shape, so, nt=30, seed=41, nsrc=2, nrec=10)
    say("two slots", kind, shape, so)
    gf, gtr, _ = gpu_run(prob, torch_dev, nslots=2)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)
    gf3, gtr3, _ = gpu_run(prob, torch_dev, nslots=3)
    for nm in gf:
        np.testing.assert_array_equal(gf[nm][1], gf3[nm][1])
        np.testing.assert_array_equal(gf[nm][0], gf3[nm][0])
    np.testing.assert_array_equal(gtr, gtr3)
    gfs, gtrs, _ = gpu_run(prob, torch_dev, nslots=2, splits=[4, 17])
    for nm in gf:
        np.testing.assert_array_equal(gf[nm][1], gfs[nm][1])
    np.testing.assert_array_equal(gtr, gtrs)


def test_kernel_timing_covers_every_launch(torch_dev):
    """Timed runs of k consecutive stencil launches cover every launch, also
    when an apply ends inside a run."""
    from paper_1807_03032_amd import fdw
    prob = W.small_problem("iso", (40, 36, 30), 8, nt=10, seed=3)
    shot = fdw.Shot(prob, torch_dev, nslots=2)
    try:
        for k in (1, 4):
            fdw.fdw_operator_set_timing(shot.op, k)
            shot.apply(0, 9)
            ms, n = fdw.fdw_operator_kernel_time(shot.op)
            assert n == 10 and ms > 0
        fdw.fdw_operator_set_timing(shot.op, 3)
        shot.apply(0, 4)
        shot.apply(5, 9)
        ms, n = fdw.fdw_operator_kernel_time(shot.op)
        assert n == 10 and ms > 0
        fdw.fdw_operator_set_timing(shot.op, 0)
    finally:
        shot.close()


@pytest.mark.parametrize("kind,shape,so", [("iso", (9, 7, 5), 16), ("tti", (11, 9, 6), 16), ("iso", (5, 3), 16),
                                           ("tti", (6, 5), 12), ("iso", (3, 70, 4), 8), ("iso", (130, 2, 3), 4)])
def test_grids_smaller_than_the_stencil(torch_dev, kind, shape, so):
    """Axes shorter than the stencil radius (or than a tile): every neighbour
    beyond the domain is the zero halo."""
    prob = W.small_problem(kind, shape, so, nt=12, seed=80, nsrc=1, nrec=3, nbl=1)
    say("tiny", kind, shape, so)
    gf, gtr, _ = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("shape,so", [((37, 29, 23), 8), ((70, 45, 33), 16), ((9, 7, 5), 4)])
def test_wide_field_form(torch_dev, monkeypatch, shape, so):
    """The raw-buffer form of the isotropic step, taken for fields of 4 GiB or
    more (forced here with FDW_ISO_WIDE=1): the oracle's results, and the same
    bits as the global-access form."""
    prob = W.small_problem("iso", shape, so, nt=25, seed=90, nsrc=2, nrec=12)
    say("wide form", shape, so)
    gf, gtr, desc = gpu_run(prob, torch_dev, nslots=2)
    assert "wide" not in desc
    monkeypatch.setenv("FDW_ISO_WIDE", "1")
    wf, wtr, wdesc = gpu_run(prob, torch_dev, nslots=2)
    assert "wide" in wdesc, wdesc
    of, otr = oracle_run(prob)
    check(prob, wf, wtr, of, otr)
    for nm in gf:
        np.testing.assert_array_equal(wf[nm][1], gf[nm][1])
        np.testing.assert_array_equal(wf[nm][0], gf[nm][0])
    np.testing.assert_array_equal(wtr, gtr)


def test_ring_engine_fields_above_2gib(torch_dev, monkeypatch):
    """The ring engine's chunk-based descriptors on a field of more than 2 GiB
    (800 x 800 x 860 at space order 8): a source and receivers in the planes
    more than 2 GiB from the field's start, the same bits as the
    shifting-queue engine (32-bit global offsets, valid below 4 GiB)."""
    from paper_1807_03032_amd import fdw
    shape, so, nt, h = (800, 800, 860), 8, 8, 10.0
    ext = tuple(h * (k - 1) for k in shape)
    m = np.full(tuple(reversed(shape)), 1.0 / 1500.0 ** 2, dtype=np.float32)  # numpy order (z, y, x)
    m[430:] = 1.0 / 2500.0 ** 2
    dt = W.cfl_dt(h, 2500.0, 3)
    src_c = np.array([[4003.0, 3991.0, 8455.0]])
    rec_c = np.array([[3950.0 + 20.0 * k, 4010.0, 8420.0 + 7.0 * k] for k in range(8)])
    src = np.asarray(W.ricker(60.0, 0.0, dt, nt), dtype=np.float32).reshape(nt, 1)
    prob = W.Problem("ring_2gib", "iso", shape, ext, (0.0,) * 3, so, 4, nt, dt, 2500.0, 0.0, {"m": m}, src_c, src,
                     rec_c)
    say("ring engine above 2 GiB", shape, so)
    runs = []
    for eng in ("0", "1"):
        monkeypatch.setenv("FDW_ENGINE", eng)
        shot = fdw.Shot(prob, torch_dev, nslots=2)
        try:
            if eng == "0":
                assert shot.lay.elems_per_slot * 4 > 2 ** 31, shot.lay.elems_per_slot
            shot.apply(0, nt - 1)
            f = shot.fields(nt - 1)["u"]
            runs.append((f[0][780:], f[1][780:], shot.traces()))
        finally:
            shot.close()
    (p0, c0, t0), (p1, c1, t1) = runs
    assert np.abs(c0).max() > 0 and np.abs(t0).max() > 0
    np.testing.assert_array_equal(c0, c1)
    np.testing.assert_array_equal(p0, p1)
    np.testing.assert_array_equal(t0, t1)


@pytest.mark.parametrize("kind,shape,so,nsrc", [("iso", (40, 36, 30), 8, 600), ("tti", (33, 28, 25), 8, 600),
                                                ("iso", (70, 55), 4, 1100)])
def test_many_sources_injected_by_gather(torch_dev, kind, shape, so, nsrc):
    """4096 or more injection lanes (sources x corners) take the gather
    kernel (one thread per distinct target element, no atomics); with
    hundreds of sources on a small grid most targets receive several
    contributions.  The oracle's results, and the same bits on a second run."""
    prob = W.small_problem(kind, shape, so, nt=20, seed=95, nsrc=nsrc, nrec=12)
    say("gather injection", kind, shape, so, nsrc)
    gf, gtr, _ = gpu_run(prob, torch_dev)
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)
    gf2, gtr2, _ = gpu_run(prob, torch_dev)
    for nm in gf:
        np.testing.assert_array_equal(gf2[nm][1], gf[nm][1])
    np.testing.assert_array_equal(gtr2, gtr)


@pytest.mark.parametrize("kind,shape,so", [("iso", (37, 29, 23), 8), ("tti", (33, 27, 21), 12), ("iso", (67, 45), 4),
                                           ("tti", (48, 39), 8), ("iso", (70, 41, 9), 16)])
def test_parameter_halos_are_not_read(torch_dev, kind, shape, so):
    """Only the domain points of a Function are read: NaN in the halo and
    padding of every parameter field changes no bit of the results."""
    from paper_1807_03032_amd import fdw
    prob = W.small_problem(kind, shape, so, nt=20, seed=91, nsrc=2, nrec=10)
    say("parameter halos", kind, shape, so)
    rf, rtr, _ = gpu_run(prob, torch_dev, nslots=2)
    shot = fdw.Shot(prob, torch_dev, nslots=2)
    try:
        for nm, arr in prob.fields.items():
            t = shot.par[nm]
            t.fill_(float("nan"))
            fdw.upload(t, shot.lay, 0, arr)
        shot.apply(0, prob.nt - 1)
        f = shot.fields(prob.nt - 1)
        tr = shot.traces()
    finally:
        shot.close()
    for nm in rf:
        np.testing.assert_array_equal(f[nm][1], rf[nm][1])
        np.testing.assert_array_equal(f[nm][0], rf[nm][0])
    np.testing.assert_array_equal(tr, rtr)


def test_tti_parameters_read_at_each_apply(torch_dev):
    """The 3D TTI kernels use per-point values derived from the parameters at
    the start of every apply: parameters rewritten after the operator was
    created are honoured by fdw_operator_apply and by fdw_batch_apply."""
    import dataclasses

    import torch

    from paper_1807_03032_amd import fdw
    p1 = W.small_problem("tti", (33, 27, 21), 12, nt=20, seed=92, nsrc=1, nrec=8)
    f2 = dict(p1.fields)
    f2["theta"] = 0.5 * p1.fields["theta"]
    f2["phi"] = p1.fields["phi"] + 0.3
    f2["m"] = 1.1 * p1.fields["m"]
    f2["eps"] = 0.5 * p1.fields["eps"]
    f2["delta"] = 0.5 * p1.fields["delta"]
    p2 = dataclasses.replace(p1, fields=f2)
    say("tti parameters at apply")
    rf, rtr, _ = gpu_run(p2, torch_dev, nslots=2)
    of, otr = oracle_run(p2)
    check(p2, rf, rtr, of, otr)
    for batched in (False, True):
        shot = fdw.Shot(p1, torch_dev, nslots=2)
        b = fdw.fdw_batch_create() if batched else None
        try:
            for nm, arr in p2.fields.items():
                fdw.upload(shot.par[nm], shot.lay, 0, arr)
            if batched:
                s = torch.cuda.current_stream(torch_dev)
                fdw.fdw_batch_apply(b, [shot.op], [0], [p1.nt - 1], s.cuda_stream)
                s.synchronize()
            else:
                shot.apply(0, p1.nt - 1)
            f = shot.fields(p1.nt - 1)
            tr = shot.traces()
        finally:
            if b is not None:
                fdw.fdw_batch_destroy(b)
            shot.close()
        for nm in rf:
            np.testing.assert_array_equal(f[nm][1], rf[nm][1])
            np.testing.assert_array_equal(f[nm][0], rf[nm][0])
        np.testing.assert_array_equal(tr, rtr)


def wide_problems(so=8, nt=10):
    """(101^3 run, 1056 x 1040 x 1040 run) around the same source on a node:
    constant model, no damping layer, so = 8 and 10 steps (or as given, with
    nt * so / 2 below 50 points), receivers within 40 points of the source."""
    h, v = 10.0, 2000.0
    assert nt * so // 2 < 50
    dt = W.cfl_dt(h, v, 3)
    src = W.f32(W.ricker(15.0, 1.0 / 15.0, dt, nt)).reshape(nt, 1)
    offs = np.array([[0.0, 0.0, 0.0], [103.7, 51.2, -77.5], [-250.0, 120.0, 30.3], [12.5, -310.0, 205.0]])

    def problem(shape, centre):
        c = np.array(centre, dtype=np.float64) * h
        m = np.full(tuple(reversed(shape)), 1.0 / v ** 2, dtype=np.float32)
        return W.Problem(f"wide_{shape[0]}", "iso", shape, tuple(h * (k - 1) for k in shape), (0.0,) * 3, so, 0, nt,
                         dt, v, 0.0, {"m": m}, c.reshape(1, 3), src, c + offs)

    return problem((101, 101, 101), (50, 50, 50)), problem((1056, 1040, 1040), (528, 520, 520))


@pytest.mark.parametrize("so,nt", [(8, 10), (16, 6)])
def test_wide_fields_at_real_size(torch_dev, so, nt):
    """A grid whose padded fields pass 4 GiB (1056 x 1040 x 1040: 4.9 GB per
    field): at so = 8 the ring engine (chunk-based buffer descriptors), at
    so = 16 the raw-buffer form of the shifting-queue engine.  With a constant
    model, a source on a node in the middle and no damping layer, nt steps
    reach nt * so / 2 < 50 points from the source, so the block around it must
    equal, bit for bit, the same block of a 101^3 run around the same source
    (whose boundary lies beyond the reach), and match the oracle's 101^3 run."""
    import torch

    from paper_1807_03032_amd import fdw
    small, big = wide_problems(so, nt)
    so, nt = big.so, big.nt
    g = fdw.fdw_grid_create(big.shape, big.extent)
    lay = fdw.fdw_field_layout(g, so)
    fdw.fdw_grid_destroy(g)
    assert lay.elems_per_slot * 4 > 2 ** 32
    say("wide fields at real size", big.shape, lay.elems_per_slot * 4 / 2 ** 30, "GiB per field")
    sf, str_, sdesc = gpu_run(small, torch_dev, nslots=2)
    assert "wide" not in sdesc
    shot = fdw.Shot(big, torch_dev, nslots=2)
    try:
        desc = fdw.fdw_operator_describe(shot.op)[0]
        assert ("wide" in desc) == (so > 8), desc
        shot.apply(0, nt - 1)
        torch.cuda.synchronize(torch_dev)
        blocks = []
        for lv in (nt - 1, nt):
            full = fdw.slot_view(shot.wave["u"], shot.lay, lv % 2)
            blocks.append(full[520 - 50:520 + 51, 520 - 50:520 + 51, 528 - 50:528 + 51].to("cpu").numpy()
                          .astype(np.float64))
        btr = shot.traces()
    finally:
        shot.close()
    np.testing.assert_array_equal(blocks[0], sf["u"][0])
    np.testing.assert_array_equal(blocks[1], sf["u"][1])
    np.testing.assert_array_equal(btr, str_)
    of, otr = oracle_run(small)
    check(small, {"u": tuple(blocks)}, btr, of, otr)


_STRIDED_CHILD = """
import sys
import numpy as np
import torch
sys.path.insert(0, sys.argv[1])
from paper_1807_03032_amd import fdw
from paper_1807_03032_amd import workloads as W
fdw.load()
kind, shape, so = sys.argv[3], tuple(int(s) for s in sys.argv[4].split("x")), int(sys.argv[5])
prob = W.small_problem(kind, shape, so, nt=16, seed=77, nsrc=1, nrec=700)
shot = fdw.Shot(prob, torch.device("cuda:0"), nslots=3)
try:
    shot.apply(0, prob.nt - 1)
    np.save(sys.argv[2], shot.traces())
finally:
    shot.close()
"""


@pytest.mark.parametrize("kind,shape,so", [("iso", (70, 41, 33), 8), ("tti", (67, 35, 29), 12)])
def test_receivers_beyond_one_per_sampling_thread(torch_dev, tmp_path, kind, shape, so):
    """700 receivers sampled inside the stencil launches by one sampling
    workgroup (FDW_INTERP_WG=1, set for a child process: the library reads it
    once), so that each sampling thread takes several receivers in turn: the
    traces equal those of the default launch (several sampling workgroups)
    bit for bit, and the oracle's."""
    import subprocess
    prob = W.small_problem(kind, shape, so, nt=16, seed=77, nsrc=1, nrec=700)
    say("strided receiver sampling", kind, shape, so)
    f, tr, desc = gpu_run(prob, torch_dev)
    assert "nrec=700" in desc and "stream" in desc, desc
    out = str(tmp_path / "traces.npy")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, FDW_INTERP_WG="1")
    r = subprocess.run([sys.executable, "-c", _STRIDED_CHILD, root, out, kind, "x".join(map(str, shape)), str(so)],
                       env=env, timeout=240, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    np.testing.assert_array_equal(np.load(out), tr)
    of, otr = oracle_run(prob)
    check(prob, f, tr, of, otr)


def test_tti_nontemporal_pointwise_loads_change_no_bit(torch_dev, monkeypatch):
    """Grids beyond the last-level cache read the TTI stages' pointwise fields
    with the non-temporal hint; forced on and off here (FDW_TTI_NT) on a
    multi-tile grid, the hint changes no bit of the levels or the traces."""
    prob = W.small_problem("tti", (150, 70, 90), 12, nt=12, seed=321, nsrc=2, nrec=40, nbl=6)
    say("tti non-temporal hint", prob.shape)
    runs = {}
    for nt in ("1", "0"):
        monkeypatch.setenv("FDW_TTI_NT", nt)
        f, tr, desc = gpu_run(prob, torch_dev)
        assert ("pointwise=nt" in desc) == (nt == "1"), desc
        runs[nt] = (f, tr)
    for nm in runs["1"][0]:
        for k in (0, 1):
            np.testing.assert_array_equal(runs["1"][0][nm][k], runs["0"][0][nm][k])
    np.testing.assert_array_equal(runs["1"][1], runs["0"][1])


def test_iso2d_nontemporal_pointwise_loads_change_no_bit(torch_dev, monkeypatch):
    """Large 2D grids read u(t-1) and m with the non-temporal hint; forced on
    and off here (FDW_ISO2D_NT) on a grid too large for the LDS-resident
    kernel, the hint changes no bit of the levels or the traces."""
    prob = W.small_problem("iso", (600, 500), 8, nt=30, seed=322, nsrc=2, nrec=40)
    say("iso2d non-temporal hint", prob.shape)
    runs = {}
    for nt in ("1", "0"):
        monkeypatch.setenv("FDW_ISO2D_NT", nt)
        f, tr, desc = gpu_run(prob, torch_dev)
        assert "iso2d_stream" in desc, desc
        runs[nt] = (f, tr)
    for k in (0, 1):
        np.testing.assert_array_equal(runs["1"][0]["u"][k], runs["0"][0]["u"][k])
    np.testing.assert_array_equal(runs["1"][1], runs["0"][1])
