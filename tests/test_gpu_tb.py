"""GPU parity of the 2D temporal blocking (several steps per launch on
overlapped LDS patches, opt-in with FDW_TB=1) against the FP64 oracle, and
its equality, bit for bit, with the one-launch-per-step kernels."""

import numpy as np
import pytest

from paper_1807_03032_amd import workloads as W

from test_gpu_parity import check, gpu_run, oracle_run, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def tile_edge_problem(shape, so, nt, seed, nsrc=3):
    """Sources and receivers on and around the inner-tile edges (x = 112 k,
    128 k; z = 64 k) and the domain edges."""
    h = 10.0
    ext = np.array([h * (s - 1) for s in shape])
    src = [[128 * h - 0.5 * h, 64 * h + 0.3 * h], [111.5 * h, 63.9 * h], [ext[0] / 2, ext[1] - 0.2 * h]][:nsrc]
    rng = np.random.default_rng(seed)
    rec = [[128 * h, 64 * h], [127.5 * h, 63.5 * h], [112 * h, 128 * h], [0.0, 0.0], list(ext),
           [ext[0], 0.0], [256 * h - 0.01, 5 * h]]
    rec += list(rng.uniform(0, 1, size=(40, 2)) * ext)
    rec = [r for r in rec if 0 <= r[0] <= ext[0] and 0 <= r[1] <= ext[1]]
    return W.small_problem("iso", shape, so, nt=nt, seed=seed, src_at=src, rec_coords=rec, nbl=8)


@pytest.fixture(autouse=True)
def tb_on(monkeypatch):
    """The temporal blocking is opt-in (FDW_TB=1)."""
    monkeypatch.setenv("FDW_TB", "1")


@pytest.mark.parametrize("so", [4, 8, 12, 16])
def test_tb_matches_oracle(torch_dev, so):
    prob = tile_edge_problem((419, 283), so, nt=37, seed=40 + so)
    say("tb", prob.shape, so)
    gf, gtr, desc = gpu_run(prob, torch_dev, nslots=2)
    assert "iso2d_tb" in desc, desc
    of, otr = oracle_run(prob)
    check(prob, gf, gtr, of, otr)


@pytest.mark.parametrize("so,nt", [(8, 37), (16, 9), (4, 1)])
def test_tb_equals_per_step_kernels(torch_dev, monkeypatch, so, nt):
    prob = tile_edge_problem((300, 211), so, nt=nt, seed=7)
    say("tb vs per-step", so, nt)
    f1, t1, d1 = gpu_run(prob, torch_dev, nslots=2)
    f2, t2, d2 = gpu_run(prob, torch_dev, nslots=2, splits=[min(4, nt - 1)] if nt > 5 else None)
    monkeypatch.setenv("FDW_TB", "0")
    f3, t3, d3 = gpu_run(prob, torch_dev, nslots=2)
    assert "iso2d_tb" in d1 and "iso2d_tb" not in d3
    for f in (f2, f3):
        np.testing.assert_array_equal(f1["u"][1], f["u"][1])
        np.testing.assert_array_equal(f1["u"][0], f["u"][0])
    np.testing.assert_array_equal(t1, t2)
    np.testing.assert_array_equal(t1, t3)


def test_tb_not_used_for_modulo3_or_many_sources(torch_dev):
    prob = tile_edge_problem((300, 211), 8, nt=5, seed=8)
    _, _, d = gpu_run(prob, torch_dev, nslots=3)
    assert "iso2d_tb" not in d
    pts = np.random.default_rng(1).uniform(0, 1, size=(6, 2)) * np.array([2990.0, 2100.0])
    many = W.small_problem("iso", (300, 211), 8, nt=5, seed=9, src_at=pts, nrec=5, nbl=8)
    _, _, d = gpu_run(many, torch_dev, nslots=2)
    assert "iso2d_tb" not in d
