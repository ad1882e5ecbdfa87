"""Graph capture of a single shot's apply: a range applied again with the same
settings is captured into a hipGraph and replayed; every replay gives the
bits of the plain launches, with unrelated eager work between replays."""
import sys

import numpy as np
import pytest

from paper_1807_03032_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available()
    from paper_1807_03032_amd import fdw
    fdw.load()
    return torch.device("cuda:0")


@pytest.mark.parametrize("kind,shape,so,nsrc", [("iso", (70, 45, 33), 8, 2), ("tti", (70, 41, 30), 12, 1),
                                                ("iso", (401, 301), 4, 2), ("iso", (50, 40, 30), 8, 600)])
def test_apply_graph_replays_give_the_same_bits(torch_dev, kind, shape, so, nsrc):
    import torch

    from paper_1807_03032_amd import fdw
    if len(shape) == 2:
        src = np.array([[1200.0, 900.0], [2100.0, 1500.0]])
        prob = W.small_problem(kind, shape, so, nt=24, seed=61, src_at=src, rec_coords=src + 20.0)
    else:
        prob = W.small_problem(kind, shape, so, nt=24, seed=61, nsrc=nsrc, nrec=20)
    say("apply graph", kind, shape, so, nsrc)
    shot = fdw.Shot(prob, torch_dev)
    try:
        runs = []
        for k in range(4):
            for t in shot.wave.values():
                t.zero_()
            shot.rec_data.zero_()
            # unrelated eager work on the same device between the runs
            a = torch.randn(512, 512, device=torch_dev)
            (a @ a).sum().item()
            torch.cuda.synchronize(torch_dev)
            shot.apply(0, prob.nt - 1)
            torch.cuda.synchronize(torch_dev)
            runs.append((shot.fields(prob.nt - 1), shot.traces()))
        builds, replays = fdw.fdw_operator_graph_stats(shot.op)
    finally:
        shot.close()
    # run 0: plain launches; run 1: captured and replayed; runs 2, 3: replays
    assert (builds, replays) == (1, 3), (builds, replays)
    f0, tr0 = runs[0]
    assert np.abs(tr0).max() > 0
    for f, tr in runs[1:]:
        for nm in f0:
            np.testing.assert_array_equal(f[nm][0], f0[nm][0])
            np.testing.assert_array_equal(f[nm][1], f0[nm][1])
        np.testing.assert_array_equal(tr, tr0)


def test_changed_range_or_saving_is_not_replayed(torch_dev):
    """Another range, or a new saving buffer, launches plainly (and is captured
    only when it repeats)."""
    import torch

    from paper_1807_03032_amd import fdw
    prob = W.small_problem("iso", (40, 33, 27), 8, nt=20, seed=62, nsrc=1, nrec=8)
    shot = fdw.Shot(prob, torch_dev)
    try:
        shot.apply(0, 9)
        shot.apply(0, 9)
        assert fdw.fdw_operator_graph_stats(shot.op) == (1, 1)
        shot.apply(10, 19)
        assert fdw.fdw_operator_graph_stats(shot.op) == (1, 1)
        buf = torch.zeros(3 * shot.lay.elems_per_slot, device=torch_dev)
        fdw.fdw_operator_set_save(shot.op, buf.data_ptr(), 3, 1, 11)
        shot.apply(10, 19)
        shot.apply(10, 19)
        assert fdw.fdw_operator_graph_stats(shot.op) == (2, 2)
        torch.cuda.synchronize(torch_dev)
        fdw.fdw_operator_set_save(shot.op, None)
    finally:
        shot.close()
