"""GPU tests of the fused multi-shot steps (fdw_batch_apply) and of the shot
server (continuous batching): every shot's result is the same alone and in
a mix, bit for bit, the server keeps within its device-memory budget, and
served results match the FP64 oracle within the parity bar (relative L2 <=
1e-4)."""
import time

import numpy as np
import pytest

import oracle
from paper_1807_03032_amd import workloads as W

from test_gpu_parity import TOL, rel_l2, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def run_alone(prob, dev):
    """Plain per-shot solve through fdw_operator_apply (two-slot storage)."""
    from paper_1807_03032_amd import fdw
    shot = fdw.Shot(prob, dev, nslots=2)
    try:
        shot.apply(0, prob.nt - 1)
        f = shot.fields(prob.nt - 1)
        tr = shot.traces()
    finally:
        shot.close()
    return tr, f


@pytest.mark.parametrize("kind,ndim,n,so", [("iso", 3, 40, 8), ("tti", 3, 36, 12), ("iso", 2, 203, 4),
                                            ("tti", 2, 201, 16), ("iso", 3, 33, 16), ("iso", 2, 101, 4),
                                            ("iso", 2, 150, 16)])
def test_batch_equals_single(torch_dev, kind, ndim, n, so):
    import torch

    from paper_1807_03032_amd import fdw
    probs = [W.serve_problem(kind, ndim, n, so, nt, seed=s, nbl=8) for s, nt in ((1, 37), (2, 52), (3, 45))]
    say("batch", kind, ndim, n, so)
    ref = [run_alone(p, torch_dev) for p in probs]
    shots = [fdw.Shot(p, torch_dev, nslots=2) for p in probs]
    batches = [fdw.fdw_batch_create(), fdw.fdw_batch_create()]
    side = torch.cuda.Stream(torch_dev)
    try:
        t = [0] * len(probs)
        calls = 0
        # a lone 3D shot runs the single-shot kernels, and 2D isotropic grids that
        # fit in LDS run one workgroup per shot in one launch: no graph either way
        lds_resident = kind == "iso" and ndim == 2 and n * n * 4 <= 152 * 1024
        graph_calls = 0
        while any(t[i] < p.nt for i, p in enumerate(probs)):
            # shots leave the batch when done: the shot count (and graph) changes
            idx = [i for i, p in enumerate(probs) if t[i] < p.nt]
            tm = [t[i] for i in idx]
            tM = [min(t[i] + 16, probs[i].nt) - 1 for i in idx]
            fdw.fdw_batch_apply(batches[calls % 2], [shots[i].op for i in idx], tm, tM, side.cuda_stream)
            for i, hi in zip(idx, tM):
                t[i] = hi + 1
            calls += 1
            graph_calls += 0 if (ndim == 3 and len(idx) == 1) or lds_resident else 1
        side.synchronize()
        builds = sum(fdw.fdw_batch_stats(b)[0] for b in batches)
        launches = sum(fdw.fdw_batch_stats(b)[1] for b in batches)
        if lds_resident:
            assert launches == builds == 0
        else:
            assert graph_calls < calls if ndim == 3 else graph_calls == calls
            assert launches == graph_calls and 1 <= builds < graph_calls
        for i, p in enumerate(probs):
            f = shots[i].fields(p.nt - 1)
            tr = shots[i].traces()
            for nm in f:
                np.testing.assert_array_equal(f[nm][1], ref[i][1][nm][1])
                np.testing.assert_array_equal(f[nm][0], ref[i][1][nm][0])
            np.testing.assert_array_equal(tr, ref[i][0])
    finally:
        for b in batches:
            fdw.fdw_batch_destroy(b)
        for s in shots:
            s.close()


def serve_all(reqs, budget=0, chunk_us=40, stagger=0, keep_field=True, watch=None):
    """Run requests through one server; `stagger` progress rounds between
    submissions.  Returns ({index: (traces, field)}, server stats)."""
    from paper_1807_03032_amd import fdw
    sv = fdw.Server(budget_bytes=budget, chunk_target_us=chunk_us, nstreams=3)
    try:
        tickets = []
        pending = list(range(len(reqs)))
        out = {}
        deadline = time.time() + 120
        while len(out) < len(reqs):
            assert time.time() < deadline, "server did not finish"
            if pending:
                i = pending.pop(0)
                tickets.append((i, sv.submit(reqs[i], keep_field=keep_field)))
            for _ in range(stagger if pending else 1):
                sv.progress()
                if watch:
                    watch(sv.stats())
            for i, tk in tickets:
                if i not in out and sv.info(tk).state == fdw.FDW_SHOT_DONE:
                    out[i] = sv.fetch(tk, field=keep_field)
                    sv.release(tk)
            if not pending:
                time.sleep(1e-4)
        return out, sv.stats()
    finally:
        sv.close()


def mixed_requests():
    return [W.serve_problem("iso", 2, 201, 8, 60, seed=11, nbl=10),
            W.serve_problem("tti", 2, 201, 8, 80, seed=12, nbl=10),
            W.serve_problem("iso", 3, 40, 8, 70, seed=13, nbl=8),
            W.serve_problem("iso", 3, 40, 8, 50, seed=14, nbl=8),   # same bucket as the previous one
            W.serve_problem("tti", 3, 36, 12, 40, seed=15, nbl=8),
            W.serve_problem("iso", 3, 48, 16, 30, seed=16, nbl=8),
            W.serve_problem("iso", 2, 201, 8, 45, seed=17, nbl=10)]  # joins the first bucket late


def test_server_alone_and_in_the_mix(torch_dev):
    reqs = mixed_requests()
    say("server alone")
    alone = {i: serve_all([r])[0][0] for i, r in enumerate(reqs)}
    say("server mix")
    mix, stats = serve_all(reqs, stagger=2)
    say("stats", stats)
    assert stats["completed"] == len(reqs) and stats["buckets"] == 5
    assert stats["graph_launches"] > stats["graph_builds"]
    for i in range(len(reqs)):
        np.testing.assert_array_equal(mix[i][0], alone[i][0])
        np.testing.assert_array_equal(mix[i][1], alone[i][1])
    # a served result against the plain per-shot solve and the oracle
    for i in (2, 6):
        tr, f = run_alone(reqs[i], torch_dev)
        if reqs[i].ndim == 3:  # same kernels in 3D: same bits
            np.testing.assert_array_equal(mix[i][0], tr)
        p = reqs[i]
        g = oracle.Grid(p.shape, p.extent, p.origin, so=p.so, dt=p.dt, nbl=p.nbl, vmax=p.vmax, rc=p.rc)
        _, uc, rec = oracle.iso_run(g, p.fields["m"], p.nt, src_coords=p.src_coords, src=p.src,
                                    rec_coords=p.rec_coords)
        e_f, e_r = rel_l2(mix[i][1], uc), rel_l2(mix[i][0], rec)
        say("oracle", p.name, f"{e_f:.2e}", f"{e_r:.2e}")
        assert e_f <= TOL and e_r <= TOL


def test_server_keeps_within_budget(torch_dev):
    from paper_1807_03032_amd import fdw
    reqs = [W.serve_problem("iso", 3, 48, 8, 40, seed=20 + k, nbl=8) for k in range(4)]
    reqs.append(W.serve_problem("iso", 2, 201, 4, 40, seed=30, nbl=10))
    fps = [fdw.Server.footprint(r) for r in reqs]
    budget = 2 * fps[0] + fps[-1]  # two 3D shots at a time, and the 2D one beside them
    seen = []
    out, stats = serve_all(reqs, budget=budget, keep_field=False, watch=lambda s: seen.append(s["used"]))
    say("budget", budget, "peak used", max(seen))
    assert max(seen) <= budget
    assert max(seen) >= 2 * fps[0]
    assert len(out) == len(reqs)
    big = W.serve_problem("iso", 3, 64, 8, 10, seed=40, nbl=8)
    sv = fdw.Server(budget_bytes=fps[0], nstreams=1)
    try:
        with pytest.raises(fdw.FdwError) as e:
            sv.submit(big)
        assert e.value.code == fdw.FDW_ERR_NOMEM
    finally:
        sv.close()


def test_server_edge_requests(torch_dev):
    """Requests without receivers, without sources, of a single step, and one
    whose operator cannot be built (dt above the stability bound): the last
    fails alone, the others are served."""
    import dataclasses

    from paper_1807_03032_amd import fdw
    a = dataclasses.replace(W.serve_problem("iso", 2, 201, 8, 5, seed=50, nbl=10), rec_coords=np.zeros((0, 2)))
    b0 = W.serve_problem("iso", 3, 40, 8, 1, seed=51, nbl=8)
    b = dataclasses.replace(b0, src_coords=np.zeros((0, 3)), src=np.zeros((1, 0), dtype=np.float32))
    c = dataclasses.replace(W.serve_problem("iso", 3, 40, 8, 10, seed=52, nbl=8), dt=3.0 * b0.dt)
    d = W.serve_problem("tti", 2, 201, 4, 12, seed=53, nbl=10)
    sv = fdw.Server(chunk_target_us=40, nstreams=2)
    try:
        tk = [sv.submit(p) for p in (a, b, c, d)]
        deadline = time.time() + 60
        final = (fdw.FDW_SHOT_DONE, fdw.FDW_SHOT_FAILED)
        while not all(sv.info(t).state in final for t in tk):
            assert time.time() < deadline
            sv.progress()
            time.sleep(1e-4)
        states = [sv.info(t).state for t in tk]
        assert states == [fdw.FDW_SHOT_DONE, fdw.FDW_SHOT_DONE, fdw.FDW_SHOT_FAILED, fdw.FDW_SHOT_DONE]
        rec_a, _ = sv.fetch(tk[0])
        assert rec_a.shape == (5, 0)
        rec_b, _ = sv.fetch(tk[1])
        assert rec_b.shape == (1, 40) and not np.any(rec_b)  # no source, zero initial state
        with pytest.raises(fdw.FdwError) as e:
            sv.fetch(tk[2])
        assert e.value.code == fdw.FDW_ERR_STATE and "stab" in str(e.value)
        rec_d, _ = sv.fetch(tk[3])
        tr, _ = run_alone(d, torch_dev)
        np.testing.assert_array_equal(rec_d, tr)
        for t in tk:
            sv.release(t)
    finally:
        sv.close()


def test_batch_rejects_what_it_cannot_fuse(torch_dev):
    """Mismatched geometry or order, scatter-injected sources and adjoint
    operators are refused before any launch."""
    from paper_1807_03032_amd import fdw
    p1 = W.serve_problem("iso", 3, 40, 8, 10, seed=60, nbl=8)
    p2 = W.serve_problem("iso", 3, 44, 8, 10, seed=61, nbl=8)     # other shape
    p3 = W.serve_problem("iso", 3, 40, 4, 10, seed=62, nbl=8)     # other order
    pts = np.random.default_rng(2).uniform(0.2, 0.8, size=(6, 3)) * np.array(p1.extent)
    p4 = W.small_problem("iso", (40, 40, 40), 8, nt=10, seed=63, src_at=pts, nrec=4, nbl=8)  # 6 sources
    shots = [fdw.Shot(p, torch_dev, nslots=2) for p in (p1, p2, p3, p4)]
    b = fdw.fdw_batch_create()
    try:
        for other in shots[1:]:
            with pytest.raises(fdw.FdwError) as e:
                fdw.fdw_batch_apply(b, [shots[0].op, other.op], [0, 0], [4, 4])
            assert e.value.code == fdw.FDW_ERR_ARG
        with pytest.raises(fdw.FdwError) as e:
            fdw.fdw_batch_apply(b, [shots[0].op], [0], [10])  # beyond the 10 source samples
        assert e.value.code == fdw.FDW_ERR_ARG
        fdw.fdw_batch_apply(b, [shots[0].op], [0], [9])
        torch_sync()
    finally:
        fdw.fdw_batch_destroy(b)
        for s in shots:
            s.close()


def torch_sync():
    import torch
    torch.cuda.synchronize()


def test_server_large_shots_run_alone(torch_dev):
    """Shots of 4 Mi grid points or more get buckets of their own (even with
    one shape) and run the single-shot kernels one at a time; their buckets
    are dropped when they finish.  Results equal the plain per-shot solves bit
    for bit, and the small request beside them equals its alone-served self."""
    reqs = [W.serve_problem("iso", 3, 162, 4, 24, seed=90 + k, nbl=8) for k in range(2)]
    reqs.append(W.serve_problem("iso", 2, 201, 8, 30, seed=92, nbl=10))
    assert all(np.prod(p.shape) >= 1 << 22 for p in reqs[:2])
    say("large shots")
    out, stats = serve_all(reqs, stagger=1)
    assert stats["completed"] == 3 and stats["buckets"] == 1, stats
    for i in (0, 1):
        tr, f = run_alone(reqs[i], torch_dev)
        np.testing.assert_array_equal(out[i][0], tr)
        np.testing.assert_array_equal(out[i][1], f["u"][1])
    alone = serve_all([reqs[2]])[0][0]
    np.testing.assert_array_equal(out[2][0], alone[0])
    np.testing.assert_array_equal(out[2][1], alone[1])



def test_server_wide_isotropic_shot(torch_dev):
    """A served isotropic request whose padded fields pass 4 GiB (1056 x 1040
    x 1040) gets a bucket of its own and runs the raw-buffer single-shot form:
    its traces equal, bit for bit, those of a plain 101^3 solve around the
    same source (the wave reaches no boundary in 10 steps); a small request
    served beside it equals its alone-served self."""
    from test_gpu_parity import wide_problems
    small, big = wide_problems()
    other = W.serve_problem("iso", 2, 201, 8, 30, seed=93, nbl=10)
    say("served wide shot", big.shape)
    tr_small, _ = run_alone(small, torch_dev)
    out, stats = serve_all([big, other], keep_field=False)
    assert stats["completed"] == 2, stats
    np.testing.assert_array_equal(out[0][0], tr_small)
    alone = serve_all([other], keep_field=False)[0][0]
    np.testing.assert_array_equal(out[1][0], alone[0])
