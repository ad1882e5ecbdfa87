"""The allocation-free apply (fdw_operator_apply_noalloc) against
fdw_operator_apply: two calls in a row, the second on a smaller operator (so
the shared device scratch holds the first call's values when the second
starts), each bit-equal to the plain apply of the same problem; the
isotropic operator (no scratch) passes through; an operator whose gradient
buffers exceed the scratch is refused."""
import numpy as np
import pytest

from paper_1807_03032_amd import workloads as W

from test_gpu_parity import TOL, oracle_run, rel_l2, say, torch_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def run(prob, dev, noalloc):
    import torch

    from paper_1807_03032_amd import fdw
    shot = fdw.Shot(prob, dev)
    try:
        s = torch.cuda.current_stream(dev).cuda_stream
        apply = fdw.fdw_operator_apply_noalloc if noalloc else fdw.fdw_operator_apply
        apply(shot.op, 0, prob.nt - 1, s)
        f = shot.fields(prob.nt - 1)
        tr = shot.traces()
    finally:
        shot.close()
    return f, tr


def same(a, b):
    fa, ta = a
    fb, tb = b
    for nm in fa:
        np.testing.assert_array_equal(fa[nm][0], fb[nm][0])
        np.testing.assert_array_equal(fa[nm][1], fb[nm][1])
    np.testing.assert_array_equal(ta, tb)


@pytest.mark.parametrize("kind,shapes", [("tti", [(70, 45, 52), (41, 33, 29)]), ("tti", [(150, 120), (90, 70)]),
                                         ("iso", [(60, 44, 38), (33, 27, 21)])])
def test_noalloc_equals_apply_two_calls(torch_dev, kind, shapes):
    probs = [W.small_problem(kind, sh, so, nt=nt, seed=400 + i, nsrc=1, nrec=12, nbl=4)
             for i, (sh, so, nt) in enumerate(zip(shapes, (12, 8), (25, 20)))]
    refs = [run(p, torch_dev, False) for p in probs]
    for p, ref in zip(probs, refs):  # back to back: the second reuses the first's scratch
        say("noalloc", kind, p.shape, p.so)
        got = run(p, torch_dev, True)
        same(got, ref)
    of, otr = oracle_run(probs[1])
    for nm, (ref_prev, ref_cur) in of.items():
        assert rel_l2(refs[1][0][nm][1], ref_cur) <= TOL
    assert rel_l2(refs[1][1], otr) <= TOL


def test_noalloc_refuses_operators_beyond_the_scratch(torch_dev):
    from paper_1807_03032_amd import fdw
    prob = W.small_problem("tti", (200, 200, 200), 4, nt=2, seed=410, nsrc=1, nrec=4, nbl=4)
    shot = fdw.Shot(prob, torch_dev)
    try:
        assert 2 * shot.lay.elems_per_slot > 16 << 20
        with pytest.raises(fdw.FdwError) as e:
            fdw.fdw_operator_apply_noalloc(shot.op, 0, 1)
        assert e.value.code == fdw.FDW_ERR_ARG and "scratch" in str(e.value)
    finally:
        shot.close()
