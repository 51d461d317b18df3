"""The plain solver as the fallback of warm-started solves
(rtg_solve_batched_fallback).

A batch of four 32x32x3 problems (the cfg1 generator, seeds 0..3) is solved
with a bfloat16 basis, at most 5 steps, stopping at the discrepancy level
eta*delta, from starting guesses chosen so that the warm start fails in the
two ways the fallback catches:
  problem 0: X0 = C (an ordinary warm start);
  problem 1: X0 = C + 1e3 * noise, far from the solution: the residual does
             not reach eta*delta within 5 steps (NOT_CONVERGED);
  problem 2: X0 = C with one NaN pixel: beta is not finite (NONFINITE);
  problem 3: X0 = the ground truth.
Every problem whose flags meet the mask must carry RTG_F_FALLBACK and hold
the plain float32 solve from X0 = 0 with m = 20 (checked against the float64
oracle's plain solve); every other problem must hold exactly what
rtg_solve_batched returns for the warm-started batch."""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.gmres import rtg_gmres
import _util as U

pytestmark = pytest.mark.gpu


def _warm_batch():
    from paper_2603_00839_amd import rtg
    probs = [synth.cfg1(s) for s in range(4)]
    ops, sks, Cs, X0s, prm, refs = [], [], [], [], [], []
    rng = np.random.default_rng(21)
    for k, p in enumerate(probs):
        C, delta = U.observation(p)
        op_o, sk_o = U.oracle_pair(p)
        refs.append(rtg_gmres(op_o, sk_o, C, 20, delta=delta, eta=1.01))
        if k == 1:
            x0 = C + 1e3 * rng.standard_normal(C.shape).astype(np.float32)
        elif k == 2:
            x0 = C.copy()
            x0[5, 7, 1] = np.nan
        elif k == 3:
            x0 = p.x_true
        else:
            x0 = C
        og, sg = U.gpu_pair(p)
        ops.append(og)
        sks.append(sg)
        Cs.append(U.to_dev(C))
        X0s.append(U.to_dev(x0))
        prm.append(rtg.make_params(5, rtg.BF16, delta=delta, eta=1.01, stop_res=1.01 * delta))
    return ops, sks, Cs, X0s, prm, refs


def test_fallback_resolves_failed_warm_starts_with_the_plain_solver():
    from paper_2603_00839_amd import rtg
    print("[case] fallback: 4 x cfg1, bf16 warm start, m' = 5", file=sys.stderr, flush=True)
    ops, sks, Cs, X0s, prm, refs = _warm_batch()
    # the warm-started batch alone
    plain = rtg.BatchPlan(ops, sks, Cs, X0s, prm)
    plain.run()
    warm_infos = plain.infos()
    warm_X = [U.from_dev(x) for x in plain.outs]
    # the same batch with the plain solver as the fallback
    fb = rtg.BatchPlan(ops, sks, Cs, X0s, prm, fallback=(20, rtg.F32))
    fb.run()
    infos = fb.infos()
    mask = rtg.FLAG_NOT_CONVERGED | rtg.FLAG_NONFINITE
    failed = [k for k in range(4) if warm_infos[k].flags & mask]
    print("warm flags", [i.flags for i in warm_infos], "iters", [i.iters for i in warm_infos],
          "after", [i.flags for i in infos], [i.iters for i in infos], file=sys.stderr)
    assert warm_infos[1].flags & rtg.FLAG_NOT_CONVERGED
    assert warm_infos[2].flags & rtg.FLAG_NONFINITE
    assert 1 in failed and 2 in failed
    assert fb.n_fallback == len(failed)
    for k in range(4):
        X = U.from_dev(fb.outs[k])
        if k in failed:
            assert infos[k].flags & rtg.FLAG_FALLBACK, (k, infos[k].flags)
            assert not infos[k].flags & mask
            assert infos[k].iters == refs[k].m_eff
            assert U.rel(X, refs[k].X) < 1e-4, (k, U.rel(X, refs[k].X))
        else:
            assert infos[k].flags == warm_infos[k].flags and infos[k].iters == warm_infos[k].iters
            np.testing.assert_array_equal(X, warm_X[k])


def test_fallback_argument_errors():
    from paper_2603_00839_amd import rtg
    print("[case] fallback argument errors", file=sys.stderr, flush=True)
    p = synth.cfg1(0)
    C, delta = U.observation(p)
    og, sg = U.gpu_pair(p)
    prm = [rtg.make_params(5, rtg.BF16, delta=delta, stop_res=1.01 * delta)]
    plan = rtg.BatchPlan([og], [sg], [U.to_dev(C)], [None], prm, fallback=(20, rtg.F32, 64))
    with pytest.raises(rtg.RTGError, match="invalid argument"):
        plan.run()
    # an fb_m the 16x16x3 sketch cannot take (m + 1 > L) has no workspace size
    with pytest.raises(rtg.RTGError):
        rtg.BatchPlan([og], [sg], [U.to_dev(C)], [None], prm, fallback=(1000, rtg.F32))


def test_fallback_in_two_calls_matches_the_single_call():
    """rtg_solve_batched_fallback_begin/_end give bit for bit what
    rtg_solve_batched_fallback gives, also with other work queued on the
    stream between the two calls (here the single-call solve of a second
    plan), and _end with no pending _begin is an argument error."""
    import torch
    from paper_2603_00839_amd import rtg
    print("[case] fallback begin/end: 4 x cfg1", file=sys.stderr, flush=True)
    ops, sks, Cs, X0s, prm, _ = _warm_batch()
    one = rtg.BatchPlan(ops, sks, Cs, X0s, prm, fallback=(20, rtg.F32))
    one.run()
    want = [U.from_dev(x) for x in one.outs]
    want_flags = [i.flags for i in one.infos()]
    two = rtg.BatchPlan(ops, sks, Cs, X0s, prm, fallback=(20, rtg.F32))
    other = rtg.BatchPlan(ops, sks, Cs, X0s, prm, fallback=(20, rtg.F32))
    for rep in range(2):
        for x in two.outs:
            x.fill_(float("nan"))
        two.begin()
        other.run()               # queued between the two halves
        two.end()
        torch.cuda.synchronize()
        assert two.n_fallback == one.n_fallback
        assert [i.flags for i in two.infos()] == want_flags
        for k in range(4):
            np.testing.assert_array_equal(U.from_dev(two.outs[k]), want[k])
    # a second end() has no begin() to finish
    with pytest.raises(rtg.RTGError, match="invalid argument"):
        two.end()
