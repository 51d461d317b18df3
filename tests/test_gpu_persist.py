"""One persistent launch for the Arnoldi process of a batch (rtg_tune.persist).

The persistent launch runs the stage bodies of the per-stage launches in the
same arithmetic: which workgroup takes a tile changes, not what the tile
computes, and every reduction keeps its fixed order.  So X and every info
field must equal, bit for bit, those of the per-stage launches of the same
batch with the same launch shapes -- which are themselves held to the float64
oracle (here again for the float32 batches).

* a small uneven batch (five shapes, J = 1..4, Toeplitz and general bands,
  X0 on three problems, a fixed mu on one, m = 6..15), float32 and mixed
  form: bitwise equal to the per-stage launches; float32: X within 1e-4 of
  the oracle with its step count;
* restarted RTG-GMRES (three problems with 0, 3 and 12 restarts): every
  cycle a persistent launch, bitwise equal to the per-stage launches and
  the oracle's steps, flags and X;
* the 256-problem uneven batch at full size in the mixed form (m = 40):
  bitwise equal to the per-stage launches, every problem at the discrepancy
  level;
* the failure path, forced from the host: with a wait limit of zero polls
  the launch is abandoned and every kernel still exits: every problem
  carries RTG_F_TIMEOUT, no steps, X = X0 (zero without X0); with the limit
  restored the same plan solves bitwise as before;
* the tune field: refused for batches that cannot take it; the autotuner's
  choice (persistent or not) solves within 1e-4 of the oracle.
"""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.gmres import rtg_gmres, rtg_gmres_restarted
from oracle.operator import Operator
from oracle.sketch import Sketch
import _util as U

pytestmark = pytest.mark.gpu

DEFAULT_WAIT = 1 << 22


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(autouse=True)
def clean_state():
    from paper_2603_00839_amd import rtg
    rtg.tune_clear()
    rtg.set_wait_limit(DEFAULT_WAIT)
    yield
    rtg.tune_clear()
    rtg.set_wait_limit(DEFAULT_WAIT)


SPECS = [
    # I1, I2, J, r1, r2, rB, l1, l2, l3, m
    (48, 32, 3, 4, 4, 1, 16, 16, 3, 12),
    (64, 80, 3, 6, 5, 2, 16, 20, 3, 15),
    (32, 48, 2, 3, 3, 1, 8, 12, 2, 9),
    (96, 40, 4, 9, 9, 2, 64, 10, 4, 10),
    (40, 24, 1, 2, 2, 0, 10, 6, 1, 6),
]


def small_batch(basis):
    import torch
    from paper_2603_00839_amd import rtg
    ops, sks, Cs, X0s, prms, refs, x0_host = [], [], [], [], [], [], []
    for k, (I1, I2, J, r1, r2, rB, l1, l2, l3, m) in enumerate(SPECS):
        p = synth.small_problem(40 + k, I1, I2, J, r1, r2, rB, l1, l2, l3, m, nu=1e-2,
                                random_bands=(k % 2 == 1))
        C, delta = U.observation(p)
        X0 = (0.3 * p.x_true).astype(np.float32) if k % 2 == 0 else None
        mu = 1e-2 if k == 2 else None
        og, sg = U.gpu_pair(p)
        ops.append(og); sks.append(sg); Cs.append(U.to_dev(C))
        X0s.append(None if X0 is None else U.to_dev(X0))
        x0_host.append(X0)
        prms.append(rtg.make_params(m, basis, mu=-1.0 if mu is None else mu, delta=delta, eta=1.01))
        if basis == rtg.F32:
            op_o, sk_o = U.oracle_pair(p)
            refs.append(rtg_gmres(op_o, sk_o, C, m, X0=X0, mu=mu, delta=None if mu is not None else delta,
                                  eta=1.01, bd_tol=1e-12))
    plan = rtg.BatchPlan(ops, sks, Cs, X0s, prms)
    torch.cuda.synchronize()
    return plan, refs, x0_host


def run(plan, persist):
    import torch
    from paper_2603_00839_amd import rtg
    plan.set_tune(rtg.make_tune(persist=persist))
    assert plan.tune().persist == persist
    plan.run()
    torch.cuda.synchronize()
    Xs = [x.cpu().numpy().copy() for x in plan.outs]
    infos = [(i.iters, i.flags, i.mu, i.beta, i.res_proj, i.res_ls) for i in plan.infos()]
    return Xs, infos


def assert_same(a, b, tag):
    Xa, ia = a
    Xb, ib = b
    for k in range(len(Xa)):
        assert ia[k] == ib[k], (tag, k, ia[k], ib[k])
        np.testing.assert_array_equal(Xa[k], Xb[k], err_msg=f"{tag} problem {k}")


@pytest.mark.parametrize("basis", ["f32", "mixed"])
def test_small_uneven_batch_bitwise_equal_to_per_stage_launches(basis):
    from paper_2603_00839_amd import rtg
    b = rtg.F32 if basis == "f32" else rtg.F32_BF16
    banner("persistent small uneven batch", basis)
    plan, refs, _ = small_batch(b)
    per_stage = run(plan, 0)
    persistent = run(plan, 1)
    assert_same(per_stage, persistent, basis)
    for k, ref in enumerate(refs):
        X = synth.from_device_layout(persistent[0][k]).astype(np.float64)
        print(f"problem {k}: iters {persistent[1][k][0]} ({ref.m_eff}) rel {U.rel(X, ref.X):.2e}", file=sys.stderr)
        assert persistent[1][k][0] == ref.m_eff
        assert U.rel(X, ref.X) < 1e-4
    # a second persistent run of the same plan (scheduling words and counters reset)
    assert_same(persistent, run(plan, 1), basis + " again")


def test_restarted_batch_persistent_cycles():
    import torch
    from paper_2603_00839_amd import rtg
    banner("persistent restarted batch")
    cases = [(48, 40, 3, 4, 0), (64, 24, 2, 5, 3), (40, 40, 3, 3, 12)]
    ops, sks, Cs, prms, refs = [], [], [], [], []
    for I1, I2, J, m, restarts in cases:
        p = synth.small_problem(60 + I1, I1, I2, J, 2, 1, 1, 8, 8, J, m, random_bands=True)
        a1 = p.a1_band.copy(); a1[:, 2] += 4.0
        a2 = p.a2_band.copy(); a2[:, 1] += 2.0
        bb = p.b_band.copy(); bb[:, 1] += 2.0
        op_o, sk_o = Operator(a1, a2, bb), Sketch(p.om1, p.om2, p.om3)
        C = (op_o(p.x_true) + 0.01 * p.noise_dir).astype(np.float32)
        eps = 1e-4 * sk_o.norm(C)
        ops.append(rtg.setup_operator(I1, I2, J, a1, a2, bb))
        sks.append(rtg.setup_sketch(I1, I2, J, p.om1, p.om2, p.om3))
        Cs.append(U.to_dev(C))
        prms.append(rtg.make_params(m, rtg.F32, mu=0.0, stop_res=eps, restarts=restarts))
        refs.append(rtg_gmres_restarted(op_o, sk_o, C, m, restarts, eps, mu=0.0))
    plan = rtg.BatchPlan(ops, sks, Cs, [None] * 3, prms)
    torch.cuda.synchronize()
    per_stage = run(plan, 0)
    persistent = run(plan, 1)
    assert_same(per_stage, persistent, "restarted")
    for k, ref in enumerate(refs):
        X = synth.from_device_layout(persistent[0][k]).astype(np.float64)
        assert persistent[1][k][0] == ref.iters and persistent[1][k][1] == ref.flags, (k, persistent[1][k], ref.iters)
        assert U.rel(X, ref.X) < 1e-4


def test_uneven_batch_of_256_mixed_persistent():
    import torch
    from paper_2603_00839_amd import rtg
    banner("persistent uneven batch 256, mixed form")
    probs = synth.cfg4(0, 256, m=40)
    ops, sks, Cs, prms = [], [], [], []
    for p in probs:
        og, sg = U.gpu_pair(p)
        C, delta = U.observation(p)
        ops.append(og); sks.append(sg); Cs.append(U.to_dev(C))
        prms.append(rtg.make_params(40, rtg.F32_BF16, delta=delta, eta=1.01))
    plan = rtg.BatchPlan(ops, sks, Cs, [None] * len(probs), prms)
    torch.cuda.synchronize()
    per_stage = run(plan, 0)
    persistent = run(plan, 1)
    assert_same(per_stage, persistent, "uneven 256")
    flags = {}
    for it, fl, *_ in persistent[1]:
        flags[fl] = flags.get(fl, 0) + 1
    print("flags", flags, file=sys.stderr)
    assert flags == {0: 256}


def test_wait_limit_abandons_the_launch_and_the_next_run_recovers():
    import torch
    from paper_2603_00839_amd import rtg
    banner("persistent launch abandoned at a zero wait limit")
    plan, _, x0_host = small_batch(rtg.F32)
    good = run(plan, 1)
    rtg.set_wait_limit(0)
    plan.run()
    torch.cuda.synchronize()
    infos = plan.infos()
    print("flags", [i.flags for i in infos], "iters", [i.iters for i in infos], file=sys.stderr)
    for k, inf in enumerate(infos):
        assert inf.flags & rtg.FLAG_TIMEOUT, (k, inf.flags)
        assert inf.iters == 0
        X = U.from_dev(plan.outs[k])
        expect = np.zeros_like(X) if x0_host[k] is None else x0_host[k].astype(np.float64)
        np.testing.assert_array_equal(X, expect)
    rtg.set_wait_limit(DEFAULT_WAIT)
    assert_same(good, run(plan, 1), "after the abandoned launch")


def test_persist_field_refused_where_it_cannot_run_and_autotuned_choice_solves():
    import torch
    from paper_2603_00839_amd import rtg
    banner("persist field")
    plan, refs, _ = small_batch(rtg.F32)
    for bad in (dict(persist=1, phi_slab=0), dict(persist=1, phi_jt=8), dict(persist=3)):
        with pytest.raises(rtg.RTGError):
            plan.set_tune(rtg.make_tune(**bad))
    # a bfloat16 basis runs the fused step kernel instead; J > 4 needs two channel tiles
    p = synth.small_problem(7, 32, 16, 3, 2, 2, 1, 8, 8, 3, 4)
    og, sg = U.gpu_pair(p)
    C, delta = U.observation(p)
    bf = rtg.BatchPlan([og], [sg], [U.to_dev(C)], [None], [rtg.make_params(4, rtg.BF16, delta=delta)])
    with pytest.raises(rtg.RTGError):
        bf.set_tune(rtg.make_tune(persist=1))
    p5 = synth.small_problem(8, 32, 16, 5, 2, 2, 1, 8, 8, 5, 4)
    og5, sg5 = U.gpu_pair(p5)
    C5, d5 = U.observation(p5)
    j5 = rtg.BatchPlan([og5], [sg5], [U.to_dev(C5)], [None], [rtg.make_params(4, rtg.F32, delta=d5)])
    with pytest.raises(rtg.RTGError):
        j5.set_tune(rtg.make_tune(persist=1))
    t, ms = plan.autotune(reps=1)
    print("autotuned", t.as_dict(), f"{ms:.3f} ms", file=sys.stderr)
    assert t.persist in (0, 1)
    plan.run()
    torch.cuda.synchronize()
    for k, ref in enumerate(refs):
        assert plan.infos()[k].iters == ref.m_eff
        assert U.rel(U.from_dev(plan.outs[k]), ref.X) < 1e-4
