"""The batching form's tile autotuner (rtg_autotune_batched, rtg_tune_*).

* Every launch shape the autotuner may choose (operator tiles, staging and
  taps, sketch rows per wave, Gram pairs per workgroup), forced in turn
  through rtg_tune_set, on small uneven batches of four kinds: float32 RTG-GMRES
  (Toeplitz bands, J = 3 and 5 so that both channel tiles are candidates),
  the fused bfloat16 step with X0, sketched Golub-Kahan, and a general PSF
  (J = 3: asynchronous slab loads are a candidate).  float32 kinds: X within
  1e-4 of the float64 oracle and the oracle's step count.  bfloat16: X within
  1e-5 of the default shapes' X and the same step count (the shapes change
  which thread computes what, not the arithmetic).
* rtg_autotune_batched returns a resolved choice that later runs use, and
  writes neither X nor info.
* rtg_tune_set refuses values outside the documented set and choices the
  batch cannot use.
"""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.gmres import rtg_gmres
from oracle.golub_kahan import rgk_solve
from oracle.operator import PSFOperator, make_observation
from oracle.sketch import Sketch
import _util as U

pytestmark = pytest.mark.gpu

M = 6


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.fixture(autouse=True)
def clear_table():
    from paper_2603_00839_amd import rtg
    rtg.tune_clear()
    yield
    rtg.tune_clear()


def make_batch(kind):
    """(BatchPlan, oracle solutions or None, maxJ) for one kind of batch."""
    import torch
    from paper_2603_00839_amd import rtg
    ops, sks, Cs, X0s, prms, refs = [], [], [], [], [], []
    if kind == "psf":
        shapes = [(48, 40, 3, 3), (40, 56, 3, 2)]
        for s, (I1, I2, J, r) in enumerate(shapes):
            p = synth.psf_problem(70 + s, I1, I2, J, r=r, l1=12, l2=10, m=M)
            op_o = PSFOperator(p.psf, p.b_band, p.dims)
            sk_o = Sketch(p.om1, p.om2, p.om3)
            C, delta, _ = make_observation(op_o, p.x_true, p.noise_dir, p.nu)
            C, delta = C.astype(np.float32), float(delta)
            ops.append(rtg.setup_operator_psf(I1, I2, J, p.psf, p.b_band))
            sks.append(rtg.setup_sketch(I1, I2, J, p.om1, p.om2, p.om3))
            Cs.append(U.to_dev(C)); X0s.append(None)
            prms.append(rtg.make_params(M, rtg.F32, delta=delta, eta=1.01))
            refs.append(rtg_gmres(op_o, sk_o, C, M, delta=delta, eta=1.01))
        maxJ = 3
    else:
        shapes = [(48, 40, 3, 3, 2), (64, 24, 5, 2, 3)]
        bf16 = kind == "bf16"
        for s, (I1, I2, J, r1, r2) in enumerate(shapes):
            p = synth.small_problem(80 + s, I1, I2, J, r1, r2, 1, 12, 10, J, M)
            op_o, sk_o = U.oracle_pair(p)
            op_g, sk_g = U.gpu_pair(p)
            C, delta = U.observation(p)
            X0 = (0.5 * C).astype(np.float32) if s == 0 else None
            ops.append(op_g); sks.append(sk_g); Cs.append(U.to_dev(C))
            X0s.append(None if X0 is None else U.to_dev(X0))
            if kind == "gk":
                prms.append(rtg.make_params(M, rtg.F32, delta=delta, eta=1.01, method=rtg.METHOD_GOLUB_KAHAN))
                refs.append(rgk_solve(op_o, sk_o, C, M, X0=X0, delta=delta, eta=1.01))
            else:
                prms.append(rtg.make_params(M, rtg.BF16 if bf16 else rtg.F32, delta=delta, eta=1.01))
                refs.append(None if bf16 else rtg_gmres(op_o, sk_o, C, M, X0=X0, delta=delta, eta=1.01))
        maxJ = 5
    plan = rtg.BatchPlan(ops, sks, Cs, X0s, prms)
    torch.cuda.synchronize()
    return plan, refs, maxJ


def candidates(kind, maxJ):
    """The launch shapes rtg_autotune_batched may pick for this kind."""
    jts = [4, 8] if maxJ > 4 else [4]
    slabs = [0, 1, 2] if (kind == "psf" and maxJ <= 3) else [0, 1]
    phi = [dict(phi_jt=jt, phi_slab=sl, phi_toeplitz=tp)
           for jt in jts for sl in slabs for tp in ([0, 1] if (kind != "psf" and sl >= 1) else [0])]
    gram = [dict(gram_pairs=g) for g in (256, 512, 1024)]
    if kind == "bf16":
        step = [dict(step_rows=r, step_toeplitz=tp) for r in (2, 4) for tp in (0, 1)]
        # the step group against both tile forms, the operator group (R0 only) once
        return ([dict(tile_rows=tr, **st) for tr in (2, 4) for st in step] + phi + gram)
    return [dict(tile_rows=tr, **ph) for tr in (2, 4) for ph in phi] + gram


def solve(plan):
    import torch
    plan.run()
    torch.cuda.synchronize()
    return [U.from_dev(x) for x in plan.outs], plan.infos()


@pytest.mark.parametrize("kind", ["fp32", "bf16", "gk", "psf"])
def test_every_launch_shape_gives_the_same_solve(kind):
    from paper_2603_00839_amd import rtg
    banner("every launch shape", kind)
    plan, refs, maxJ = make_batch(kind)
    X_def, inf_def = solve(plan)
    cands = candidates(kind, maxJ)
    for c in cands:
        plan.set_tune(rtg.make_tune(**c))
        got = plan.tune().as_dict()
        for k, v in c.items():
            assert got[k] == v, (c, got)
        Xs, infos = solve(plan)
        for b in range(plan.count):
            if refs[b] is None:
                assert infos[b].iters == inf_def[b].iters, (c, b)
                assert U.rel(Xs[b], X_def[b]) < 1e-5, (c, b, U.rel(Xs[b], X_def[b]))
            else:
                ref = refs[b]
                iters = getattr(ref, "m_eff", None)
                assert infos[b].iters == iters, (c, b, infos[b].iters, iters)
                assert U.rel(Xs[b], ref.X) < 1e-4, (c, b, U.rel(Xs[b], ref.X))
    print(f"{kind}: {len(cands)} launch shapes, all within bounds", file=sys.stderr)


@pytest.mark.parametrize("kind", ["fp32", "bf16", "gk", "psf"])
def test_autotune_records_a_resolved_choice(kind):
    import torch
    from paper_2603_00839_amd import rtg
    banner("autotune", kind)
    plan, refs, maxJ = make_batch(kind)
    X_def, _ = solve(plan)
    for x in plan.outs:
        x.fill_(float("nan"))
    plan.info.fill_(0xAB)
    torch.cuda.synchronize()
    t, ms = plan.autotune(reps=2)
    chosen = t.as_dict()
    print(f"{kind}: chose {chosen} at {ms:.3f} ms", file=sys.stderr)
    assert all(v >= 0 for v in chosen.values()) and ms > 0
    assert plan.tune().as_dict() == chosen
    # outputs untouched
    for x in plan.outs:
        assert bool(torch.isnan(x).all())
    assert bool((plan.info == 0xAB).all())
    # the next run uses the choice and solves the same problems
    Xs, infos = solve(plan)
    for b in range(plan.count):
        if refs[b] is None:
            assert U.rel(Xs[b], X_def[b]) < 1e-5
        else:
            assert U.rel(Xs[b], refs[b].X) < 1e-4


def test_tune_set_refuses_impossible_choices():
    from paper_2603_00839_amd import rtg
    banner("tune errors")
    plan, _, _ = make_batch("fp32")
    bad = [dict(phi_jt=6), dict(tile_rows=3), dict(step_rows=1), dict(phi_slab=2),   # separable: no async slabs
           dict(phi_slab=3), dict(phi_toeplitz=2), dict(phi_slab=0, phi_toeplitz=1), dict(gram_pairs=300)]
    for c in bad:
        with pytest.raises(rtg.RTGError):
            plan.set_tune(rtg.make_tune(**c))
    t = rtg.make_tune()
    t.persist = 2
    with pytest.raises(rtg.RTGError):
        plan.set_tune(t)
    # random (non-Toeplitz) bands: no Toeplitz forms
    p = synth.small_problem(5, 32, 16, 3, 2, 2, 1, 8, 8, 3, 4, random_bands=True)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    plan2 = rtg.BatchPlan([op_g], [sk_g], [U.to_dev(C)], [None], [rtg.make_params(4, rtg.F32, delta=delta)])
    assert plan2.tune().phi_toeplitz == 0 and plan2.tune().step_toeplitz == 0
    for c in (dict(phi_toeplitz=1), dict(step_toeplitz=1)):
        with pytest.raises(rtg.RTGError):
            plan2.set_tune(rtg.make_tune(**c))
    # a recorded choice is forgotten by rtg_tune_clear
    plan.set_tune(rtg.make_tune(tile_rows=4, phi_slab=0))
    assert plan.tune().tile_rows == 4 and plan.tune().phi_slab == 0
    rtg.tune_clear()
    assert plan.tune().tile_rows == 2 and plan.tune().phi_slab == 1
