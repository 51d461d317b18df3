"""GCV selection of mu (Sec. 3, parameter selection via GCV) in the GPU
solve, against the float64 oracle minimising the same function on its own
H.  Bars of the float32 solver: mu within 1e-3 relative, solutions within
1e-4 relative Frobenius error; and the GPU's mu is a minimiser: GCV of the
oracle's projected problem at the GPU's mu within 1e-6 of its minimum."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.gmres import rtg_gmres
from oracle.projected import SVDProblem, gcv
import _util as U

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def check(info, X, ref):
    P = SVDProblem(ref.arnoldi.H, ref.arnoldi.beta)
    g_ref, g_gpu = gcv(P, ref.mu), gcv(P, info.mu)
    print(f"iters {info.iters} (oracle {ref.m_eff}) mu {info.mu:.6e} (oracle {ref.mu:.6e}) "
          f"GCV {g_gpu:.6e} (oracle {g_ref:.6e}) rel {U.rel(X, ref.X):.3e}", file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
    assert g_gpu <= g_ref * (1 + 1e-6)
    assert U.rel(X, ref.X) < 1e-4


@pytest.mark.parametrize("cfg,m", [("cfg1", 20), ("cfg1", 8)])
def test_gcv_solve_matches_oracle(cfg, m):
    from paper_2603_00839_amd import rtg
    banner("gcv solve", cfg, m)
    p = getattr(synth, cfg)(0)
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, _ = U.observation(p)
    prm = rtg.make_params(m, rtg.F32, bd_tol=1e-6, mu_rule=rtg.MU_GCV)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    ref = rtg_gmres(op_o, sk_o, C, m, bd_tol=1e-12, mu_rule="gcv")
    check(rtg.read_info(ib), U.from_dev(Xg), ref)


def test_gcv_mixed_with_other_rules_in_one_batch():
    """A batch whose problems choose mu by GCV, by the discrepancy principle
    and fixed: each matches the oracle run with its own rule."""
    import torch
    from paper_2603_00839_amd import rtg
    banner("gcv batched")
    shapes = [(48, 40, 3, 4, 4, 1, 12), (64, 24, 2, 5, 3, 1, 10), (40, 40, 3, 3, 3, 1, 14)]
    rules = ["gcv", "discrepancy", "fixed"]
    ops, sks, Cs, prms, refs, outs = [], [], [], [], [], []
    for (I1, I2, J, r1, r2, rB, m), rule in zip(shapes, rules):
        p = synth.small_problem(90 + I1, I1, I2, J, r1, r2, rB, 8, 8, J, m, nu=1e-2, random_bands=True)
        op_o, sk_o = U.oracle_pair(p)
        op_g, sk_g = U.gpu_pair(p)
        C, delta = U.observation(p)
        if rule == "gcv":
            prm = rtg.make_params(m, rtg.F32, mu_rule=rtg.MU_GCV)
            ref = rtg_gmres(op_o, sk_o, C, m, mu_rule="gcv")
        elif rule == "discrepancy":
            prm = rtg.make_params(m, rtg.F32, delta=delta, eta=1.01)
            ref = rtg_gmres(op_o, sk_o, C, m, delta=delta, eta=1.01)
        else:
            prm = rtg.make_params(m, rtg.F32, mu=3e-3)
            ref = rtg_gmres(op_o, sk_o, C, m, mu=3e-3)
        ops.append(op_g); sks.append(sk_g); Cs.append(U.to_dev(C)); prms.append(prm); refs.append(ref)
    plan = rtg.solve_batched(ops, sks, Cs, [None] * 3, prms)
    torch.cuda.synchronize()
    for b, (rule, ref) in enumerate(zip(rules, refs)):
        info = plan.infos()[b]
        X = U.from_dev(plan.outs[b])
        print(f"problem {b} ({rule}):", end=" ", file=sys.stderr)
        if rule == "gcv":
            check(info, X, ref)
        else:
            print(f"mu {info.mu:.6e} (oracle {ref.mu:.6e}) rel {U.rel(X, ref.X):.3e}", file=sys.stderr)
            assert info.iters == ref.m_eff and info.flags == ref.flags
            np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
            assert U.rel(X, ref.X) < 1e-4
