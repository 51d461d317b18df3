"""Sketched Block Golub-Kahan (Sec. 4.5) on the GPU against the float64
oracle.

* One-step parity: every coefficient the GPU computed, alpha_k and
  beta_{k+1}, against the oracle's float64 Theta-norm of the same update of
  the GPU's own stored tensors, and every stored tensor against the oracle's
  update of its predecessors (the bidiagonal relations, with the operator
  and its adjoint applied in float64).  This holds each step to float32
  rounding independently of how far the float32 and float64 recurrences
  drift apart over many steps (the short recurrence keeps no
  reorthogonalisation).
* End to end: beta_1, the bidiagonal matrix, mu and X against the oracle's
  own run on the same canonical float32 inputs, alone and batched (uneven
  shapes, mixed mu rules, an initial guess).
"""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.golub_kahan import sketched_golub_kahan, rgk_solve
import _util as U

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def one_step_parity(op_o, sk_o, U_t, V_t, B, m_done, tol_coef, tol_vec):
    """Coefficients and stored tensors of the GPU bidiagonalisation against
    float64 updates of the GPU's own stored tensors."""
    worst_c, worst_v = 0.0, 0.0
    for k in range(m_done):
        a, b = B[k, k], B[k + 1, k]
        # alpha_k from U_k (and beta_k, V_{k-1}); V_k is that update over alpha_k
        PU = op_o.transpose_apply(U_t[k])
        Z = PU - (B[k, k - 1] * V_t[k - 1] if k > 0 else 0.0)
        a_ref = sk_o.norm(Z)
        worst_c = max(worst_c, abs(a - a_ref) / sk_o.norm(PU))
        worst_v = max(worst_v, U.rel(V_t[k], Z / a))
        # beta_{k+1} from V_k and U_k; U_{k+1} is that update over beta_{k+1}
        PV = op_o(V_t[k])
        Wk = PV - a * U_t[k]
        b_ref = sk_o.norm(Wk)
        worst_c = max(worst_c, abs(b - b_ref) / sk_o.norm(PV))
        worst_v = max(worst_v, U.rel(U_t[k + 1], Wk / b))
    print(f"one-step parity: coefficients {worst_c:.3e}, stored tensors {worst_v:.3e}", file=sys.stderr)
    assert worst_c < tol_coef
    assert worst_v < tol_vec


def gpu_bidiag(p, m, basis=None, bd_tol=1e-6):
    from paper_2603_00839_amd import rtg
    basis = rtg.F32 if basis is None else basis
    op_g, sk_g = U.gpu_pair(p)
    C, _ = U.observation(p)
    out = rtg.golub_kahan(op_g, sk_g, U.to_dev(C), m, basis, bd_tol=bd_tol)
    import torch
    torch.cuda.synchronize()
    md = int(out["m_done"].item())
    B = out["B"].cpu().numpy()
    U_t = [U.from_dev(out["U"][k]) for k in range(md + 1)]
    V_t = [U.from_dev(out["V"][k]) for k in range(md)]
    return C, B, float(out["beta"].item()), md, U_t, V_t


SHAPES = [
    # I1, I2, J, r1, r2, rB, l1, l2, l3, m
    (48, 40, 3, 4, 4, 1, 12, 10, 3, 10),       # ragged tiles, full channel mix
    (72, 70, 2, 8, 5, 1, 16, 16, 2, 8),        # two channel tiles, wide band
    (40, 33, 5, 3, 2, 2, 8, 8, 3, 12),         # Om3 given (l3 < J), rB = 2
]


@pytest.mark.parametrize("shape", SHAPES)
def test_gk_bidiagonalisation_one_step_parity(shape):
    I1, I2, J, r1, r2, rB, l1, l2, l3, m = shape
    banner("gk bidiag", shape)
    p = synth.small_problem(300 + I1, I1, I2, J, r1, r2, rB, l1, l2, l3, m, random_bands=True)
    op_o, sk_o = U.oracle_pair(p)
    C, B, beta, md, U_t, V_t = gpu_bidiag(p, m)
    assert md == m
    # lower bidiagonal, zero elsewhere
    assert np.all(np.triu(B, 1) == 0) and np.all(np.tril(B, -2) == 0)
    np.testing.assert_allclose(beta, sk_o.norm(C), rtol=1e-5)
    assert U.rel(U_t[0] * beta, C) < 1e-6
    one_step_parity(op_o, sk_o, U_t, V_t, B, md, 1e-4, 1e-4)
    for X in U_t + V_t:
        assert abs(sk_o.norm(X) - 1.0) < 1e-4
    # the leading columns against the oracle's own run
    ref = sketched_golub_kahan(op_o, op_o.transpose_apply, sk_o, C.astype(np.float64), m)
    k0 = 3
    err = U.maxrel(B[:k0 + 1, :k0], ref.B[:k0 + 1, :k0])
    print(f"leading {k0} columns vs oracle {err:.3e}", file=sys.stderr)
    assert err < 1e-4


def test_gk_bidiagonalisation_bf16_basis():
    """bfloat16 basis: each stored tensor is its float64 update rounded to
    bfloat16 (relative error within 2^-8 per entry, 2^-7 in norm)."""
    from paper_2603_00839_amd import rtg
    banner("gk bidiag bf16")
    p = synth.small_problem(77, 64, 48, 3, 4, 4, 1, 16, 12, 3, 8, random_bands=True)
    op_o, sk_o = U.oracle_pair(p)
    C, B, beta, md, U_t, V_t = gpu_bidiag(p, 8, basis=rtg.BF16)
    assert md == 8
    one_step_parity(op_o, sk_o, U_t, V_t, B, md, 1e-3, 2.0 ** -7)


@pytest.mark.parametrize("cfg,m,rule", [("cfg1", 10, "discrepancy"), ("cfg1", 40, "discrepancy"),
                                        ("cfg1", 6, "fixed"), ("cfg1", 10, "gcv")])
def test_gk_solve_matches_oracle(cfg, m, rule):
    from paper_2603_00839_amd import rtg
    banner("gk solve", cfg, m, rule)
    p = getattr(synth, cfg)(0)
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    kw = dict(method=rtg.METHOD_GOLUB_KAHAN, bd_tol=1e-6)
    if rule == "discrepancy":
        prm = rtg.make_params(m, rtg.F32, delta=delta, eta=1.01, **kw)
        ref = rgk_solve(op_o, sk_o, C, m, delta=delta, eta=1.01)
    elif rule == "gcv":
        prm = rtg.make_params(m, rtg.F32, mu_rule=rtg.MU_GCV, **kw)
        ref = rgk_solve(op_o, sk_o, C, m, mu_rule="gcv")
    else:
        prm = rtg.make_params(m, rtg.F32, mu=2e-3, **kw)
        ref = rgk_solve(op_o, sk_o, C, m, mu=2e-3)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    info = rtg.read_info(ib)
    X = U.from_dev(Xg)
    print(f"iters {info.iters} (oracle {ref.m_eff}) flags {info.flags} ({ref.flags}) beta {info.beta:.8e} "
          f"({ref.beta:.8e}) mu {info.mu:.6e} ({ref.mu:.6e}) rel {U.rel(X, ref.X):.3e} "
          f"RE {U.rel(X, p.x_true):.4f} ({U.rel(ref.X, p.x_true):.4f})", file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    np.testing.assert_allclose(info.beta, ref.beta, rtol=1e-5)
    np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
    assert U.rel(X, ref.X) < 1e-4


def test_gk_batched_uneven_with_initial_guess():
    import torch
    from paper_2603_00839_amd import rtg
    banner("gk batched")
    shapes = [(48, 40, 3, 4, 4, 1, 10), (64, 24, 2, 5, 3, 1, 8), (40, 40, 3, 3, 3, 1, 12)]
    rules = ["discrepancy", "gcv", "fixed"]
    ops, sks, Cs, X0s, prms, refs = [], [], [], [], [], []
    for (I1, I2, J, r1, r2, rB, m), rule in zip(shapes, rules):
        p = synth.small_problem(500 + I1, I1, I2, J, r1, r2, rB, 8, 8, J, m, nu=1e-2, random_bands=True)
        op_o, sk_o = U.oracle_pair(p)
        op_g, sk_g = U.gpu_pair(p)
        C, delta = U.observation(p)
        X0 = (0.5 * p.x_true).astype(np.float32) if rule == "discrepancy" else None
        kw = dict(method=rtg.METHOD_GOLUB_KAHAN)
        if rule == "discrepancy":
            prm = rtg.make_params(m, rtg.F32, delta=delta, eta=1.01, **kw)
            ref = rgk_solve(op_o, sk_o, C, m, X0=X0, delta=delta, eta=1.01)
        elif rule == "gcv":
            prm = rtg.make_params(m, rtg.F32, mu_rule=rtg.MU_GCV, **kw)
            ref = rgk_solve(op_o, sk_o, C, m, mu_rule="gcv")
        else:
            prm = rtg.make_params(m, rtg.F32, mu=3e-3, **kw)
            ref = rgk_solve(op_o, sk_o, C, m, mu=3e-3)
        ops.append(op_g); sks.append(sk_g); Cs.append(U.to_dev(C)); prms.append(prm); refs.append(ref)
        X0s.append(None if X0 is None else U.to_dev(X0))
    plan = rtg.solve_batched(ops, sks, Cs, X0s, prms)
    torch.cuda.synchronize()
    infos = plan.infos()
    for b, (rule, ref) in enumerate(zip(rules, refs)):
        info = infos[b]
        X = U.from_dev(plan.outs[b])
        print(f"problem {b} ({rule}): iters {info.iters} ({ref.m_eff}) mu {info.mu:.6e} ({ref.mu:.6e}) "
              f"rel {U.rel(X, ref.X):.3e}", file=sys.stderr)
        assert info.iters == ref.m_eff and info.flags == ref.flags
        np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
        assert U.rel(X, ref.X) < 1e-4


def test_gk_argument_errors():
    """The all-identity sketch and batches mixing methods are refused before
    any launch."""
    import torch
    from paper_2603_00839_amd import rtg
    banner("gk argument errors")
    p = synth.small_problem(5, 32, 16, 3, 2, 2, 1, 8, 8, 3, 4, random_bands=True)
    op_g, sk_g = U.gpu_pair(p)
    ident = rtg.setup_sketch(32, 16, 3, None, None, None)
    C = U.to_dev(U.observation(p)[0])
    prm = rtg.make_params(4, rtg.F32, mu=1e-3, method=rtg.METHOD_GOLUB_KAHAN)
    with pytest.raises(rtg.RTGError):
        rtg.solve(op_g, ident, C, None, prm)
    prm_g = rtg.make_params(4, rtg.F32, mu=1e-3)
    with pytest.raises(rtg.RTGError):
        rtg.solve_batched([op_g, op_g], [sk_g, sk_g], [C, C], [None, None], [prm, prm_g])
    bad = rtg.make_params(4, rtg.F32, mu=1e-3, method=7)
    with pytest.raises(rtg.RTGError):
        rtg.solve(op_g, sk_g, C, None, bad)
    torch.cuda.synchronize()


def test_gk_bf16_basis_solve_restores_like_the_oracle():
    """Golub-Kahan with a bfloat16 basis (operator and AXPY tiles on the
    bfloat16 tensors, norms in float64): the restoration error stays within
    1 % of the float64 oracle's Golub-Kahan solve."""
    from paper_2603_00839_amd import rtg
    banner("gk bf16 solve")
    p = synth.cfg1(0)
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    prm = rtg.make_params(20, rtg.BF16, delta=delta, eta=1.01, method=rtg.METHOD_GOLUB_KAHAN)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    ref = rgk_solve(op_o, sk_o, C, 20, delta=delta, eta=1.01)
    re_g, re_o = U.rel(U.from_dev(Xg), p.x_true), U.rel(ref.X, p.x_true)
    info = rtg.read_info(ib)
    print(f"iters {info.iters} ({ref.m_eff}) RE bf16 {re_g:.5f} oracle {re_o:.5f}", file=sys.stderr)
    assert re_g <= 1.01 * re_o
