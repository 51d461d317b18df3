"""General (non-separable) PSF operator (eqs. (56)-(57)) on the GPU against
the float64 oracle: the operator itself (float32 and bfloat16 input,
residual form, stencil radii of every tier, ragged tiles), the sketched
Arnoldi process (W sketched after it is formed), RTG-GMRES solves (discrepancy
and fixed mu, an initial guess, the identity sketch, a bfloat16 basis), a
batch of uneven PSF problems, and the argument errors (mixed operator kinds
in a batch, Golub-Kahan)."""
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.arnoldi import sketched_global_arnoldi
from oracle.gmres import rtg_gmres
from oracle.operator import PSFOperator, make_observation
from oracle.sketch import Sketch, identity_sketch
import _util as U

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def oracle_psf(p):
    return PSFOperator(p.psf, p.b_band, p.dims), Sketch(p.om1, p.om2, p.om3)


def gpu_psf(p, identity=False):
    from paper_2603_00839_amd import rtg
    I1, I2, J = p.dims
    op = rtg.setup_operator_psf(I1, I2, J, p.psf, p.b_band)
    sk = rtg.setup_sketch(I1, I2, J) if identity else rtg.setup_sketch(I1, I2, J, p.om1, p.om2, p.om3)
    return op, sk


def observation(p):
    op, _ = oracle_psf(p)
    C, delta, _ = make_observation(op, p.x_true, p.noise_dir, p.nu)
    return C.astype(np.float32), float(delta)


OP_SHAPES = [
    # I1, I2, J, r
    (48, 40, 3, 4),       # ragged i1 and i2 tiles
    (72, 70, 2, 8),       # tier 8, two channels
    (64, 36, 1, 12),      # tier 12, one channel
    (136, 33, 5, 3),      # several row tiles, five channels (JT = 8)
]


@pytest.mark.parametrize("shape", OP_SHAPES)
def test_psf_operator_parity(shape):
    import torch
    from paper_2603_00839_amd import rtg
    I1, I2, J, r = shape
    banner("psf operator", shape)
    p = synth.psf_problem(40 + I1, I1, I2, J, r=r, l1=8, l2=8, m=4)
    op_o, _ = oracle_psf(p)
    op_g, _ = gpu_psf(p)
    rng = np.random.default_rng(I1 + r)
    X = rng.standard_normal(p.dims).astype(np.float32)
    C = rng.standard_normal(p.dims).astype(np.float32)
    Y = U.from_dev(rtg.apply_operator(op_g, U.to_dev(X)))
    ref = op_o(X)
    assert U.maxrel(Y, ref) < 1e-5
    Yr = U.from_dev(rtg.apply_operator(op_g, U.to_dev(X), C=U.to_dev(C)))
    assert U.maxrel(Yr, C - ref) < 1e-5
    Yb = U.from_dev(rtg.apply_operator(op_g, U.to_dev(X, torch.bfloat16)))
    assert U.maxrel(Yb, op_o(U.bf16_round(X))) < 1e-5


def test_psf_arnoldi_parity():
    from paper_2603_00839_amd import rtg
    banner("psf arnoldi")
    p = synth.psf_problem(7, 48, 40, 3, r=4, l1=12, l2=10, m=10)
    op_o, sk_o = oracle_psf(p)
    op_g, sk_g = gpu_psf(p)
    C, _ = observation(p)
    out = rtg.arnoldi(op_g, sk_g, U.to_dev(C), 10, rtg.F32, bd_tol=1e-6)
    ar = sketched_global_arnoldi(op_o, sk_o, C.astype(np.float64), 10)
    H = out["H"].cpu().numpy()
    print(f"beta {out['beta'].item():.8e} ({ar.beta:.8e}) H maxrel {U.maxrel(H, ar.H):.3e}", file=sys.stderr)
    np.testing.assert_allclose(out["beta"].item(), ar.beta, rtol=1e-5)
    assert U.maxrel(H, ar.H) < 1e-4


@pytest.mark.parametrize("case", ["discrepancy", "fixed_x0", "identity_sketch"])
def test_psf_solve_matches_oracle(case):
    from paper_2603_00839_amd import rtg
    banner("psf solve", case)
    p = synth.psf_problem(11, 64, 48, 3, r=4, l1=16, l2=12, m=16)
    op_o, sk_o = oracle_psf(p)
    op_g, sk_g = gpu_psf(p, identity=(case == "identity_sketch"))
    C, delta = observation(p)
    X0 = None
    if case == "fixed_x0":
        X0 = (0.5 * p.x_true).astype(np.float32)
        prm = rtg.make_params(16, rtg.F32, mu=2e-3)
        ref = rtg_gmres(op_o, sk_o, C, 16, X0=X0, mu=2e-3)
    elif case == "identity_sketch":
        prm = rtg.make_params(16, rtg.F32, delta=delta, eta=1.01)
        ref = rtg_gmres(op_o, identity_sketch(), C, 16, delta=delta, eta=1.01)
    else:
        prm = rtg.make_params(16, rtg.F32, delta=delta, eta=1.01)
        ref = rtg_gmres(op_o, sk_o, C, 16, delta=delta, eta=1.01)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None if X0 is None else U.to_dev(X0), prm)
    info = rtg.read_info(ib)
    X = U.from_dev(Xg)
    print(f"iters {info.iters} ({ref.m_eff}) flags {info.flags} ({ref.flags}) mu {info.mu:.6e} ({ref.mu:.6e}) "
          f"rel {U.rel(X, ref.X):.3e} RE {U.rel(X, p.x_true):.4f}", file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    np.testing.assert_allclose(info.beta, ref.beta, rtol=1e-5)
    np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
    assert U.rel(X, ref.X) < 1e-4


def test_psf_bf16_basis_restores_like_the_oracle():
    """bfloat16 basis with a general PSF (no fused step): the restoration
    error stays within 1 % of the float64 oracle's."""
    from paper_2603_00839_amd import rtg
    banner("psf bf16")
    p = synth.psf_problem(12, 64, 48, 3, r=4, l1=16, l2=12, m=16)
    op_o, sk_o = oracle_psf(p)
    op_g, sk_g = gpu_psf(p)
    C, delta = observation(p)
    prm = rtg.make_params(16, rtg.BF16, delta=delta, eta=1.01)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    ref = rtg_gmres(op_o, sk_o, C, 16, delta=delta, eta=1.01)
    re_g, re_o = U.rel(U.from_dev(Xg), p.x_true), U.rel(ref.X, p.x_true)
    print(f"RE bf16 {re_g:.5f} oracle {re_o:.5f}", file=sys.stderr)
    assert re_g <= 1.01 * re_o


def test_psf_batched_uneven():
    import torch
    from paper_2603_00839_amd import rtg
    banner("psf batched")
    shapes = [(48, 40, 3, 4, 10), (72, 24, 2, 3, 8), (40, 40, 3, 6, 12)]
    ops, sks, Cs, prms, refs = [], [], [], [], []
    for I1, I2, J, r, m in shapes:
        p = synth.psf_problem(200 + I1, I1, I2, J, r=r, l1=8, l2=8, m=m)
        op_o, sk_o = oracle_psf(p)
        op_g, sk_g = gpu_psf(p)
        C, delta = observation(p)
        ops.append(op_g); sks.append(sk_g); Cs.append(U.to_dev(C))
        prms.append(rtg.make_params(m, rtg.F32, delta=delta, eta=1.01))
        refs.append(rtg_gmres(op_o, sk_o, C, m, delta=delta, eta=1.01))
    plan = rtg.solve_batched(ops, sks, Cs, [None] * 3, prms)
    torch.cuda.synchronize()
    for b, ref in enumerate(refs):
        info = plan.infos()[b]
        X = U.from_dev(plan.outs[b])
        print(f"problem {b}: iters {info.iters} ({ref.m_eff}) mu {info.mu:.6e} ({ref.mu:.6e}) "
              f"rel {U.rel(X, ref.X):.3e}", file=sys.stderr)
        assert info.iters == ref.m_eff and info.flags == ref.flags
        np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
        assert U.rel(X, ref.X) < 1e-4


def test_psf_argument_errors():
    import torch
    from paper_2603_00839_amd import rtg
    banner("psf argument errors")
    p = synth.psf_problem(3, 32, 16, 3, r=2, l1=8, l2=8, m=4)
    op_g, sk_g = gpu_psf(p)
    q = synth.small_problem(3, 32, 16, 3, 2, 2, 1, 8, 8, 3, 4)
    op_s, sk_s = U.gpu_pair(q)
    C = U.to_dev(observation(p)[0])
    prm = rtg.make_params(4, rtg.F32, mu=1e-3)
    with pytest.raises(rtg.RTGError):         # a PSF and a banded operator in one batch
        rtg.solve_batched([op_g, op_s], [sk_g, sk_s], [C, C], [None, None], [prm, prm])
    with pytest.raises(rtg.RTGError):         # Golub-Kahan needs the banded adjoint
        rtg.solve(op_g, sk_g, C, None, rtg.make_params(4, rtg.F32, mu=1e-3, method=rtg.METHOD_GOLUB_KAHAN))
    with pytest.raises(rtg.RTGError):         # PSF radius beyond the supported 12
        rtg.setup_operator_psf(64, 64, 3, np.ones((27, 27), np.float32), p.b_band)
    torch.cuda.synchronize()
