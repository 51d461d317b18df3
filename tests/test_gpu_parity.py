"""Parity of the HIP path (through the C ABI) with the float64 oracle on the
same seeded float32 inputs.  Tolerances: float32 arithmetic with float32
accumulation over at most a few hundred terms for the operator and sketch
(relative 1e-5 of the largest output); 1e-4 relative Frobenius error for
RTG-GMRES solutions (the float32 bar of the solver)."""
import math
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.operator import Operator
from oracle.sketch import Sketch
from oracle.gmres import rtg_gmres
from oracle.metrics import relative_error
import _util as U

pytestmark = pytest.mark.gpu


def banner(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


OP_SHAPES = [
    # (I1, I2, J, r1, r2, rB, random_bands)
    (8, 5, 1, 2, 1, 0, True),
    (40, 37, 3, 4, 3, 2, True),
    (64, 70, 5, 8, 8, 2, True),
    (136, 96, 3, 9, 9, 2, False),
    (72, 33, 12, 6, 5, 2, True),
]


@pytest.mark.parametrize("shape", OP_SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_operator_parity_small(shape, dtype):
    import torch
    from paper_2603_00839_amd import rtg
    I1, I2, J, r1, r2, rB, rnd = shape
    banner("operator", shape, dtype)
    p = synth.small_problem(1, I1, I2, J, r1, r2, rB, I1 // 2, max(I2 // 2, 1), J, 3, random_bands=rnd)
    op_o = Operator(p.a1_band, p.a2_band, p.b_band)
    op_g = rtg.setup_operator(I1, I2, J, p.a1_band, p.a2_band, p.b_band)
    X = p.x_true
    Xd = U.to_dev(X, torch.bfloat16 if dtype == "bf16" else None)
    Xref = U.bf16_round(X) if dtype == "bf16" else X
    Y = U.from_dev(rtg.apply_operator(op_g, Xd))
    assert U.maxrel(Y, op_o(Xref)) < 1e-5
    # residual form C - Phi(X)
    C = p.noise_dir
    R = U.from_dev(rtg.apply_operator(op_g, Xd, C=U.to_dev(C)))
    assert U.maxrel(R, C - op_o(Xref)) < 1e-5


@pytest.mark.parametrize("cfg", ["cfg2", "cfg3"])
def test_operator_parity_full_size(cfg):
    from paper_2603_00839_amd import rtg
    banner("operator full", cfg)
    p = getattr(synth, cfg)(0)
    op_o = Operator(p.a1_band, p.a2_band, p.b_band)
    op_g = rtg.setup_operator(*p.dims, p.a1_band, p.a2_band, p.b_band)
    Y = U.from_dev(rtg.apply_operator(op_g, U.to_dev(p.x_true)))
    assert U.maxrel(Y, op_o(p.x_true)) < 1e-5


SK_SHAPES = [
    # (I1, I2, J, l1, l2, l3 or None for identity)
    (32, 32, 3, 16, 16, None),
    (64, 48, 3, 16, 12, None),
    (40, 24, 7, 8, 5, 4),
    (520, 40, 2, 128, 10, None),
    (16, 100, 5, 3, 100, 2),
]


@pytest.mark.parametrize("shape", SK_SHAPES)
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_sketch_parity_small(shape, dtype):
    import torch
    from paper_2603_00839_amd import rtg
    I1, I2, J, l1, l2, l3 = shape
    banner("sketch", shape, dtype)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((I1, I2, J)).astype(np.float32)
    om1 = synth.sketch_matrix(rng, l1, I1)
    om2 = synth.sketch_matrix(rng, l2, I2)
    om3 = synth.sketch_matrix(rng, l3, J) if l3 else None
    om1, om2 = [None if o is None else o.astype(np.float32) for o in (om1, om2)]
    om3 = None if om3 is None else om3.astype(np.float32)
    sk_g = rtg.setup_sketch(I1, I2, J, om1, om2, om3)
    if dtype == "bf16":
        Xd = U.to_dev(X, torch.bfloat16)
        Xref = U.bf16_round(X)
        om1_ref = None if om1 is None else U.bf16_round(om1)
    else:
        Xd = U.to_dev(X)
        Xref = X
        om1_ref = om1
    S = rtg.sketch(sk_g, Xd).cpu().numpy()          # (l3, l2, l1) = column-major (l1, l2, l3)
    S = S.transpose(2, 1, 0).astype(np.float64)
    ref = Sketch(om1_ref, om2, om3)(Xref)
    assert U.maxrel(S, ref) < 2e-5


@pytest.mark.parametrize("cfg", ["cfg2", "cfg3"])
def test_sketch_parity_full_size(cfg):
    from paper_2603_00839_amd import rtg
    banner("sketch full", cfg)
    p = getattr(synth, cfg)(0)
    sk_g = rtg.setup_sketch(*p.dims, p.om1, p.om2, p.om3)
    S = rtg.sketch(sk_g, U.to_dev(p.x_true)).cpu().numpy().transpose(2, 1, 0)
    ref = Sketch(p.om1, p.om2, p.om3)(p.x_true)
    assert U.maxrel(S, ref) < 2e-5


def test_arnoldi_parity_and_relation():
    """H against the oracle's H on the same R0; the GPU basis satisfies the
    Arnoldi relation Phi(V_j) = sum_i h_ij V_i and is Theta-orthonormal."""
    from paper_2603_00839_amd import rtg
    banner("arnoldi cfg1")
    p = synth.cfg1(0)
    m = 12
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, _ = U.observation(p)
    out = rtg.arnoldi(op_g, sk_g, U.to_dev(C), m, bd_tol=1e-10)
    H = out["H"].cpu().numpy()
    ar = __import__("oracle.arnoldi", fromlist=["x"]).sketched_global_arnoldi(op_o, sk_o, C, m)
    assert int(out["m_done"].item()) == m
    np.testing.assert_allclose(out["beta"].item(), ar.beta, rtol=1e-5)
    assert U.maxrel(H, ar.H) < 1e-4
    V = [U.from_dev(out["V"][i]) for i in range(m + 1)]
    for j in range(m):
        lhs = op_o(V[j])
        rhs = sum(H[i, j] * V[i] for i in range(j + 2))
        assert U.rel(rhs, lhs) < 1e-5
    SV = out["SV"][:m].cpu().numpy().astype(np.float64)
    assert np.abs(SV @ SV.T - np.eye(m)).max() < 1e-4
    # the stored sketches are the sketches of the stored basis
    for i in range(m):
        np.testing.assert_allclose(np.linalg.norm(SV[i]), sk_o.norm(V[i]), rtol=1e-5)


MANY_CHANNELS = [
    # (I1, I2, J, r1, r2, rB, l1, l2, l3): J x (32-column tiles) above 48 and
    # l3 <= 16 take the Gram step's split finish (32 pairs per workgroup,
    # eight threads per pair): Om3 given (J = 40, l3 = 8) and the identity
    # (J = l3 = 16, four workgroups of 32 pairs); J = 20 with l3 = 20 keeps
    # the one-thread-per-pair finish
    (32, 64, 40, 2, 2, 2, 16, 16, 8),
    (16, 128, 16, 2, 2, 1, 8, 16, 16),
    (24, 96, 20, 3, 2, 1, 12, 24, 20),
]


@pytest.mark.parametrize("shape", MANY_CHANNELS)
def test_arnoldi_and_solve_many_channels(shape):
    """Many channels: every sketch pair's finish in the Gram step sums
    J x (column tiles) partials per buffer through the mode-3 factor.  H
    against the oracle, the Arnoldi relation on the stored basis, and the
    solve."""
    from paper_2603_00839_amd import rtg
    I1, I2, J, r1, r2, rB, l1, l2, l3 = shape
    banner("many channels", shape)
    m = 8
    p = synth.small_problem(90 + J, I1, I2, J, r1, r2, rB, l1, l2, l3, m, random_bands=True)
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, _ = U.observation(p)
    out = rtg.arnoldi(op_g, sk_g, U.to_dev(C), m, bd_tol=1e-10)
    H = out["H"].cpu().numpy()
    ar = __import__("oracle.arnoldi", fromlist=["x"]).sketched_global_arnoldi(op_o, sk_o, C, m)
    assert int(out["m_done"].item()) == m
    np.testing.assert_allclose(out["beta"].item(), ar.beta, rtol=1e-5)
    assert U.maxrel(H, ar.H) < 1e-4, U.maxrel(H, ar.H)
    V = [U.from_dev(out["V"][i]) for i in range(m + 1)]
    for j in range(m):
        assert U.rel(sum(H[i, j] * V[i] for i in range(j + 2)), op_o(V[j])) < 1e-5
    X, info, ref = solve_both(p)
    print(f"{shape}: H maxrel {U.maxrel(H, ar.H):.2e} solve iters {info.iters} ({ref.m_eff}) rel {U.rel(X, ref.X):.2e}",
          file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    assert U.rel(X, ref.X) < 1e-4


@pytest.mark.parametrize("shape", MANY_CHANNELS[:2])
def test_golub_kahan_many_channels(shape):
    """Sketched Golub-Kahan through the split finish of the Gram step (both
    sides' sketches finished with the mode-3 factor): X and the step count
    against the oracle."""
    from paper_2603_00839_amd import rtg
    from oracle.golub_kahan import rgk_solve
    I1, I2, J, r1, r2, rB, l1, l2, l3 = shape
    banner("golub-kahan many channels", shape)
    m = 8
    p = synth.small_problem(70 + J, I1, I2, J, r1, r2, rB, l1, l2, l3, m, random_bands=True)
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    prm = rtg.make_params(m, rtg.F32, delta=delta, eta=1.01, method=rtg.METHOD_GOLUB_KAHAN)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    info = rtg.read_info(ib)
    ref = rgk_solve(op_o, sk_o, C, m, delta=delta, eta=1.01)
    X = U.from_dev(Xg)
    print(f"{shape}: GK iters {info.iters} ({ref.m_eff}) rel {U.rel(X, ref.X):.2e}", file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    assert U.rel(X, ref.X) < 1e-4


def solve_both(p, basis="f32", mu=None, X0=None, stop_res=0.0, m=None):
    from paper_2603_00839_amd import rtg
    op_o, sk_o = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    m = p.m if m is None else m
    prm = rtg.make_params(m, rtg.BF16 if basis == "bf16" else rtg.F32,
                          mu=-1.0 if mu is None else mu, delta=delta, eta=1.01, stop_res=stop_res,
                          bd_tol=1e-6)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None if X0 is None else U.to_dev(X0), prm)
    info = rtg.read_info(ib)
    ref = rtg_gmres(op_o, sk_o, C, m, X0=X0, mu=mu, delta=None if mu is not None else delta,
                    eta=1.01, bd_tol=1e-12, stop_res=stop_res if stop_res > 0 else None)
    return U.from_dev(Xg), info, ref


@pytest.mark.parametrize("cfg", ["cfg1", "cfg2"])
def test_solve_parity_fp32(cfg):
    banner("solve fp32", cfg)
    p = getattr(synth, cfg)(0)
    X, info, ref = solve_both(p)
    print(f"{cfg}: iters {info.iters} mu {info.mu:.4e} (oracle {ref.mu:.4e}) flags {info.flags} "
          f"rel {U.rel(X, ref.X):.3e} RE {relative_error(p.x_true, X):.5f} (oracle "
          f"{relative_error(p.x_true, ref.X):.5f})", file=sys.stderr)
    assert info.iters == ref.m_eff and info.flags == ref.flags
    np.testing.assert_allclose(info.beta, ref.beta, rtol=1e-5)
    np.testing.assert_allclose(info.mu, ref.mu, rtol=1e-3)
    assert U.rel(X, ref.X) < 1e-4


def test_solve_bf16_restoration_error_cfg1():
    """BF16 basis and MFMA at nu = 1e-2: the restoration error stays within
    1% of the float64 oracle's."""
    banner("solve bf16 cfg1")
    p = synth.cfg1(0)
    X, info, ref = solve_both(p, basis="bf16")
    re_g = relative_error(p.x_true, X)
    re_o = relative_error(p.x_true, ref.X)
    print(f"cfg1 bf16: iters {info.iters} mu {info.mu:.4e} (oracle {ref.mu:.4e}) rel {U.rel(X, ref.X):.3e} "
          f"RE {re_g:.5f} (oracle {re_o:.5f})", file=sys.stderr)
    assert info.flags == 0
    assert re_g <= 1.01 * re_o


def test_solve_bf16_from_observation_cfg2():
    """cfg2 (nu = 1e-3) with a BF16 basis started from X0 = C: the basis only
    carries the correction, whose rounding stays below the noise level; the
    restoration error is within 1% of the plain float64 oracle (X0 = 0)."""
    banner("solve bf16 cfg2 from X0 = C")
    p = synth.cfg2(0)
    C, _ = U.observation(p)
    X, info, _ = solve_both(p, basis="bf16", X0=C, m=30)
    _, _, ref_plain = solve_both(p)
    re_g = relative_error(p.x_true, X)
    re_o = relative_error(p.x_true, ref_plain.X)
    print(f"cfg2 bf16 X0=C: iters {info.iters} mu {info.mu:.4e} flags {info.flags} RE {re_g:.5f} "
          f"(plain oracle {re_o:.5f})", file=sys.stderr)
    assert info.flags == 0
    assert re_g <= 1.01 * re_o


def test_bf16_batch_mixing_x0_and_none():
    """A bfloat16-basis batch in which some problems start from X0 and one
    from zero: where X0 is given the operator kernel stores R0 = C - Phi(X0)
    rounded to bfloat16 as V_1 and the first tile pass only sketches it;
    where it is absent the pass stores R0 = C itself.  Every problem holds
    what its own single-problem solve returns (to 1e-6), beta agrees
    with the float64 oracle's ||S(R0)|| to the bfloat16 rounding of R0, and
    the restoration error is within 1% of the oracle's from the same X0."""
    from paper_2603_00839_amd import rtg
    banner("bf16 batch, X0 given and absent")
    probs = [synth.cfg1(s) for s in range(3)]
    ops, sks, Cs, X0s, prm, x0_host, refs = [], [], [], [], [], [], []
    rng = np.random.default_rng(5)
    for k, p in enumerate(probs):
        C, delta = U.observation(p)
        x0 = None if k == 0 else (C if k == 1 else
                                  (0.5 * p.x_true + 0.01 * rng.standard_normal(C.shape)).astype(np.float32))
        og, sg = U.gpu_pair(p)
        ops.append(og)
        sks.append(sg)
        Cs.append(U.to_dev(C))
        X0s.append(None if x0 is None else U.to_dev(x0))
        x0_host.append(x0)
        prm.append(rtg.make_params(20, rtg.BF16, delta=delta, eta=1.01))
        op_o, sk_o = U.oracle_pair(p)
        refs.append(rtg_gmres(op_o, sk_o, C, 20, X0=x0, delta=delta, eta=1.01))
    plan = rtg.BatchPlan(ops, sks, Cs, X0s, prm)
    plan.run()
    infos = plan.infos()
    for k, p in enumerate(probs):
        X = U.from_dev(plan.outs[k])
        Xs, ib = rtg.solve(ops[k], sks[k], Cs[k], X0s[k], prm[k])
        inf1 = rtg.read_info(ib)
        re_g = relative_error(p.x_true, X)
        re_o = relative_error(p.x_true, refs[k].X)
        print(f"problem {k} (X0 {'none' if x0_host[k] is None else 'given'}): iters {infos[k].iters} "
              f"beta {infos[k].beta:.6e} (oracle {refs[k].beta:.6e}) RE {re_g:.5f} (oracle {re_o:.5f})",
              file=sys.stderr)
        assert U.rel(X, U.from_dev(Xs)) < 1e-6 and infos[k].iters == inf1.iters
        np.testing.assert_allclose(infos[k].beta, refs[k].beta, rtol=4e-3)
        assert re_g <= 1.01 * re_o


def test_bf16_from_zero_reports_unreachable_discrepancy():
    """From X0 = 0 at nu = 1e-3 the bfloat16 rounding of the basis (relative
    2^-9) exceeds the noise level: the projected least-squares residual
    cannot reach eta * delta and the solver says so."""
    from paper_2603_00839_amd import rtg
    banner("bf16 cfg2 from zero")
    p = synth.cfg2(0)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    _, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, rtg.make_params(50, rtg.BF16, delta=delta))
    info = rtg.read_info(ib)
    assert info.flags & rtg.FLAG_DISCREP_UNREACHABLE
    assert info.res_ls > 1.01 * delta


def test_solve_fixed_mu_with_x0():
    banner("solve fixed mu + X0")
    p = synth.cfg1(1)
    X0 = 0.5 * p.x_true + 0.01 * p.noise_dir
    X, info, ref = solve_both(p, mu=3e-3, X0=X0, m=15)
    assert info.iters == 15 and info.flags == 0
    assert U.rel(X, ref.X) < 1e-4


def test_stop_residual_matches_oracle_step():
    banner("solve stop_res")
    p = synth.cfg1(2)
    # stop at the oracle's LS residual after 9 steps (slightly above it)
    _, _, ref_full = solve_both(p, m=20)
    tau = float(ref_full.arnoldi.ls_res[8]) * 1.0001
    X, info, ref = solve_both(p, stop_res=tau, m=20)
    assert ref.m_eff <= 9 and info.iters == ref.m_eff
    assert U.rel(X, ref.X) < 1e-4


def test_breakdown_scaled_identity():
    """Phi = c Id: breakdown at j = 1 and X = X0 + R0 / c."""
    from paper_2603_00839_amd import rtg
    banner("breakdown")
    I1, I2, J, c = 16, 8, 3, 2.5
    one = np.ones((I1, 1), np.float32)
    op_g = rtg.setup_operator(I1, I2, J, one, np.ones((I2, 1), np.float32), np.full((J, 1), c, np.float32))
    rng = np.random.default_rng(0)
    sk_g = rtg.setup_sketch(I1, I2, J, (rng.standard_normal((8, I1)) / 3).astype(np.float32), None, None)
    C = rng.standard_normal((I1, I2, J)).astype(np.float32)
    X0 = rng.standard_normal((I1, I2, J)).astype(np.float32)
    prm = rtg.make_params(5, mu=0.0, bd_tol=1e-5)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), U.to_dev(X0), prm)
    info = rtg.read_info(ib)
    assert info.iters == 1 and info.flags & rtg.FLAG_BREAKDOWN
    assert U.rel(U.from_dev(Xg), X0 + (C - c * X0) / c) < 1e-5


def test_zero_residual_and_mu_inf():
    from paper_2603_00839_amd import rtg
    banner("edge: zero residual, mu inf")
    p = synth.cfg1(3)
    op_o, _ = U.oracle_pair(p)
    op_g, sk_g = U.gpu_pair(p)
    X0 = p.x_true
    C = U.from_dev(rtg.apply_operator(op_g, U.to_dev(X0))).astype(np.float32)
    # exact X0: R0 = C - Phi(X0) = 0 exactly (same kernel) -> X = X0
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), U.to_dev(X0), rtg.make_params(10, mu=0.0))
    info = rtg.read_info(ib)
    assert info.iters == 0
    np.testing.assert_array_equal(U.from_dev(Xg), X0.astype(np.float64))
    # noise estimate above ||R0||: mu = inf, y = 0, X = X0 = 0
    C2, delta = U.observation(p)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C2), None, rtg.make_params(10, delta=1e6))
    info = rtg.read_info(ib)
    assert info.flags & rtg.FLAG_MU_INF
    assert np.all(U.from_dev(Xg) == 0)


def test_nonfinite_input_is_flagged():
    from paper_2603_00839_amd import rtg
    banner("edge: NaN")
    p = synth.cfg1(4)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    C[3, 4, 1] = np.nan
    _, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, rtg.make_params(10, delta=delta))
    assert rtg.read_info(ib).flags & rtg.FLAG_NONFINITE


@pytest.mark.parametrize("basis", ["f32", "bf16"])
def test_nonfinite_at_step_two_returns_the_one_step_solve(basis):
    """A coefficient that overflows float32 at step 2 stops the solve with
    the one complete column: X, mu and the projected residual are those of
    the oracle's one-step solve (in float64 nothing overflows there).

    The bands are tridiagonal (diagonal 1, off-diagonals 0.5) except for
    A1[5, 5] = 1e20 and A2[7, 7] = 1e25; C is one pixel at (6, 8).  V_1 is
    zero on row 5 and column 7, so Phi(V_1) is finite; V_2 has an entry of
    about 0.2 at (5, 7), where Phi(V_2) and its sketch reach 1e44."""
    from paper_2603_00839_amd import rtg
    banner("edge: overflow at step 2", basis)
    I1, I2, J = 16, 16, 1

    def band(I, hot, big):
        b = np.zeros((I, 3), np.float32)
        b[:, 0] = 0.5
        b[:, 1] = 1.0
        b[:, 2] = 0.5
        b[hot, 1] = big
        return b

    a1, a2, bb = band(I1, 5, 1e20), band(I2, 7, 1e25), np.ones((1, 1), np.float32)
    rng = np.random.default_rng(8)
    o1 = (rng.standard_normal((8, I1)) / np.sqrt(8)).astype(np.float32)
    o2 = (rng.standard_normal((8, I2)) / np.sqrt(8)).astype(np.float32)
    C = np.zeros((I1, I2, J), np.float32)
    C[6, 8, 0] = 1.0
    op_o, sk_o = Operator(a1, a2, bb), Sketch(o1, o2, None)
    ref = rtg_gmres(op_o, sk_o, C, 1, mu=1e-3)
    full = rtg_gmres(op_o, sk_o, C, 2, mu=1e-3)
    assert full.m_eff == 2 and np.abs(full.arnoldi.V[1][5, 7, 0]) > 0.1     # the premise: V_2 at (5, 7)
    op_g = rtg.setup_operator(I1, I2, J, a1, a2, bb)
    sk_g = rtg.setup_sketch(I1, I2, J, o1, o2, None)
    prm = rtg.make_params(5, rtg.BF16 if basis == "bf16" else rtg.F32, mu=1e-3)
    Xg, ib = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    info = rtg.read_info(ib)
    assert info.flags & rtg.FLAG_NONFINITE and info.iters == 1, (info.flags, info.iters)
    assert np.all(np.isfinite(U.from_dev(Xg)))
    tol = 2e-2 if basis == "bf16" else 1e-4      # one bfloat16 rounding of V_1
    assert U.rel(U.from_dev(Xg), ref.X) < tol
    assert abs(info.res_proj - ref.res_proj) <= tol * ref.res_proj, (info.res_proj, ref.res_proj)
    # (the bfloat16 path sketches with Om1 rounded to bfloat16, so its beta
    # differs from the oracle's at that rounding)
    assert abs(info.beta - ref.beta) <= (1e-2 if basis == "bf16" else 1e-5) * ref.beta


def test_batched_uneven_problems_match_oracle():
    """Problems of different sizes, operators, m, mu rules and X0 in one batch."""
    import torch
    from paper_2603_00839_amd import rtg
    banner("batched uneven")
    specs = [
        (48, 32, 3, 4, 4, 2, 16, 16, 3, 12),
        (64, 80, 3, 6, 5, 2, 16, 20, 3, 15),
        (32, 48, 2, 3, 3, 1, 8, 12, 2, 9),
        (96, 40, 3, 9, 9, 2, 24, 10, 3, 20),
        (40, 24, 6, 2, 2, 2, 10, 6, 3, 8),
    ]
    probs, ops, sks, Cs, X0s, prms, refs = [], [], [], [], [], [], []
    for k, (I1, I2, J, r1, r2, rB, l1, l2, l3, m) in enumerate(specs):
        p = synth.small_problem(20 + k, I1, I2, J, r1, r2, rB, l1, l2, l3, m, nu=1e-2,
                                random_bands=(k % 2 == 1))
        op_o, sk_o = U.oracle_pair(p)
        C, delta = U.observation(p)
        X0 = 0.3 * p.x_true if k % 2 == 0 else None
        mu = 1e-2 if k == 2 else None
        ref = rtg_gmres(op_o, sk_o, C, m, X0=X0, mu=mu, delta=None if mu is not None else delta,
                        eta=1.01, bd_tol=1e-12)
        og, sg = U.gpu_pair(p)
        ops.append(og); sks.append(sg); Cs.append(U.to_dev(C))
        X0s.append(None if X0 is None else U.to_dev(X0))
        prms.append(rtg.make_params(m, mu=-1.0 if mu is None else mu, delta=delta))
        refs.append(ref)
    plan = rtg.solve_batched(ops, sks, Cs, X0s, prms)
    torch.cuda.synchronize()
    for k, (ref, X, info) in enumerate(zip(refs, plan.outs, plan.infos())):
        assert info.iters == ref.m_eff, k
        assert U.rel(U.from_dev(X), ref.X) < 1e-4, k


def test_solve_is_deterministic():
    import torch
    from paper_2603_00839_amd import rtg
    banner("determinism")
    p = synth.cfg1(5)
    op_g, sk_g = U.gpu_pair(p)
    C, delta = U.observation(p)
    prm = rtg.make_params(20, delta=delta)
    a, _ = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    b, _ = rtg.solve(op_g, sk_g, U.to_dev(C), None, prm)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
