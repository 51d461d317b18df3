"""Pins of the oracle's sketched Block Golub-Kahan solve (Sec. 4.5) against
facts that do not depend on how its recurrence is written:

* Phi^T is the Frobenius adjoint of Phi (and the transpose of its matrix);
* V_1..V_k span the Krylov space K_k(Phi^T Phi, Phi^T R0) and U_1..U_k span
  K_k(Phi Phi^T, R0), whatever norms scale them (explicit Krylov bases);
* the two bidiagonal relations hold entry by entry, and every basis tensor
  has unit sketched norm;
* with Omega = I it is textbook Golub-Kahan / LSQR: orthonormal bases, the
  iterate minimises ||c - A x|| over x0 + K_m (dense least squares), and
  B^T B is the Lanczos matrix of A^T A on that Krylov space;
* an orthogonal square Omega gives the Omega = I result, and scaling Omega
  by c leaves X unchanged.
"""
import numpy as np
import pytest

from oracle import tensor_algebra as ta
from oracle.golub_kahan import sketched_golub_kahan, rgk_solve, FLAG_BREAKDOWN
from oracle.operator import Operator
from oracle.sketch import Sketch, identity_sketch
from paper_2603_00839_amd import synth

from test_oracle_pins import rel, tiny_problem


def krylov(A, v0, k):
    """Orthonormal basis of span{v0, A v0, ..., A^{k-1} v0} (QR of the powers)."""
    K = np.empty((v0.size, k))
    v = v0 / np.linalg.norm(v0)
    for j in range(k):
        K[:, j] = v
        v = A @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    return Q


def out_of_span(Q, x):
    return float(np.linalg.norm(x - Q @ (Q.T @ x)) / np.linalg.norm(x))


def test_transpose_apply_is_the_frobenius_adjoint():
    p, op, _ = tiny_problem(seed=11)
    rng = np.random.default_rng(5)
    X = rng.standard_normal(p.dims)
    Y = rng.standard_normal(p.dims)
    lhs = ta.frobenius(op(X), Y)
    rhs = ta.frobenius(X, op.transpose_apply(Y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    A = op.dense()
    assert rel(ta.vec(op.transpose_apply(Y)), A.T @ ta.vec(Y)) < 1e-13
    # the operator is not symmetric, so the adjoint matters
    assert rel(A, A.T) > 1e-2


@pytest.mark.parametrize("seed", [0, 4])
def test_bases_span_the_normal_equation_krylov_spaces(seed):
    p, op, sk = tiny_problem(seed=seed)
    A = op.dense()
    rng = np.random.default_rng(seed + 100)
    R0 = rng.standard_normal(p.dims)
    m = 5
    bd = sketched_golub_kahan(op, op.transpose_apply, sk, R0, m)
    assert bd.m_eff == m and bd.flags == 0
    r0 = ta.vec(R0)
    QV = krylov(A.T @ A, A.T @ r0, m)
    QU = krylov(A @ A.T, r0, m + 1)
    for k in range(m):
        assert out_of_span(QV, ta.vec(bd.V[k])) < 1e-9
    for k in range(m + 1):
        assert out_of_span(QU, ta.vec(bd.U[k])) < 1e-9
    # and V_m does not fit in the smaller space (the spaces grow by one each step)
    assert out_of_span(QV[:, :m - 1], ta.vec(bd.V[m - 1])) > 1e-6


def test_bidiagonal_relations_and_unit_sketched_norms():
    p, op, sk = tiny_problem(seed=2)
    rng = np.random.default_rng(9)
    R0 = rng.standard_normal(p.dims)
    m = 4
    bd = sketched_golub_kahan(op, op.transpose_apply, sk, R0, m, full_last=True)
    B = bd.B
    assert B.shape == (m + 1, m)
    assert np.all(np.triu(B, 1) == 0) and np.all(np.tril(B, -2) == 0)
    assert rel(bd.U[0] * bd.beta, R0) < 1e-14
    for k in range(m):
        # Phi(V_k) = alpha_k U_k + beta_{k+1} U_{k+1}
        lhs = op(bd.V[k])
        assert rel(lhs, B[k, k] * bd.U[k] + B[k + 1, k] * bd.U[k + 1]) < 1e-12
        # Phi^T(U_{k+1}) = beta_{k+1} V_k + alpha_{k+1} V_{k+1}
        alpha_next = B[k + 1, k + 1] if k + 1 < m else sk.norm(op.transpose_apply(bd.U[k + 1])
                                                               - B[k + 1, k] * bd.V[k])
        assert rel(op.transpose_apply(bd.U[k + 1]), B[k + 1, k] * bd.V[k] + alpha_next * bd.V[k + 1]) < 1e-12
    # Phi^T(U_1) = alpha_1 V_1
    assert rel(op.transpose_apply(bd.U[0]), B[0, 0] * bd.V[0]) < 1e-13
    for X in bd.U + bd.V:
        assert abs(sk.norm(X) - 1.0) < 1e-13
    # a sketch that is not an isometry: the Frobenius norms differ from one
    assert max(abs(ta.fro_norm(X) - 1.0) for X in bd.U) > 1e-2


def test_identity_sketch_is_lsqr():
    p, op, _ = tiny_problem(seed=3)
    A = op.dense()
    c = ta.vec(p.x_true) + 0.3
    x0 = 0.1 * ta.vec(p.noise_dir)
    m = 6
    C = c.reshape(p.dims, order="F")
    X0 = x0.reshape(p.dims, order="F")
    res = rgk_solve(op, identity_sketch(), C, m, X0=X0, mu=0.0)
    r0 = c - A @ x0
    Q = krylov(A.T @ A, A.T @ r0, m)
    z, *_ = np.linalg.lstsq(A @ Q, r0, rcond=None)
    assert rel(ta.vec(res.X), x0 + Q @ z) < 1e-9
    np.testing.assert_allclose(res.beta, np.linalg.norm(r0), rtol=1e-13)
    # orthonormal bases in the Frobenius product
    Vm = np.stack([ta.vec(v) for v in res.bidiag.V[:m]], 1)
    Um = np.stack([ta.vec(u) for u in res.bidiag.U[:m + 1]], 1)
    assert np.abs(Vm.T @ Vm - np.eye(m)).max() < 1e-10
    assert np.abs(Um.T @ Um - np.eye(m + 1)).max() < 1e-10
    # the projected residual is the true residual
    np.testing.assert_allclose(np.linalg.norm(c - A @ ta.vec(res.X)), res.res_proj, rtol=1e-9)


def test_identity_sketch_lanczos_tridiagonal():
    """Omega = I: B^T B is the Lanczos tridiagonal matrix of A^T A started
    from A^T r0, i.e. Q^T A^T A Q with Q from the QR factorisation (positive
    diagonal of R) of the Krylov matrix [A^T r0, (A^T A) A^T r0, ...]."""
    p, op, _ = tiny_problem(seed=8)
    A = op.dense()
    R0 = np.random.default_rng(21).standard_normal(p.dims)
    r0 = ta.vec(R0)
    m = 5
    bd = sketched_golub_kahan(op, op.transpose_apply, identity_sketch(), R0, m)
    assert bd.m_eff == m
    K = np.empty((r0.size, m))
    v = A.T @ r0
    for j in range(m):
        K[:, j] = v / np.linalg.norm(v)
        v = A.T @ (A @ K[:, j])
    Q, Rq = np.linalg.qr(K)
    Q = Q * np.sign(np.diag(Rq))
    T = Q.T @ A.T @ A @ Q
    BtB = bd.B.T @ bd.B
    assert np.abs(BtB - T).max() < 1e-9 * np.abs(T).max()
    # first entries in closed form
    np.testing.assert_allclose(bd.beta, np.linalg.norm(r0), rtol=1e-14)
    np.testing.assert_allclose(bd.B[0, 0], np.linalg.norm(A.T @ r0) / np.linalg.norm(r0), rtol=1e-13)


def test_orthogonal_sketch_equals_identity_and_scaling_invariance():
    p, op, _ = tiny_problem(seed=6)
    I1, I2, J = p.dims
    rng = np.random.default_rng(17)
    qs = [np.linalg.qr(rng.standard_normal((k, k)))[0] for k in (I1, I2, J)]
    C = p.x_true + 0.2
    res_i = rgk_solve(op, identity_sketch(), C, 4, mu=0.05)
    res_q = rgk_solve(op, Sketch(*qs), C, 4, mu=0.05)
    assert rel(res_q.X, res_i.X) < 1e-10
    np.testing.assert_allclose(res_q.bidiag.B, res_i.bidiag.B, rtol=1e-10, atol=1e-12)
    # Omega_k -> 2 Omega_k on every sketched mode: S scales by f = 2^modes,
    # beta_1 by f, B is unchanged, y scales by f for the same mu, and the
    # bases by 1 / f, so X is unchanged
    _, _, sk = tiny_problem(seed=6)
    f = 2.0 ** sum(o is not None for o in sk.om)
    assert f > 1.0
    sk2 = Sketch(*[2.0 * o if o is not None else None for o in sk.om])
    r1 = rgk_solve(op, sk, C, 4, mu=0.05)
    r2 = rgk_solve(op, sk2, C, 4, mu=0.05)
    np.testing.assert_allclose(r2.beta, f * r1.beta, rtol=1e-13)
    np.testing.assert_allclose(r2.y, f * r1.y, rtol=1e-10)
    np.testing.assert_allclose(r2.bidiag.B, r1.bidiag.B, rtol=1e-12)
    assert rel(r2.X, r1.X) < 1e-12


def test_breakdown_for_a_multiple_of_the_identity():
    """Phi = c I: Phi^T R0 is parallel to R0, so beta_2 = 0 after one column
    and X_1 is the exact solution R0 / c (mu = 0)."""
    p = synth.small_problem(2, 8, 3, 2, 0, 0, 0, 8, 3, 2, m=3, random_bands=False)
    op = Operator(np.full((8, 1), 2.0), np.ones((3, 1)), np.ones((2, 1)))
    C = np.random.default_rng(0).standard_normal(p.dims)
    res = rgk_solve(op, identity_sketch(), C, 3, mu=0.0)
    assert res.m_eff == 1 and (res.flags & FLAG_BREAKDOWN)
    assert rel(res.X, C / 2.0) < 1e-13
