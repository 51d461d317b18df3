"""Pins of the oracle's general-PSF operator (eqs. (56)-(57)): the
shift-sum convolution against the element-by-element definition, against
the fourth-order tensor built from the PSF entries through the Einstein
product, against the separable banded operator for an outer-product PSF; its
adjoint; and the unsketched solve against textbook GMRES on the operator's
matrix.  The synthetic PSF is checked to be genuinely non-separable."""
import numpy as np

from oracle import tensor_algebra as ta
from oracle.gmres import rtg_gmres
from oracle.operator import (Operator, PSFOperator, convolve_psf_zero_bc, psf_tensor, band_to_dense)
from oracle.sketch import identity_sketch
from paper_2603_00839_amd import synth

from test_oracle_pins import rel, krylov_basis


def nonsep_psf(r, seed):
    """A rotated Gaussian PSF with a random non-symmetric perturbation (so
    that flips and transposes change it)."""
    rng = np.random.default_rng(seed)
    return synth.rotated_gaussian_psf(r, 1.6, 0.7, 0.5) + 0.02 * rng.uniform(0.0, 1.0, (2 * r + 1, 2 * r + 1))


def random_b_band(J, seed):
    rng = np.random.default_rng(seed)
    b = rng.uniform(0.1, 1.0, (J, 3))
    b[0, 0] = 0.0
    b[-1, 2] = 0.0
    return b


def test_shift_sum_equals_elementwise_definition():
    rng = np.random.default_rng(1)
    P = nonsep_psf(2, 3)
    X = rng.standard_normal((7, 6, 2))
    r = 2
    ref = np.zeros_like(X)
    for i in range(7):
        for j in range(6):
            for a in range(-r, r + 1):
                for b in range(-r, r + 1):
                    if 0 <= i + a < 7 and 0 <= j + b < 6:
                        ref[i, j, :] += P[r - a, r - b] * X[i + a, j + b, :]
    np.testing.assert_allclose(convolve_psf_zero_bc(X, P), ref, rtol=1e-13, atol=1e-13)


def test_psf_operator_matches_fourth_order_einstein_form():
    dims = (6, 5, 3)
    rng = np.random.default_rng(2)
    P = nonsep_psf(2, 4)
    bb = random_b_band(3, 5)
    X = rng.standard_normal(dims)
    op = PSFOperator(P, bb, dims)
    A4 = psf_tensor(P, dims[0], dims[1])
    lit = ta.einstein_product(ta.einstein_product(A4, X, 2), band_to_dense(bb), 1)
    np.testing.assert_allclose(op(X), lit, rtol=1e-13, atol=1e-13)


def test_outer_product_psf_equals_separable_operator():
    rng = np.random.default_rng(6)
    t1 = rng.uniform(0.1, 1.0, 5)
    t2 = rng.uniform(0.1, 1.0, 5)
    dims = (9, 8, 3)
    bb = random_b_band(3, 7)
    sep = Operator(synth.toeplitz_band(9, t1), synth.toeplitz_band(8, t2), bb)
    psf = PSFOperator(np.outer(t1, t2), bb, dims)
    X = rng.standard_normal(dims)
    np.testing.assert_allclose(psf(X), sep(X), rtol=1e-13, atol=1e-13)


def test_psf_adjoint():
    dims = (7, 6, 3)
    rng = np.random.default_rng(8)
    op = PSFOperator(nonsep_psf(2, 9), random_b_band(3, 10), dims)
    X = rng.standard_normal(dims)
    Y = rng.standard_normal(dims)
    lhs = ta.frobenius(op(X), Y)
    assert abs(lhs - ta.frobenius(X, op.transpose_apply(Y))) <= 1e-12 * abs(lhs)
    A = op.dense()
    assert rel(ta.vec(op.transpose_apply(Y)), A.T @ ta.vec(Y)) < 1e-13
    assert rel(A, A.T) > 1e-2


def test_synthetic_psf_is_not_separable():
    P = synth.rotated_gaussian_psf(4, 2.0, 0.8, 0.6)
    s = np.linalg.svd(P, compute_uv=False)
    assert s[1] > 1e-2 * s[0]
    np.testing.assert_allclose(P.sum(), 1.0, rtol=1e-14)
    # a rotation by pi/2 swaps the roles of the two axes: the transpose
    np.testing.assert_allclose(synth.rotated_gaussian_psf(3, 2.0, 0.8, 0.0).T,
                               synth.rotated_gaussian_psf(3, 2.0, 0.8, np.pi / 2), atol=1e-15)


def test_psf_identity_sketch_solve_is_gmres():
    p = synth.psf_problem(3, 8, 7, 3, r=2, l1=8, l2=7, m=6)
    op = PSFOperator(p.psf, p.b_band, p.dims)
    A = op.dense()
    c = ta.vec(p.x_true) + 0.2
    m = 6
    res = rtg_gmres(op, identity_sketch(), c.reshape(p.dims, order="F"), m, mu=0.0)
    Q = krylov_basis(A, c, m)
    z, *_ = np.linalg.lstsq(A @ Q, c, rcond=None)
    assert rel(ta.vec(res.X), Q @ z) < 1e-10
