"""The pins are strong enough: each plausible mistake planted in the oracle
(a transposed factor, a dropped sketch mode, a wrong index, a Frobenius norm
where the sketched norm belongs, a wrong filter factor, an unsquared target)
makes at least one pin fail.  Mistakes are planted on the CPU only, by
monkeypatching oracle functions for the duration of one test."""
import math

import numpy as np
import pytest

import test_oracle_pins as pins
import oracle.operator as opm
import oracle.sketch as skm
import oracle.projected as pm
import oracle.arnoldi as am
import oracle.gmres as gm
from oracle.tensor_algebra import mode_product, frobenius


def expect_failure(fn, *args):
    with pytest.raises(Exception):
        fn(*args)


def test_pins_pass_unmutated():
    pins.test_phi_matches_literal_einstein_form_and_kronecker()
    pins.test_sketch_vectorised_form()
    pins.test_arnoldi_relation_and_theta_orthonormality("tiny")


def test_untransposed_b_is_caught(monkeypatch):
    def bad_phi(X, A1, A2, B):
        return mode_product(mode_product(mode_product(X, A1, 0), A2, 1), B, 2)
    monkeypatch.setattr(opm, "phi", bad_phi)
    expect_failure(pins.test_phi_matches_literal_einstein_form_and_kronecker)


def test_transposed_blur_factor_is_caught(monkeypatch):
    good = opm.phi

    def bad_phi(X, A1, A2, B):
        return good(X, np.asarray(A1).T, A2, B)
    monkeypatch.setattr(opm, "phi", bad_phi)
    monkeypatch.setattr(pins, "phi", bad_phi)
    expect_failure(pins.test_phi_is_psf_convolution_with_zero_boundary)
    expect_failure(pins.test_phi_matches_literal_einstein_form_and_kronecker)


def test_dropped_sketch_mode_is_caught(monkeypatch):
    def bad_call(self, X):
        Y = np.asarray(X, np.float64)
        for k, om in enumerate(self.om[:2]):
            if om is not None:
                Y = mode_product(Y, om, k)
        return Y
    monkeypatch.setattr(skm.Sketch, "__call__", bad_call)
    expect_failure(pins.test_sketch_vectorised_form)


def _mutated_arnoldi(kind):
    def arnoldi(phi, sketch, R0, m, reorth=True, bd_tol=1e-12, stop_res=None):
        R0 = np.asarray(R0, dtype=np.float64)
        s0 = sketch(R0)
        beta = math.sqrt(frobenius(s0, s0))
        V = [R0 / beta]
        SV = [sketch(V[0])]
        H = np.zeros((m + 1, m))
        for j in range(m):
            W = phi(V[j])
            s = sketch(W)
            for _ in range(2):
                for i in range(j + 1):
                    h = frobenius(SV[i], s)
                    H[i, j] += h
                    s = s - h * SV[i]
                    W = W - h * (V[j] if kind == "index" else V[i])
            hn = math.sqrt(frobenius(W, W)) if kind == "frobenius" else math.sqrt(frobenius(s, s))
            H[j + 1, j] = hn
            V.append(W / hn)
            SV.append(sketch(V[-1]))
        return am.ArnoldiResult(V, SV, H, beta, m, 0, np.zeros(m))
    return arnoldi


@pytest.mark.parametrize("kind", ["index", "frobenius"])
def test_arnoldi_mistakes_are_caught(monkeypatch, kind):
    monkeypatch.setattr(pins, "sketched_global_arnoldi", _mutated_arnoldi(kind))
    expect_failure(pins.test_arnoldi_relation_and_theta_orthonormality, "tiny")


def test_wrong_filter_factor_is_caught(monkeypatch):
    monkeypatch.setattr(pm.SVDProblem, "y",
                        lambda self, mu: self.W @ (self.s ** 2 / (self.s ** 2 + mu) * self.ghat))
    expect_failure(pins.test_eq13_eq14_and_svd_filter_agree)


def test_unsquared_discrepancy_target_is_caught(monkeypatch):
    good = pm.discrepancy_mu
    monkeypatch.setattr(pm, "discrepancy_mu", lambda P, target, iters=200: good(P, math.sqrt(target), iters))
    expect_failure(pins.test_discrepancy_root_and_monotonicity)


def test_reversed_assembly_is_caught(monkeypatch):
    good = gm.projected_tikhonov

    def bad(H, beta, **kw):
        out = good(H, beta, **kw)
        out["y"] = out["y"][::-1].copy()
        return out
    monkeypatch.setattr(gm, "projected_tikhonov", bad)
    expect_failure(pins.test_matches_dense_direct_solve_on_krylov_space, 5)


def test_gcv_trace_over_k_rows_is_caught(monkeypatch):
    """The trace taken over k instead of k + 1 rows (dropping the identity's
    extra row) is caught by both GCV pins."""
    def bad_gcv(P, mu):
        den = P.k - float(np.sum(P.s ** 2 / (P.s ** 2 + mu)))
        return P.residual2(mu) / (den * den)
    monkeypatch.setattr(pm, "gcv", bad_gcv)
    monkeypatch.setattr(pins, "gcv", bad_gcv)
    expect_failure(pins.test_gcv_matches_its_definition_with_explicit_matrices)
    expect_failure(pins.test_gcv_minimiser_closed_form_for_equal_singular_values)


def test_gcv_unsquared_denominator_is_caught(monkeypatch):
    def bad_gcv(P, mu):
        den = (P.k + 1) - float(np.sum(P.s ** 2 / (P.s ** 2 + mu)))
        return P.residual2(mu) / den
    monkeypatch.setattr(pm, "gcv", bad_gcv)
    monkeypatch.setattr(pins, "gcv", bad_gcv)
    expect_failure(pins.test_gcv_matches_its_definition_with_explicit_matrices)
    expect_failure(pins.test_gcv_minimiser_closed_form_for_equal_singular_values)


# --------------------------------------------------------------------------
# sketched Block Golub-Kahan (Sec. 4.5)
# --------------------------------------------------------------------------
import oracle.golub_kahan as gkm
import test_oracle_gk as gkpins


def _mutated_golub_kahan(kind):
    def gk(phi, phi_t, sketch, R0, m, bd_tol=1e-12, stop_res=None, full_last=False):
        def tnorm(X):
            s = X if kind == "frobenius" else sketch(X)
            return math.sqrt(frobenius(s, s))
        adj = phi if kind == "forward" else phi_t
        R0 = np.asarray(R0, dtype=np.float64)
        beta1 = tnorm(R0)
        U = [R0 / beta1]
        Wt = adj(U[0])
        alpha = tnorm(Wt)
        V = [Wt / alpha]
        B = np.zeros((m + 1, m))
        for k in range(m):
            B[k, k] = alpha
            uk = U[max(k - 1, 0)] if kind == "index" else U[k]
            W = phi(V[k]) - (0.0 if kind == "drop_alpha" else alpha) * uk
            beta = tnorm(W)
            B[k + 1, k] = beta
            U.append(W / beta)
            if k + 1 == m and not full_last:
                break
            Z = adj(U[k + 1]) - (0.0 if kind == "drop_beta" else beta) * V[k]
            alpha = tnorm(Z)
            V.append(Z / alpha)
        return gkm.BidiagResult(U, V, B, beta1, m, 0, np.zeros(m))
    return gk


@pytest.mark.parametrize("kind", ["drop_alpha", "drop_beta", "index", "frobenius", "forward"])
def test_golub_kahan_mistakes_are_caught(monkeypatch, kind):
    """Each planted mistake in the bidiagonalisation fails at least one pin."""
    bad = _mutated_golub_kahan(kind)
    monkeypatch.setattr(gkm, "sketched_golub_kahan", bad)
    monkeypatch.setattr(gkpins, "sketched_golub_kahan", bad)
    failed = 0
    for fn, args in [(gkpins.test_bases_span_the_normal_equation_krylov_spaces, (0,)),
                     (gkpins.test_bidiagonal_relations_and_unit_sketched_norms, ()),
                     (gkpins.test_identity_sketch_is_lsqr, ()),
                     (gkpins.test_identity_sketch_lanczos_tridiagonal, ())]:
        try:
            fn(*args)
        except Exception:
            failed += 1
    assert failed >= 1


def test_golub_kahan_pins_pass_unmutated():
    gkpins.test_bases_span_the_normal_equation_krylov_spaces(0)
    gkpins.test_bidiagonal_relations_and_unit_sketched_norms()
    gkpins.test_identity_sketch_is_lsqr()
    gkpins.test_identity_sketch_lanczos_tridiagonal()


def test_untransposed_channel_mix_in_the_adjoint_is_caught(monkeypatch):
    def bad_t(self, X):
        return mode_product(mode_product(mode_product(np.asarray(X, np.float64), self.A1.T, 0), self.A2.T, 1),
                            self.B.T, 2)
    monkeypatch.setattr(opm.Operator, "transpose_apply", bad_t)
    expect_failure(gkpins.test_transpose_apply_is_the_frobenius_adjoint)
    expect_failure(gkpins.test_bases_span_the_normal_equation_krylov_spaces, 0)


# --------------------------------------------------------------------------
# general PSF operator (eqs. (56)-(57))
# --------------------------------------------------------------------------
import test_oracle_psf as psfpins


def test_unflipped_psf_is_caught(monkeypatch):
    good = opm.convolve_psf_zero_bc

    def bad(X, P):
        return good(X, np.asarray(P)[::-1, ::-1])
    monkeypatch.setattr(opm, "convolve_psf_zero_bc", bad)
    monkeypatch.setattr(psfpins, "convolve_psf_zero_bc", bad)
    expect_failure(psfpins.test_shift_sum_equals_elementwise_definition)
    expect_failure(psfpins.test_psf_operator_matches_fourth_order_einstein_form)


def test_transposed_psf_is_caught(monkeypatch):
    good_call = opm.PSFOperator.__call__

    def bad_call(self, X):
        return mode_product(opm.convolve_psf_zero_bc(X, self.P.T), self.B.T, 2)
    monkeypatch.setattr(opm.PSFOperator, "__call__", bad_call)
    expect_failure(psfpins.test_psf_operator_matches_fourth_order_einstein_form)
    monkeypatch.setattr(opm.PSFOperator, "__call__", good_call)


def test_unrotated_psf_adjoint_is_caught(monkeypatch):
    def bad_t(self, Y):
        return opm.convolve_psf_zero_bc(mode_product(np.asarray(Y, np.float64), self.B, 2), self.P)
    monkeypatch.setattr(opm.PSFOperator, "transpose_apply", bad_t)
    expect_failure(psfpins.test_psf_adjoint)


def test_restart_from_the_old_start_is_caught(monkeypatch):
    """Restarting every cycle from the first X0 instead of X_m never
    converges: the dense-solution pin fails."""
    good = gm.rtg_gmres

    def stuck(phi, sketch, C, m, X0=None, **kw):
        return good(phi, sketch, C, m, X0=None, **kw)
    monkeypatch.setattr(gm, "rtg_gmres", stuck)
    expect_failure(pins.test_restarted_gmres_converges_to_the_dense_solution)
