"""Sketched Einstein Block Golub-Kahan bidiagonalisation and the regularised
solve it feeds, float64 (Sec. 4.5, algorithm "Block Golub-Kahan via Sketched
Einstein Product"; the Tikhonov-regularised solutions of Sec. 5-6).

TEST INFRASTRUCTURE ONLY (see the package docstring).

For min ||C - Phi(X)||_F with R_0 = C - Phi(X_0):
    beta_1 = ||R_0||_Theta,            U_1 = R_0 / beta_1,
    W = Phi^T(U_1),                    alpha_1 = ||W||_Theta,   V_1 = W / alpha_1,
    for k = 1, 2, ...:
        W = Phi(V_k) - alpha_k U_k,        beta_{k+1} = ||W||_Theta,   U_{k+1} = W / beta_{k+1},
        Z = Phi^T(U_{k+1}) - beta_{k+1} V_k, alpha_{k+1} = ||Z||_Theta, V_{k+1} = Z / alpha_{k+1},
so that Phi(V_m) = U_{m+1} B_m with the (m+1) x m lower bidiagonal B_m
(alpha_k on the diagonal, beta_{k+1} below it) and
Phi^T(U_{k+1}) = beta_{k+1} V_k + alpha_{k+1} V_{k+1}.  The correction is
X_m = X_0 + sum_k y_k V_k with y from min ||beta_1 e1 - B_m y||^2 + mu ||y||^2
(mu fixed, by the discrepancy principle, or by GCV: the projected problem of
eqs. (12)-(13) with B_m in place of the Hessenberg matrix).

Readings:
* Phi^T is the adjoint of Phi for the Frobenius product,
  Phi^T(U) = U x_1 A1^T x_2 A2^T x_3 B (the transpose of the operator of
  eq. (2)); the sketch enters only through the norms, as printed.
* The tests "beta_{k+1} = 0" and "alpha_{k+1} = 0" become
  beta_{k+1} <= bd_tol ||S(Phi(V_k))|| and
  alpha_{k+1} <= bd_tol ||S(Phi^T(U_{k+1}))||.  A stop at beta_{k+1} keeps k
  columns (the last row of B_k is then about zero); a stop at alpha_{k+1}
  keeps k columns as well.
* The backward half of the last pass (V_{m+1}) does not enter B_m or X_m;
  it is formed only when ``full_last`` is set, as the listing does.
* With X_0 != 0 the penalty acts on the correction, as for RTG-GMRES.
* An optional stop after column k when the least-squares residual of the
  projected problem, |gamma_{k+1}| from the plane rotations, is at most
  ``stop_res`` (the residual test used for RTG-GMRES).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from .projected import givens_residuals, projected_tikhonov
from .tensor_algebra import frobenius

FLAG_BREAKDOWN = 1


@dataclasses.dataclass
class BidiagResult:
    U: List[np.ndarray]          # U_1 .. U_{m_eff+1}
    V: List[np.ndarray]          # V_1 .. V_{m_eff} (and V_{m_eff+1} with full_last)
    B: np.ndarray                # (m_eff + 1) x m_eff lower bidiagonal
    beta: float                  # beta_1 = ||R0||_Theta
    m_eff: int
    flags: int
    ls_res: np.ndarray           # least-squares residual of the projected problem after each column


def sketched_golub_kahan(phi: Callable, phi_t: Callable, sketch: Callable, R0: np.ndarray, m: int,
                         bd_tol: float = 1e-12, stop_res: Optional[float] = None,
                         full_last: bool = False) -> BidiagResult:
    def tnorm(X):
        s = sketch(X)
        return math.sqrt(frobenius(s, s))

    R0 = np.asarray(R0, dtype=np.float64)
    beta1 = tnorm(R0)
    if beta1 == 0.0:
        return BidiagResult([], [], np.zeros((1, 0)), 0.0, 0, FLAG_BREAKDOWN, np.zeros(0))
    U = [R0 / beta1]
    Wt = phi_t(U[0])
    alpha = tnorm(Wt)
    if alpha == 0.0:                         # Phi^T(R0) = 0: no Krylov space
        return BidiagResult(U, [], np.zeros((1, 0)), beta1, 0, FLAG_BREAKDOWN, np.zeros(0))
    V = [Wt / alpha]
    B = np.zeros((m + 1, m))
    flags = 0
    m_eff = m
    ls_res = []
    for k in range(m):                       # column k + 1 of B
        B[k, k] = alpha
        PV = phi(V[k])
        beta = tnorm(PV - alpha * U[k])
        B[k + 1, k] = beta
        ls_res.append(givens_residuals(B[:k + 2, :k + 1], beta1)[-1])
        if beta <= bd_tol * tnorm(PV):
            flags |= FLAG_BREAKDOWN
            m_eff = k + 1
            break
        U.append((PV - alpha * U[k]) / beta)
        if stop_res is not None and ls_res[-1] <= stop_res:
            m_eff = k + 1
            break
        if k + 1 == m and not full_last:
            break
        PU = phi_t(U[k + 1])
        Z = PU - beta * V[k]
        alpha = tnorm(Z)
        if alpha <= bd_tol * tnorm(PU):
            flags |= FLAG_BREAKDOWN
            m_eff = k + 1
            break
        V.append(Z / alpha)
    B = B[:m_eff + 1, :m_eff]
    return BidiagResult(U, V, B, beta1, m_eff, flags, np.array(ls_res))


@dataclasses.dataclass
class GKSolveResult:
    X: np.ndarray
    y: np.ndarray
    mu: float
    flags: int
    m_eff: int
    beta: float
    res_proj: float
    res_ls: float
    bidiag: BidiagResult


def rgk_solve(op, sketch, C, m, X0=None, mu: Optional[float] = None,
              delta: Optional[float] = None, eta: float = 1.01, bd_tol: float = 1e-12,
              stop_res: Optional[float] = None, mu_rule: str = "discrepancy") -> GKSolveResult:
    """Sketched Block Golub-Kahan solve: ``op`` provides ``op(X)`` = Phi(X)
    and ``op.transpose_apply(X)`` = Phi^T(X)."""
    C = np.asarray(C, dtype=np.float64)
    X0 = np.zeros_like(C) if X0 is None else np.asarray(X0, dtype=np.float64)
    R0 = C - op(X0)
    bd = sketched_golub_kahan(op, op.transpose_apply, sketch, R0, m, bd_tol=bd_tol, stop_res=stop_res)
    if bd.m_eff == 0:
        return GKSolveResult(X0.copy(), np.zeros(0), 0.0, bd.flags, 0, bd.beta, 0.0, 0.0, bd)
    if mu is None and delta is None and mu_rule != "gcv":
        mu = 0.0
    pt = projected_tikhonov(bd.B, bd.beta, mu=mu, delta=delta, eta=eta, rule=mu_rule)
    X = X0.copy()
    for k in range(bd.m_eff):
        X = X + pt["y"][k] * bd.V[k]
    return GKSolveResult(X, pt["y"], pt["mu"], bd.flags | pt["flags"], bd.m_eff, bd.beta,
                         pt["res_proj"], pt["res_ls"], bd)
