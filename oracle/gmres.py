"""RTG-GMRES driver, float64 (algorithm "Block GMRES via Sketched Einstein
Product", Sec. 4.4, with the projected Tikhonov problem of eqs. (12)-(13)).

R_0 = C - Phi(X_0); beta = ||R_0||_Theta; m steps of the sketched global
Arnoldi process; y from the projected Tikhonov problem
min ||beta e1 - H y||^2 + mu ||y||^2 (mu fixed, or by the discrepancy
principle); X_m = X_0 + sum_j y_j V_j.

With X_0 != 0 the penalty mu ||y||^2 acts on the correction: the basis is
Theta-orthonormal, so ||y|| = ||X_m - X_0||_Theta (eq. (12) sets X_0 = 0).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .arnoldi import sketched_global_arnoldi, ArnoldiResult
from .projected import projected_tikhonov
from .tensor_algebra import fro_norm


@dataclasses.dataclass
class SolveResult:
    X: np.ndarray
    y: np.ndarray
    mu: float
    flags: int
    m_eff: int
    beta: float
    res_proj: float          # ||beta e1 - H y||
    res_ls: float            # least-squares residual of the projected problem
    arnoldi: ArnoldiResult


def rtg_gmres(phi, sketch, C, m, X0=None, mu: Optional[float] = None,
              delta: Optional[float] = None, eta: float = 1.01,
              reorth: bool = True, bd_tol: float = 1e-12,
              stop_res: Optional[float] = None, mu_rule: str = "discrepancy") -> SolveResult:
    C = np.asarray(C, dtype=np.float64)
    X0 = np.zeros_like(C) if X0 is None else np.asarray(X0, dtype=np.float64)
    R0 = C - phi(X0)
    ar = sketched_global_arnoldi(phi, sketch, R0, m, reorth=reorth,
                                 bd_tol=bd_tol, stop_res=stop_res)
    if ar.m_eff == 0:
        return SolveResult(X0.copy(), np.zeros(0), 0.0, ar.flags, 0, ar.beta,
                           0.0, 0.0, ar)
    if mu is None and delta is None and mu_rule != "gcv":
        mu = 0.0
    pt = projected_tikhonov(ar.H, ar.beta, mu=mu, delta=delta, eta=eta, rule=mu_rule)
    X = X0.copy()
    for j in range(ar.m_eff):
        X = X + pt["y"][j] * ar.V[j]
    return SolveResult(X, pt["y"], pt["mu"], ar.flags | pt["flags"], ar.m_eff,
                       ar.beta, pt["res_proj"], pt["res_ls"], ar)


def true_residual(phi, C, X) -> float:
    return fro_norm(np.asarray(C, np.float64) - phi(X))
