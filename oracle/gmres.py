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


@dataclasses.dataclass
class RestartResult:
    X: np.ndarray
    iters: int               # Arnoldi steps over all cycles
    cycles: int              # cycles that took at least one step
    flags: int
    last: SolveResult


FLAG_NOT_CONVERGED = 16


def rtg_gmres_restarted(phi, sketch, C, m, restarts, stop_res, X0=None, mu: Optional[float] = None,
                        delta: Optional[float] = None, eta: float = 1.01, bd_tol: float = 1e-12,
                        mu_rule: str = "discrepancy") -> RestartResult:
    """Restarted RTG-GMRES(m): the algorithm of Sec. 4.4 ends a solve by
    testing the sketched norm of the true residual, ||C - Phi(X_m)||_Theta <
    eps; while that test fails, another solve starts from X_0 = X_m, at most
    ``restarts`` times.  Each solve stops early when its projected
    least-squares residual reaches eps (``stop_res``); NOT_CONVERGED is set
    when the last solve ran all m steps without reaching it."""
    C = np.asarray(C, dtype=np.float64)
    X = np.zeros_like(C) if X0 is None else np.asarray(X0, dtype=np.float64)
    iters, cycles, flags, last = 0, 0, 0, None
    for cycle in range(restarts + 1):
        if cycle > 0 and sketch.norm(C - phi(X)) < stop_res:
            break
        last = rtg_gmres(phi, sketch, C, m, X0=X, mu=mu, delta=delta, eta=eta, bd_tol=bd_tol,
                         stop_res=stop_res, mu_rule=mu_rule)
        X = last.X
        iters += last.m_eff
        cycles += 1
        reached = (last.m_eff < m or bool(last.flags & 1)
                   or (last.arnoldi.ls_res.size > 0 and last.arnoldi.ls_res[-1] <= stop_res))
        flags = (last.flags & ~FLAG_NOT_CONVERGED) | (0 if reached else FLAG_NOT_CONVERGED)
    return RestartResult(X, iters, cycles, flags, last)
