"""The small projected problems of RTG-GMRES, in float64.

Given the (k+1) x k upper Hessenberg matrix H (the tilde-H_m of the Arnoldi
relation) and beta = ||R0||_Theta:

* least squares (11S): y = argmin ||beta e1 - H y||_2, and its residual
  computed by Givens rotations (the residual of the first j columns for every
  j, used as a stopping test);
* projected Tikhonov (12S)/(12): min ||beta e1 - H y||^2 + mu ||y||^2, solved
  through the thin SVD H = U diag(s) W^T (the filter-factor form of the
  stacked least-squares problem (13)); (13) itself and the normal equations
  (14) are provided as cross-checks;
* the discrepancy principle for mu: the projected residual
  phi(mu) = ||beta e1 - H y_mu||^2 increases monotonically from phi(0) (the
  least-squares residual) to beta^2, and mu is the root of
  phi(mu) = (eta delta)^2, found by bisection in log(mu).
"""
from __future__ import annotations

import math

import numpy as np

FLAG_DISCREP_UNREACHABLE = 2
FLAG_MU_INF = 4


def rhs(beta: float, k: int) -> np.ndarray:
    g = np.zeros(k + 1)
    g[0] = beta
    return g


def givens_residuals(H: np.ndarray, beta: float) -> np.ndarray:
    """|gamma_{j+1}| = min_y ||beta e1 - H[:j+1, :j] y|| for j = 1..k, by
    applying one plane rotation per column to the Hessenberg matrix."""
    H = np.array(H, dtype=np.float64)
    k = H.shape[1]
    g = rhs(beta, k)
    cs = np.zeros(k)
    sn = np.zeros(k)
    res = np.zeros(k)
    for j in range(k):
        for i in range(j):                      # previous rotations on column j
            a, b = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * b
            H[i + 1, j] = -sn[i] * a + cs[i] * b
        a, b = H[j, j], H[j + 1, j]
        rho = math.hypot(a, b)
        if rho == 0.0:
            cs[j], sn[j] = 1.0, 0.0
        else:
            cs[j], sn[j] = a / rho, b / rho
        H[j, j] = rho
        H[j + 1, j] = 0.0
        g[j], g[j + 1] = cs[j] * g[j], -sn[j] * g[j]
        res[j] = abs(g[j + 1])
    return res


def ls_solve(H, beta):
    """y = argmin ||beta e1 - H y|| (11S), with numpy's least squares."""
    k = H.shape[1]
    y, *_ = np.linalg.lstsq(H, rhs(beta, k), rcond=None)
    return y


def solve_13(H, beta, mu):
    """Eq. (13): least squares on the stacked matrix [H; sqrt(mu) I]."""
    k = H.shape[1]
    M = np.vstack([H, math.sqrt(mu) * np.eye(k)])
    b = np.concatenate([rhs(beta, k), np.zeros(k)])
    y, *_ = np.linalg.lstsq(M, b, rcond=None)
    return y


def solve_14(H, beta, mu):
    """Eq. (14): (H^T H + mu I) y = H^T beta e1."""
    k = H.shape[1]
    return np.linalg.solve(H.T @ H + mu * np.eye(k), H.T @ rhs(beta, k))


class SVDProblem:
    """H = U diag(s) W^T; g_hat = U^T (beta e1); g_perp = beta e1 - U g_hat."""

    def __init__(self, H, beta):
        H = np.asarray(H, dtype=np.float64)
        self.k = H.shape[1]
        self.beta = float(beta)
        U, s, Wt = np.linalg.svd(H, full_matrices=False)
        self.U, self.s, self.W = U, s, Wt.T
        g = rhs(beta, self.k)
        self.ghat = U.T @ g
        gperp = g - U @ self.ghat
        self.gperp2 = float(gperp @ gperp)

    def residual2(self, mu: float) -> float:
        """phi(mu) = sum_i (mu / (s_i^2 + mu))^2 ghat_i^2 + ||g_perp||^2."""
        if mu == 0.0:
            return self.gperp2
        f = mu / (self.s ** 2 + mu)
        return float(np.sum((f * self.ghat) ** 2) + self.gperp2)

    def y(self, mu: float) -> np.ndarray:
        """Tikhonov solution W diag(s / (s^2 + mu)) g_hat (filter form of (13))."""
        return self.W @ (self.s / (self.s ** 2 + mu) * self.ghat)


def discrepancy_mu(P: SVDProblem, target: float, iters: int = 200):
    """Root of phi(mu) = target^2 by bisection in log(mu).

    Returns (mu, flags).  mu = 0 with FLAG_DISCREP_UNREACHABLE when even the
    least-squares residual exceeds the target; mu = inf with FLAG_MU_INF when
    the target is at least beta (then y = 0)."""
    t2 = target * target
    if t2 <= P.gperp2:
        return 0.0, FLAG_DISCREP_UNREACHABLE
    if t2 >= P.beta * P.beta:
        return math.inf, FLAG_MU_INF
    smax2 = float(P.s[0] ** 2) if P.s.size and P.s[0] > 0 else 1.0
    lo, hi = math.log(smax2) - 80.0, math.log(smax2) + 80.0
    while P.residual2(math.exp(lo)) > t2:
        lo -= 40.0
    while P.residual2(math.exp(hi)) < t2:
        hi += 40.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if P.residual2(math.exp(mid)) < t2:
            lo = mid
        else:
            hi = mid
    return math.exp(0.5 * (lo + hi)), 0


def gcv(P: SVDProblem, mu: float) -> float:
    """Generalized cross-validation function of the projected problem (Sec. 3,
    parameter selection via GCV):
        GCV(mu) = ||H y_mu - beta e1||^2 / tr(I - H (H^T H + mu I)^{-1} H^T)^2,
    I the (k+1) x (k+1) identity.  With H = U diag(s) W^T the influence matrix
    is U diag(s^2 / (s^2 + mu)) U^T, so the trace is (k + 1) - sum_i
    s_i^2 / (s_i^2 + mu), and the numerator is phi(mu)."""
    den = (P.k + 1) - float(np.sum(P.s ** 2 / (P.s ** 2 + mu)))
    return P.residual2(mu) / (den * den)


GCV_GRID = 512


def gcv_mu(P: SVDProblem) -> float:
    """Minimiser of GCV over log(mu): the best of GCV_GRID points spread evenly
    over [log(s_min^2) - 10, log(s_max^2) + 10] (s_min the smallest positive
    singular value, floored at 1e-30 s_max), then golden-section search
    between the neighbours of that point, to a bracket of 1e-12."""
    s = P.s[P.s > 0]
    smax2 = float(s[0] ** 2) if s.size else 1.0
    smin2 = max(float(s[-1] ** 2), 1e-30 * smax2) if s.size else 1.0
    lo, hi = math.log(smin2) - 10.0, math.log(smax2) + 10.0
    xs = lo + (hi - lo) * np.arange(GCV_GRID) / (GCV_GRID - 1)
    vals = [gcv(P, math.exp(x)) for x in xs]
    i = int(np.argmin(vals))
    a, b = xs[max(i - 1, 0)], xs[min(i + 1, GCV_GRID - 1)]
    r = (math.sqrt(5.0) - 1.0) / 2.0
    c, d = b - r * (b - a), a + r * (b - a)
    fc, fd = gcv(P, math.exp(c)), gcv(P, math.exp(d))
    while b - a > 1e-12:
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - r * (b - a)
            fc = gcv(P, math.exp(c))
        else:
            a, c, fc = c, d, fd
            d = a + r * (b - a)
            fd = gcv(P, math.exp(d))
    return math.exp(0.5 * (a + b))


def projected_tikhonov(H, beta, mu=None, delta=None, eta=1.01, rule="discrepancy"):
    """Solve the projected problem; ``mu`` fixed (>= 0) or, when ``mu`` is
    None, chosen by the discrepancy principle with noise norm ``delta``
    (``rule="discrepancy"``) or by minimising GCV (``rule="gcv"``).

    Returns dict(y, mu, flags, res_proj, res_ls)."""
    H = np.asarray(H, dtype=np.float64)
    k = H.shape[1]
    P = SVDProblem(H, beta)
    flags = 0
    if mu is None and rule == "gcv":
        mu = gcv_mu(P)
    elif mu is None:
        mu, flags = discrepancy_mu(P, eta * delta)
    if math.isinf(mu):
        y = np.zeros(k)
    else:
        y = P.y(mu)
    r = rhs(beta, k) - H @ y
    return {"y": y, "mu": mu, "flags": flags,
            "res_proj": float(np.sqrt(r @ r)),
            "res_ls": float(np.sqrt(P.gperp2)), "svd": P}
