"""Sketched tensor global Arnoldi process, float64 (Sec. 4.3).

V_1 = R_0 / ||R_0||_Theta.  For j = 1..m:  W = Phi(V_j);
h_ij = <V_i, W>_Theta and W <- W - h_ij V_i for i = 1..j;
h_{j+1,j} = ||W||_Theta;  V_{j+1} = W / h_{j+1,j}.

Readings taken where the text is loose:
* W is the full-space tensor Phi(V_j); the sketch enters only through the
  inner products and norms (Sec. 4.3 and Sec. 5.4 state that all norms and
  orthogonality tests use <.,.>_Theta).
* The inner products are evaluated in sketch space: s = S(W) is kept next to
  W and updated with the same coefficients (s <- s - h_ij S(V_i)), which is
  exact by linearity of S.  One reorthogonalisation pass of the same form is
  applied and its coefficients are added to h_ij (``reorth=False`` gives the
  single-pass modified Gram-Schmidt of the algorithm as printed).
* S(V_{j+1}) is obtained by sketching the stored V_{j+1}.
* The breakdown test h_{j+1,j} = 0 becomes h_{j+1,j} <= bd_tol ||S(Phi(V_j))||.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional

import numpy as np

from .tensor_algebra import frobenius
from .projected import givens_residuals

FLAG_BREAKDOWN = 1


@dataclasses.dataclass
class ArnoldiResult:
    V: List[np.ndarray]          # V_1..V_{m_eff+1} (the last only if no stop)
    SV: List[np.ndarray]         # sketches of the stored V_i
    H: np.ndarray                # (m_eff + 1) x m_eff
    beta: float
    m_eff: int
    flags: int
    ls_res: np.ndarray           # Givens LS residual after each step


def orthogonalise(SV: List[np.ndarray], V: List[np.ndarray], s: np.ndarray, W: np.ndarray,
                  reorth: bool = True):
    """Column j of H from s = S(W), W = Phi(V_j), against the basis V_1..V_j
    with sketches SV_i = S(V_i): modified Gram-Schmidt in sketch space, in
    the algorithm's order (h_ij = <V_i, W>_Theta, then W <- W - h_ij V_i,
    i = 1..j), with the same updates applied to the full-space W, and (with
    reorth) one more pass of the same form whose coefficients are added.
    Returns (h_1j..h_jj, the orthogonalised s, the orthogonalised W)."""
    j = len(V)
    h = np.zeros(j)
    for _ in range(2 if reorth else 1):
        for i in range(j):
            hi = frobenius(SV[i], s)
            h[i] += hi
            s = s - hi * SV[i]
            W = W - hi * V[i]
    return h, s, W


def sketched_global_arnoldi(phi: Callable, sketch: Callable, R0: np.ndarray,
                            m: int, reorth: bool = True, bd_tol: float = 1e-12,
                            stop_res: Optional[float] = None) -> ArnoldiResult:
    R0 = np.asarray(R0, dtype=np.float64)
    s0 = sketch(R0)
    beta = math.sqrt(frobenius(s0, s0))
    if beta == 0.0:
        return ArnoldiResult([], [], np.zeros((1, 0)), 0.0, 0, FLAG_BREAKDOWN, np.zeros(0))
    V = [R0 / beta]
    SV = [sketch(V[0])]
    H = np.zeros((m + 1, m))
    flags = 0
    m_eff = m
    ls_res = []
    for j in range(m):
        W = phi(V[j])
        s = sketch(W)
        rho = math.sqrt(frobenius(s, s))
        h, s, W = orthogonalise(SV[:j + 1], V[:j + 1], s, W, reorth)
        H[:j + 1, j] = h
        hn = math.sqrt(frobenius(s, s))
        H[j + 1, j] = hn
        ls_res.append(givens_residuals(H[:j + 2, :j + 1], beta)[-1])
        if hn <= bd_tol * rho:
            flags |= FLAG_BREAKDOWN
            m_eff = j + 1
            break
        if stop_res is not None and ls_res[-1] <= stop_res:
            m_eff = j + 1
            break
        V.append(W / hn)
        SV.append(sketch(V[-1]))
    H = H[:m_eff + 1, :m_eff]
    return ArnoldiResult(V, SV, H, beta, m_eff, flags, np.array(ls_res))
