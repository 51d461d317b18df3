"""The bfloat16-basis Arnoldi step (operator applied tile by tile, multi-AXPY,
rounding, and the sketches of V_{j+1} and of Phi(V_{j+1}) taken in the same
pass) against float64 arithmetic on the basis the GPU stored.

With a bfloat16 basis the GPU result is not the float64 oracle's basis, so
the checks are properties of the stored basis that hold at any size:

* the sketches S(V_i) the GPU kept are the sketches of the stored V_i (the
  bfloat16 path sketches with Om1 rounded to bfloat16; exact bfloat16
  products, float32 accumulation: relative 1e-4);
* column j of H is what the oracle's orthogonalisation of Sec. 4.3
  (modified Gram-Schmidt in sketch space with one reorthogonalisation pass,
  oracle.arnoldi.orthogonalise) gives for W = Phi(V_j), s = S(W) against
  the stored V_1..V_j and their sketches, in float64 (1e-3 of the column,
  from the high/low bfloat16 split of the composed matrix Om1 A1); the GPU
  evaluates the same column by classical Gram-Schmidt through the sketched
  Gram matrix, equal in exact arithmetic for a Theta-orthonormal basis;
* the Arnoldi relation Phi(V_j) = sum_{i<=j+1} h_ij V_i holds up to the
  rounding of h_{j+1,j} V_{j+1} to bfloat16 (unit roundoff 2^-9, bound
  taken as 2^-7 of ||h_{j+1,j} V_{j+1}|| plus float32 noise).

The shapes cover ragged tiles (I1 not a multiple of 64, I2 not of 32), one
and several row blocks, channel bands of one, three and five input
channels, J = 1, Om3 given and absent, l1 above 64 (four row tiles per
wave), band half-widths in each operator tier (4, 8, 12), and a run of 70
steps (beyond the 64 whose block of G is staged in LDS)."""
import dataclasses
import sys

import numpy as np
import pytest

from paper_2603_00839_amd import synth
from oracle.operator import Operator
from oracle.sketch import Sketch
from oracle.arnoldi import orthogonalise
from oracle.tensor_algebra import fro_norm
import _util as U

pytestmark = pytest.mark.gpu

CASES = [
    # (I1, I2, J, r1, r2, rB, l1, l2, l3, with_om3, random_bands, m)
    (72, 33, 3, 3, 3, 1, 16, 12, 3, False, True, 6),
    (64, 70, 5, 8, 8, 2, 32, 24, 5, False, True, 6),
    (136, 96, 12, 10, 9, 2, 80, 40, 4, True, False, 5),
    (520, 40, 3, 8, 8, 1, 64, 16, 3, False, False, 5),
    (48, 32, 1, 4, 4, 0, 16, 16, 1, False, True, 6),
    (96, 64, 8, 6, 6, 2, 24, 24, 4, True, True, 6),
    # more steps than the Gram kernel stages in LDS (G read from global memory)
    (48, 32, 2, 3, 3, 1, 16, 8, 2, False, True, 70),
    # the widest channel band (rB = 8: up to 17 input channels per output
    # channel, staged in six groups of three)
    (48, 40, 20, 3, 3, 8, 16, 16, 4, True, True, 4),
]


@pytest.mark.parametrize("case", CASES)
def test_bf16_step_properties(case):
    _check_step(case, toeplitz=True)


# Bands whose rows differ (not a convolution): the step kernel's general form,
# with the band rows streamed per block
NON_TOEPLITZ = [CASES[0], CASES[3], CASES[5]]


@pytest.mark.parametrize("case", NON_TOEPLITZ)
def test_bf16_step_properties_general_bands(case):
    _check_step(case, toeplitz=False)


def _check_step(case, toeplitz):
    from paper_2603_00839_amd import rtg
    I1, I2, J, r1, r2, rB, l1, l2, l3, with_om3, rnd, m = case
    print("[case] bf16 step", case, "toeplitz" if toeplitz else "general bands", file=sys.stderr, flush=True)
    p = synth.small_problem(40 + I1 + J, I1, I2, J, r1, r2, rB, l1, l2, l3, m, nu=1e-2, random_bands=rnd)
    if not with_om3:
        p = dataclasses.replace(p, om3=None)
    if not toeplitz:
        # scale the in-range entries of a few rows of each band
        a1 = p.a1_band.copy()
        a2 = p.a2_band.copy()
        a1[[1, I1 // 2, I1 - 2]] *= np.float32(1.07)
        a2[[0, I2 // 3]] *= np.float32(0.93)
        p = dataclasses.replace(p, a1_band=a1, a2_band=a2)
    op_o = Operator(p.a1_band, p.a2_band, p.b_band)
    sk_b = Sketch(U.bf16_round(p.om1), p.om2, p.om3)        # the sketch the bfloat16 path uses
    og, sg = U.gpu_pair(p)
    C, _ = U.observation(p)
    out = rtg.arnoldi(og, sg, U.to_dev(C), m, basis_dtype=rtg.BF16, bd_tol=1e-10)
    md = int(out["m_done"].item())
    assert md == m
    H = out["H"].cpu().numpy()
    V = [U.from_dev(out["V"][i]) for i in range(m + 1)]
    SVg = out["SV"][:m].cpu().numpy().astype(np.float64)
    SV = np.stack([sk_b(V[i]).ravel() for i in range(m + 1)])      # (a, b, c3) row-major, as stored
    # stored sketches are the sketches of the stored basis
    for i in range(m):
        assert U.rel(SVg[i], SV[i]) < 1e-4, ("S(V_i)", i)
    SVt = [sk_b(V[i]) for i in range(m + 1)]                            # oracle layout
    for j in range(m):
        W = op_o(V[j])
        # column j of H: the oracle's sketch-space MGS + reorthogonalisation
        # against the stored basis
        h, s_orth, _ = orthogonalise(SVt[:j + 1], V[:j + 1], sk_b(W), W, reorth=True)
        ref = np.concatenate([h, [fro_norm(s_orth)]])
        got = H[:j + 2, j]
        assert np.linalg.norm(got - ref) <= 1e-3 * np.linalg.norm(ref), ("H column", j, got, ref)
        # Arnoldi relation on the stored basis
        resid = W - sum(H[i, j] * V[i] for i in range(j + 2))
        bound = 2.0 ** -7 * abs(H[j + 1, j]) * np.linalg.norm(V[j + 1]) + 1e-5 * np.linalg.norm(W)
        assert np.linalg.norm(resid) <= bound, ("relation", j, np.linalg.norm(resid), bound)
