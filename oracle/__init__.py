"""FP64 CPU oracle for RTG-GMRES (randomized tensor global GMRES).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, float64 NumPy
implementation of what the GPU hot path computes, written from the paper
(Badahmane, "Randomized Tensor Krylov Subspace Methods via Sketched Einstein
Product").  Only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import it.  It shares no code with the HIP library and
imports nothing from it; the only common module is the seeded input generator
``paper_2603_00839_amd.synth``, which holds no solver arithmetic.

Modules
-------
tensor_algebra  Einstein product, Frobenius product, mode-k products and the
                unfolding Psi_IJ (Sec. 2, Sec. 4.1).
operator        Phi(X) = A *_2 X *_1 B with separable banded factors
                (eq. (2), Sec. 5.1-5.3).
sketch          the mode-wise sketch S(X) and the sketched inner product
                (Sec. 3, Definition of the sketched Einstein inner product).
arnoldi         sketched tensor global Arnoldi (Sec. 4.3).
projected       Givens least squares, projected Tikhonov (eqs. (12)-(14)),
                discrepancy-principle choice of mu.
gmres           RTG-GMRES driver (algorithm "Block GMRES via Sketched Einstein
                Product", Sec. 4.4).
golub_kahan     sketched Block Golub-Kahan bidiagonalisation and its
                regularised solve (Sec. 4.5).
metrics         RE and PSNR (Sec. 5.5).
cnn             float64 reference of the warm-start convolutional network.
"""
from . import tensor_algebra, operator, sketch, arnoldi, projected, gmres, golub_kahan, metrics  # noqa: F401

FLAG_BREAKDOWN = 1
FLAG_DISCREP_UNREACHABLE = 2
FLAG_MU_INF = 4
FLAG_NONFINITE = 8
FLAG_NOT_CONVERGED = 16
