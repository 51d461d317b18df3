"""The restoration operator Phi (eq. (2); Sec. 5.1-5.3), in float64.

Phi(X) = A *_2 X *_1 B with a separable blur A = A1 (x) A2, i.e.
a[i1, i2, k1, k2] = A1[i1, k1] A2[i2, k2], acting on the two spatial modes,
and B acting on the third mode from the right:
(X *_1 B)[i1, i2, j] = sum_k X[i1, i2, k] B[k, j].
Hence Phi(X)[i1, i2, j] = sum A1[i1,k1] A2[i2,k2] X[k1,k2,k] B[k,j], which is
X x_1 A1 x_2 A2 x_3 B^T.  Zero boundary conditions (Sec. 5.1) are encoded in
the factors: rows of a band that reach outside the image are truncated.
"""
from __future__ import annotations

import numpy as np

from .tensor_algebra import einstein_product, mode_product, fro_norm


def band_to_dense(band: np.ndarray) -> np.ndarray:
    """Square matrix M with M[i, i + d] = band[i, d + r] (zero outside)."""
    band = np.asarray(band, dtype=np.float64)
    I, w = band.shape
    r = (w - 1) // 2
    M = np.zeros((I, I))
    for i in range(I):
        for d in range(-r, r + 1):
            k = i + d
            if 0 <= k < I:
                M[i, k] = band[i, d + r]
    return M


class Operator:
    """Dense float64 factors of Phi built from the band arrays."""

    def __init__(self, a1_band, a2_band, b_band):
        self.A1 = band_to_dense(a1_band)
        self.A2 = band_to_dense(a2_band)
        self.B = band_to_dense(b_band)

    @property
    def shape(self):
        return (self.A1.shape[0], self.A2.shape[0], self.B.shape[0])

    def __call__(self, X: np.ndarray) -> np.ndarray:
        return phi(X, self.A1, self.A2, self.B)

    def transpose_apply(self, X: np.ndarray) -> np.ndarray:
        """Phi^T(X) = X x_1 A1^T x_2 A2^T x_3 B (adjoint w.r.t. <.,.>_F)."""
        return phi(X, self.A1.T, self.A2.T, self.B.T)

    def dense(self) -> np.ndarray:
        """n x n matrix of vec(Phi(X)) = (B^T (x) A2 (x) A1) vec(X)."""
        return np.kron(self.B.T, np.kron(self.A2, self.A1))


def phi(X, A1, A2, B) -> np.ndarray:
    """Phi(X) = X x_1 A1 x_2 A2 x_3 B^T (dense factors, any sizes)."""
    Y = mode_product(X, A1, 0)
    Y = mode_product(Y, A2, 1)
    return mode_product(Y, np.asarray(B, np.float64).T, 2)


def blur_tensor(A1, A2) -> np.ndarray:
    """Fourth-order blur tensor a[i1, i2, k1, k2] = A1[i1, k1] A2[i2, k2]."""
    return np.einsum("ik,jl->ijkl", np.asarray(A1, np.float64), np.asarray(A2, np.float64))


def phi_einstein(X, A1, A2, B) -> np.ndarray:
    """Phi(X) = (A *_2 X) *_1 B evaluated literally with Einstein products
    (tiny sizes only: builds the fourth-order tensor)."""
    AX = einstein_product(blur_tensor(A1, A2), X, 2)
    return einstein_product(AX, B, 1)


def convolve_psf_zero_bc(X, P) -> np.ndarray:
    """Direct 2-D convolution of every channel with a (2r+1) x (2r+1) PSF,
    zero boundary conditions (eq. (57) generalised to any odd PSF size):
    C[i, j, k] = sum_{a,b} P[r - a, r - b] X[i + a, j + b, k],
    summed as one shifted copy of X per PSF entry (terms whose X index leaves
    the image are zero)."""
    X = np.asarray(X, np.float64)
    P = np.asarray(P, np.float64)
    r = (P.shape[0] - 1) // 2
    I1, I2, _ = X.shape
    out = np.zeros_like(X)
    for a in range(-r, r + 1):
        for b in range(-r, r + 1):
            i_lo, i_hi = max(0, -a), min(I1, I1 - a)      # output rows with 0 <= i + a < I1
            j_lo, j_hi = max(0, -b), min(I2, I2 - b)
            if i_lo >= i_hi or j_lo >= j_hi:
                continue
            out[i_lo:i_hi, j_lo:j_hi, :] += P[r - a, r - b] * X[i_lo + a:i_hi + a, j_lo + b:j_hi + b, :]
    return out


def psf_tensor(P, I1: int, I2: int) -> np.ndarray:
    """Fourth-order blur tensor built directly from the PSF entries (eqs.
    (56)-(57)): a[i1, i2, k1, k2] = P[r - (k1 - i1), r - (k2 - i2)] when both
    offsets lie within the PSF, else 0 (tiny sizes only)."""
    P = np.asarray(P, np.float64)
    r = (P.shape[0] - 1) // 2
    a = np.zeros((I1, I2, I1, I2))
    for i1 in range(I1):
        for i2 in range(I2):
            for k1 in range(max(0, i1 - r), min(I1, i1 + r + 1)):
                for k2 in range(max(0, i2 - r), min(I2, i2 + r + 1)):
                    a[i1, i2, k1, k2] = P[r - (k1 - i1), r - (k2 - i2)]
    return a


class PSFOperator:
    """Phi(X) = (A *_2 X) *_1 B with A built from a general (non-separable)
    PSF (eqs. (56)-(57)): every channel convolved with P (zero boundary
    conditions), then the channel mix, (X *_1 B)[.., j] = sum_k X[.., k] B[k, j]."""

    def __init__(self, psf, b_band, dims):
        self.P = np.asarray(psf, np.float64)
        self.B = band_to_dense(b_band)
        self.dims = tuple(dims)

    @property
    def shape(self):
        return self.dims

    def __call__(self, X: np.ndarray) -> np.ndarray:
        return mode_product(convolve_psf_zero_bc(X, self.P), self.B.T, 2)

    def transpose_apply(self, Y: np.ndarray) -> np.ndarray:
        """Adjoint w.r.t. <.,.>_F: the channel mix transposed, then the
        convolution with the PSF rotated by 180 degrees."""
        return convolve_psf_zero_bc(mode_product(np.asarray(Y, np.float64), self.B, 2), self.P[::-1, ::-1])

    def dense(self) -> np.ndarray:
        """n x n matrix of vec(Phi(X)) (column-major vec), column by column."""
        n = int(np.prod(self.dims))
        M = np.empty((n, n))
        for c in range(n):
            e = np.zeros(n)
            e[c] = 1.0
            M[:, c] = self(e.reshape(self.dims, order="F")).ravel(order="F")
        return M


def make_observation(op: Operator, x_true, noise_dir, nu):
    """C = Phi(X_true) + N with N = nu ||Phi(X_true)||_F G / ||G||_F, so the
    noise level nu = ||N||_F / ||C_hat||_F is met exactly (eq. (59)).

    Returns (C float64, delta = ||N||_F, C_hat)."""
    c_hat = op(np.asarray(x_true, np.float64))
    G = np.asarray(noise_dir, np.float64)
    delta = nu * fro_norm(c_hat)
    N = G * (delta / fro_norm(G))
    return c_hat + N, delta, c_hat
