"""Tensor algebra of the paper's Sec. 2 and Sec. 4.1, in float64.

* Einstein product over N modes (Sec. 2.1).
* Frobenius inner product and norm (Sec. 2.2).
* Mode-k product: (X x_k M)[..., a, ...] = sum_{i_k} M[a, i_k] X[..., i_k, ...]
  (the successive mode products of Sec. 3.1).
* The unfolding Psi_IJ with the ``ivec`` linearisation (Sec. 4.1), under
  which the Einstein product becomes an ordinary matrix product.
"""
from __future__ import annotations

import itertools

import numpy as np


def einstein_product(A: np.ndarray, B: np.ndarray, N: int) -> np.ndarray:
    """(A *_N B)[i..., j...] = sum_{k_1..k_N} A[i..., k_1..k_N] B[k_1..k_N, j...].

    The last N modes of A contract with the first N modes of B (Sec. 2.1).
    """
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    if A.shape[A.ndim - N:] != B.shape[:N]:
        raise ValueError("contracted modes differ")
    return np.tensordot(A, B, axes=(list(range(A.ndim - N, A.ndim)), list(range(N))))


def einstein_product_loops(A: np.ndarray, B: np.ndarray, N: int) -> np.ndarray:
    """The same contraction written as explicit sums (tiny tensors only)."""
    L = A.ndim - N
    ishape, kshape = A.shape[:L], A.shape[L:]
    jshape = B.shape[N:]
    out = np.zeros(ishape + jshape)
    for i in itertools.product(*[range(s) for s in ishape]):
        for j in itertools.product(*[range(s) for s in jshape]):
            acc = 0.0
            for k in itertools.product(*[range(s) for s in kshape]):
                acc += A[i + k] * B[k + j]
            out[i + j] = acc
    return out


def frobenius(X: np.ndarray, Y: np.ndarray) -> float:
    """<X, Y>_F = sum over all indices of x * y (Sec. 2.2)."""
    return float(np.sum(np.asarray(X, np.float64) * np.asarray(Y, np.float64)))


def fro_norm(X: np.ndarray) -> float:
    return float(np.sqrt(frobenius(X, X)))


def mode_product(X: np.ndarray, M: np.ndarray, k: int) -> np.ndarray:
    """X x_k M: contract mode k (0-based) of X with the columns of M."""
    X = np.asarray(X, dtype=np.float64)
    M = np.asarray(M, dtype=np.float64)
    Y = np.tensordot(M, X, axes=([1], [k]))   # new mode first
    return np.moveaxis(Y, 0, k)


def ivec(idx, dims) -> int:
    """ivec(i, I) = i_1 + sum_{r>=2} (i_r - 1) prod_{u<r} I_u, written 0-based:
    the first index runs fastest (Sec. 4.1)."""
    out, stride = 0, 1
    for i, d in zip(idx, dims):
        out += i * stride
        stride *= d
    return out


def unfold(X: np.ndarray, N: int) -> np.ndarray:
    """Psi_IJ(X): rows ivec over the first N modes, columns over the rest."""
    X = np.asarray(X)
    I, J = X.shape[:N], X.shape[N:]
    rows = int(np.prod(I)) if I else 1
    cols = int(np.prod(J)) if J else 1
    out = np.zeros((rows, cols))
    for i in itertools.product(*[range(s) for s in I]):
        for j in itertools.product(*[range(s) for s in J]):
            out[ivec(i, I), ivec(j, J)] = X[i + j]
    return out


def vec(X: np.ndarray) -> np.ndarray:
    """Column-major vectorisation (first index fastest), as in Sec. 3.1.2."""
    return np.asarray(X, dtype=np.float64).reshape(-1, order="F")
