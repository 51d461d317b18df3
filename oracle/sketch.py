"""Mode-wise sketch and the sketched Einstein inner product (Sec. 3).

S(X) = X x_1 Om1 x_2 Om2 x_3 Om3 (the global tensor sketching operator of
Sec. 3.1 / the compressed tensor X_Theta), and
<X, Y>_Theta = <S(X), S(Y)>_F (Definition of the sketched Einstein inner
product).  ``None`` stands for an identity factor.
"""
from __future__ import annotations

import numpy as np

from .tensor_algebra import mode_product, frobenius


class Sketch:
    def __init__(self, om1=None, om2=None, om3=None):
        self.om = [None if o is None else np.asarray(o, np.float64) for o in (om1, om2, om3)]

    def __call__(self, X: np.ndarray) -> np.ndarray:
        Y = np.asarray(X, np.float64)
        for k, om in enumerate(self.om):
            if om is not None:
                Y = mode_product(Y, om, k)
        return Y

    def inner(self, X, Y) -> float:
        return frobenius(self(X), self(Y))

    def norm(self, X) -> float:
        s = self(X)
        return float(np.sqrt(frobenius(s, s)))

    def dense(self, dims) -> np.ndarray:
        """Theta = Om3 (x) Om2 (x) Om1 with vec(S(X)) = Theta vec(X)
        (vectorised form, Sec. 3.1.2)."""
        mats = [np.eye(d) if om is None else om for om, d in zip(self.om, dims)]
        return np.kron(mats[2], np.kron(mats[1], mats[0]))


def identity_sketch() -> Sketch:
    return Sketch(None, None, None)
