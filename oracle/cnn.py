"""Float64 reference of the warm-start network (test infrastructure).

The network maps an observation C (I1 x I2 x 3) to an initial guess
X0 = C + f(C), where f is six 3x3 "same" convolutions with zero padding,
3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3 channels, ReLU after the first five,
and biases.  It is trained with the mean squared error to the RTG-GMRES
solution and Adam.  This module writes the forward pass, the hand-derived
backward pass and Adam out in plain NumPy; tests pin it with central finite
differences and closed forms.

Conventions: activations are arrays x[i1, i2, c]; a weight tensor is
w[co, t1, t2, ci] with taps t1, t2 in {0, 1, 2} meaning offsets -1, 0, +1:
out[i1, i2, co] = b[co] + sum w[co, t1, t2, ci] x[i1 + t1 - 1, i2 + t2 - 1, ci].
"""
from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

CHANNELS = [3, 32, 32, 32, 32, 32, 3]


def pad1(x: np.ndarray) -> np.ndarray:
    return np.pad(x, ((1, 1), (1, 1), (0, 0)))


def conv3x3(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Zero-padded 3x3 correlation with bias."""
    I1, I2, _ = x.shape
    xp = pad1(np.asarray(x, np.float64))
    out = np.broadcast_to(np.asarray(b, np.float64), (I1, I2, w.shape[0])).copy()
    for t1 in range(3):
        for t2 in range(3):
            out += np.einsum("ijc,oc->ijo", xp[t1:t1 + I1, t2:t2 + I2, :], w[:, t1, t2, :])
    return out


def conv3x3_loops(x, w, b):
    """The same correlation as explicit sums (tiny inputs only)."""
    I1, I2, Ci = x.shape
    Co = w.shape[0]
    out = np.zeros((I1, I2, Co))
    for i in range(I1):
        for j in range(I2):
            for o in range(Co):
                acc = b[o]
                for t1 in range(3):
                    for t2 in range(3):
                        a, c = i + t1 - 1, j + t2 - 1
                        if 0 <= a < I1 and 0 <= c < I2:
                            acc += sum(w[o, t1, t2, q] * x[a, c, q] for q in range(Ci))
                out[i, j, o] = acc
    return out


def init_params(rng, channels=CHANNELS) -> List[Dict[str, np.ndarray]]:
    """He-normal weights, zero biases; the last layer is all zero so that the
    untrained network returns X0 = C."""
    params = []
    L = len(channels) - 1
    for l in range(L):
        ci, co = channels[l], channels[l + 1]
        if l == L - 1:
            w = np.zeros((co, 3, 3, ci))
        else:
            w = rng.standard_normal((co, 3, 3, ci)) * math.sqrt(2.0 / (9 * ci))
        params.append({"w": w, "b": np.zeros(co)})
    return params


def forward(params, C):
    """Returns (X0, acts) with acts[0] = C and acts[l] the (post-ReLU)
    output of layer l for the hidden layers, acts[L] the last conv output."""
    acts = [np.asarray(C, np.float64)]
    L = len(params)
    x = acts[0]
    for l, p in enumerate(params):
        y = conv3x3(x, p["w"], p["b"])
        if l < L - 1:
            y = np.maximum(y, 0.0)
        acts.append(y)
        x = y
    return acts[0] + acts[-1], acts


def mse(X0, Y) -> float:
    d = np.asarray(X0, np.float64) - np.asarray(Y, np.float64)
    return float(np.mean(d * d))


def conv3x3_backward(x, w, g):
    """Gradients of out = conv3x3(x, w, b) given g = dL/dout:
    dW[co,t1,t2,ci] = sum_{i1,i2} g[i1,i2,co] x[i1+t1-1, i2+t2-1, ci],
    db[co] = sum g[..., co],
    dx[a1,a2,ci] = sum_{co,t1,t2} w[co,t1,t2,ci] g[a1-t1+1, a2-t2+1, co]."""
    I1, I2, _ = x.shape
    xp = pad1(x)
    dW = np.zeros_like(w)
    for t1 in range(3):
        for t2 in range(3):
            dW[:, t1, t2, :] = np.einsum("ijo,ijc->oc", g, xp[t1:t1 + I1, t2:t2 + I2, :])
    db = g.sum(axis=(0, 1))
    dxp = np.zeros_like(xp)
    for t1 in range(3):
        for t2 in range(3):
            dxp[t1:t1 + I1, t2:t2 + I2, :] += np.einsum("ijo,oc->ijc", g, w[:, t1, t2, :])
    return dW, db, dxp[1:-1, 1:-1, :]


def backward(params, acts, Y):
    """Gradients of mse(X0, Y) w.r.t. every weight and bias."""
    L = len(params)
    X0 = acts[0] + acts[-1]
    g = 2.0 * (X0 - Y) / X0.size          # dL/dX0 = dL/d(last conv output)
    grads = [None] * L
    for l in range(L - 1, -1, -1):
        dW, db, dx = conv3x3_backward(acts[l], params[l]["w"], g)
        grads[l] = {"w": dW, "b": db}
        if l > 0:
            g = dx * (acts[l] > 0.0)          # through the ReLU of layer l - 1
    return grads


class Adam:
    """Adam with bias correction (beta1 0.9, beta2 0.999, eps 1e-8)."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [{k: np.zeros_like(v) for k, v in p.items()} for p in params]
        self.v = [{k: np.zeros_like(v) for k, v in p.items()} for p in params]
        self.t = 0

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for p, g, m, v in zip(params, grads, self.m, self.v):
            for k in p:
                m[k] = self.b1 * m[k] + (1 - self.b1) * g[k]
                v[k] = self.b2 * v[k] + (1 - self.b2) * g[k] * g[k]
                p[k] = p[k] - lr * (m[k] / c1) / (np.sqrt(v[k] / c2) + self.eps)
        return params
