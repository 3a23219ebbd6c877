"""Oracle: the start-vector network (a 3-layer perceptron) in FP64, forward,
backward and Adam, with the GPU's BF16 rounding points reproduced.

TEST INFRASTRUCTURE ONLY -- see ``oracle/__init__.py``.

The network is not part of the paper.  It maps the parameters (Re, alpha) of a
linear stability problem to a block of low Fourier coefficients from which an
Arnoldi start vector (Algorithm 1 takes any start vector) is assembled.

Architecture: x = features(Re, alpha) (2) -> tanh(x W1 + b1) (512) -> tanh(. W2 + b2) (512) ->
. W3 + b3 (2048).  Loss L = sum (y - t)^2 / (B * 2048).
Numerics of the GPU form, reproduced here: the operands of the two large
products in each direction (layers 2 and 3 forward, their weight gradients and
back-propagated activations) are rounded to bfloat16 (round to nearest, ties
to even, from FP32) before the product; everything else (layer 1, biases,
tanh, the loss, Adam) is exact here and FP32 on the GPU.  With ``quantize =
False`` the oracle is the plain FP64 network (used for finite differences).

Adam: Kingma & Ba (2015), m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
w -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Parity status: pinned -- backward against central finite differences of the
unquantised loss; bfloat16 rounding against hand-checked bit patterns; Adam
against its closed forms (first step -lr g/(|g| + eps); constant gradients move
lr g/(|g| + eps) per step) and a two-step case worked by hand; see
tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import numpy as np

from .rng import splitmix64

WIDTH = 512
OUT = 2048
IN_LO = (5.0, 0.25)     # (Re, alpha) box of the neutral-curve sweep
IN_HI = (40.0, 1.0)
ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16(x):
    """Round to bfloat16 (via FP32, round to nearest even) and return FP64."""
    x32 = np.asarray(x, dtype=np.float32)
    b = x32.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    r = ((b + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def init_params(seed, width=WIDTH, out=OUT):
    """Xavier-uniform weights (Glorot & Bengio 2010: U(-l, l), l = sqrt(6/(fan_in +
    fan_out))), zero biases.  Element e of the flat parameter vector (layout of
    ``flatten``) draws u = (splitmix64 output e of ``seed``) >> 11 times 2^-53 and
    takes l (2u - 1); the values are then held in FP32 like the GPU master copy."""
    shapes = dict(W1=(2, width), b1=(width,), W2=(width, width), b2=(width,), W3=(width, out), b3=(out,))
    P, o = {}, 0
    for k in ORDER:
        cnt = int(np.prod(shapes[k]))
        if k.startswith("W"):
            a, b = shapes[k]
            lim = np.float32(np.sqrt(6.0 / (a + b)))
            u = (splitmix64(seed, cnt, o) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
            P[k] = (lim * (2.0 * u - 1.0)).astype(np.float32).astype(np.float64).reshape(shapes[k])
        else:
            P[k] = np.zeros(shapes[k])
        o += cnt
    return P


def features(re_alpha, lo=IN_LO, hi=IN_HI):
    """Network input: (Re, alpha) mapped affinely onto [-1, 1] over the training
    box [lo, hi]."""
    x = np.asarray(re_alpha, dtype=np.float64).reshape(-1, 2)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    return 2.0 * (x - lo) / (hi - lo) - 1.0


def forward(P, X, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    Z1 = X @ P["W1"] + P["b1"]
    A1 = np.tanh(Z1)
    Z2 = q(A1) @ q(P["W2"]) + P["b2"]
    A2 = np.tanh(Z2)
    Y = q(A2) @ q(P["W3"]) + P["b3"]
    return Y, (A1, A2)


def loss(P, X, T, quantize=True):
    Y, _ = forward(P, X, quantize)
    return float(np.sum((Y - T) ** 2) / Y.size)


def grads(P, X, T, quantize=True):
    q = bf16 if quantize else (lambda a: np.asarray(a, dtype=np.float64))
    Y, (A1, A2) = forward(P, X, quantize)
    dY = 2.0 * (Y - T) / Y.size
    g = {}
    g["W3"] = q(A2).T @ q(dY)
    g["b3"] = dY.sum(axis=0)
    dA2 = q(dY) @ q(P["W3"]).T
    dZ2 = dA2 * (1.0 - A2 ** 2)
    g["W2"] = q(A1).T @ q(dZ2)
    g["b2"] = dZ2.sum(axis=0)
    dA1 = q(dZ2) @ q(P["W2"]).T
    dZ1 = dA1 * (1.0 - A1 ** 2)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g, float(np.sum((Y - T) ** 2) / Y.size)


def adam_step(P, G, state, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    for key in P:
        m, v = state.setdefault(key, (np.zeros_like(P[key]), np.zeros_like(P[key])))
        m = b1 * m + (1 - b1) * G[key]
        v = b2 * v + (1 - b2) * G[key] ** 2
        state[key] = (m, v)
        P[key] = P[key] - lr * (m / (1 - b1 ** t)) / (np.sqrt(v / (1 - b2 ** t)) + eps)
    return P


def flatten(P):
    """Parameters (or gradients) as one vector in the GPU's layout: W1, b1, W2,
    b2, W3, b3, each row-major [in][out]."""
    return np.concatenate([np.asarray(P[k], dtype=np.float64).ravel() for k in ORDER])


def unflatten(vec, width=WIDTH, out=OUT):
    shapes = dict(W1=(2, width), b1=(width,), W2=(width, width), b2=(width,), W3=(width, out), b3=(out,))
    P, o = {}, 0
    for k in ORDER:
        n = int(np.prod(shapes[k]))
        P[k] = np.asarray(vec[o:o + n], dtype=np.float64).reshape(shapes[k])
        o += n
    return P
