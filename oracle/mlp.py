"""FP64 reference of the sizing network -- TEST INFRASTRUCTURE ONLY.

40 -> 64 -> 64 -> 64 -> 11 perceptron, exact-erf GELU on the hidden layers,
loss = mean squared error over all samples and outputs.  Parameters use the
flat layout of aiwc_sizer_get_params: W1[64][40], b1, W2[64][64], b2,
W3[64][64], b3, W4[11][64], b4.  Forward and backward are written out by
hand (chain rule) and pinned by central finite differences in the tests.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NF, NH, NT = 40, 64, 11
SHAPES = [(NH, NF), (NH,), (NH, NH), (NH,), (NH, NH), (NH,), (NT, NH), (NT,)]
NPARAM = sum(int(np.prod(s)) for s in SHAPES)


def unpack(p):
    out, o = [], 0
    for s in SHAPES:
        n = int(np.prod(s))
        out.append(np.asarray(p[o:o + n], dtype=np.float64).reshape(s))
        o += n
    return out


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(p, x):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ W1.T + b1
    a1 = gelu(z1)
    z2 = a1 @ W2.T + b2
    a2 = gelu(z2)
    z3 = a2 @ W3.T + b3
    a3 = gelu(z3)
    out = a3 @ W4.T + b4
    return out, (x, z1, a1, z2, a2, z3, a3)


def loss_and_grad(p, x, y):
    W1, b1, W2, b2, W3, b3, W4, b4 = unpack(p)
    out, (x, z1, a1, z2, a2, z3, a3) = forward(p, x)
    y = np.asarray(y, dtype=np.float64)
    n = out.size
    loss = float(np.sum((out - y) ** 2) / n)
    d4 = 2.0 * (out - y) / n
    d3 = (d4 @ W4) * gelu_grad(z3)
    d2 = (d3 @ W3) * gelu_grad(z2)
    d1 = (d2 @ W2) * gelu_grad(z1)
    g = [d1.T @ x, d1.sum(0), d2.T @ a1, d2.sum(0), d3.T @ a2, d3.sum(0), d4.T @ a3, d4.sum(0)]
    return loss, np.concatenate([a.ravel() for a in g])


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest even), returned as float32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (r.astype(np.uint32) << 16).view(np.float32)
