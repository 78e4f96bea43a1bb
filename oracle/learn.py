"""Oracle of the learned importance proposal (an extension of the paper's
sampler; the paper has no learned component).

TEST INFRASTRUCTURE ONLY (see the package docstring).

  * The network: 8 -> 64 -> 64 -> 1, ReLU, ReLU, sigmoid, so
      z1 = W1 f + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2),
      z3 = w3 . h2 + b3, g = 1 / (1 + exp(-z3)).
    Parameters are one float32 vector of 4,801 entries in the order
    W1 [64, 8] (row = unit), b1 [64], W2 [64, 64], b2 [64], w3 [64], b3 [1].
    ``forward`` evaluates it in binary64.  With ``bf16=True`` it mimics the
    storage precision of the GPU kernels: the weight matrices, the features
    and the two hidden activations are rounded to bfloat16 (round to
    nearest even), biases stay float32.
  * Loss: mean binary cross-entropy of g against y in {0, 1}; gradients by
    the chain rule in binary64 (rounding treated as the identity).
  * Adam: the update of Kingma and Ba (ICLR 2015) with bias correction.
  * Quantisation: h = eps + (1 - eps) g, h_int = max(1, floor(h 2^s + 1/2))
    with s = clamp(63 - bitlen(W), 1, 16), every step in float32 as the GPU
    does it (the integer h_int is decided in the same precision).
  * ``is_expectation``: the exact expectation of the importance-sampling
    estimate over every delta-centred path, in rational arithmetic.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np

N_IN, N_H = 8, 64
OFF_W1 = 0
OFF_B1 = OFF_W1 + N_H * N_IN
OFF_W2 = OFF_B1 + N_H
OFF_B2 = OFF_W2 + N_H * N_H
OFF_W3 = OFF_B2 + N_H
OFF_B3 = OFF_W3 + N_H
N_PARAMS = OFF_B3 + 1  # 4801


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (nearest even) and return as float64.  float64
    input is first rounded to float32."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r.astype(np.uint32)).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def bf16_bits(x) -> np.ndarray:
    """bfloat16 bit patterns (uint16) of float32 values (nearest even)."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint16)


def bf16_from_bits(b) -> np.ndarray:
    u = np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def unpack(params):
    p = np.asarray(params, dtype=np.float32)
    assert p.shape == (N_PARAMS,)
    return (p[OFF_W1:OFF_B1].reshape(N_H, N_IN), p[OFF_B1:OFF_W2], p[OFF_W2:OFF_B2].reshape(N_H, N_H),
            p[OFF_B2:OFF_W3], p[OFF_W3:OFF_B3], p[OFF_B3:])


def forward(params, F, bf16: bool = True):
    """Forward pass over rows of F [n, 8]; returns a dict of the
    intermediate values (each [n, ...]) and g."""
    W1, b1, W2, b2, w3, b3 = (np.asarray(a, dtype=np.float64) for a in unpack(params))
    F = np.asarray(F, dtype=np.float64)
    rnd = bf16_round if bf16 else (lambda x: np.asarray(x, dtype=np.float64))
    if bf16:
        W1, W2, w3 = rnd(W1), rnd(W2), rnd(w3)
        F = rnd(F)
    z1 = F @ W1.T + b1
    h1 = rnd(np.maximum(z1, 0.0))
    z2 = h1 @ W2.T + b2
    h2 = rnd(np.maximum(z2, 0.0))
    z3 = h2 @ w3 + b3[0]
    g = 1.0 / (1.0 + np.exp(-z3))
    return dict(F=F, W1=W1, W2=W2, w3=w3, z1=z1, h1=h1, z2=z2, h2=h2, z3=z3, g=g)


def softplus(x):
    return np.logaddexp(0.0, x)


def bce_loss(z3, y) -> float:
    """mean of -(y log g + (1 - y) log(1 - g)) with g = sigmoid(z3)."""
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(y * softplus(-z3) + (1.0 - y) * softplus(z3)))


def grad(params, F, y, bf16: bool = True):
    """(loss, gradient [4801]) of the mean BCE over the rows of F."""
    c = forward(params, F, bf16)
    y = np.asarray(y, dtype=np.float64)
    n = F.shape[0]
    dz3 = (c["g"] - y) / n
    G = np.zeros(N_PARAMS, np.float64)
    G[OFF_B3] = dz3.sum()
    G[OFF_W3:OFF_B3] = c["h2"].T @ dz3
    dz2 = np.outer(dz3, c["w3"]) * (c["z2"] > 0)
    G[OFF_B2:OFF_W3] = dz2.sum(axis=0)
    G[OFF_W2:OFF_B2] = (dz2.T @ c["h1"]).ravel()
    dz1 = (dz2 @ c["W2"]) * (c["z1"] > 0)
    G[OFF_B1:OFF_W2] = dz1.sum(axis=0)
    G[OFF_W1:OFF_B1] = (dz1.T @ c["F"]).ravel()
    return bce_loss(c["z3"], y), G


def adam_step(params, m, v, g, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update in binary64; returns (params, m, v)."""
    p = np.asarray(params, dtype=np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def quant_shift(W: int) -> int:
    return min(16, max(1, 63 - int(W).bit_length()))


def quantize(g, W: int, eps: float = 0.1, normalize: bool = False) -> np.ndarray:
    """h_int per edge from g (float32), every operation in float32; g is
    taken as 0 where it is NaN and clamped to [0, 1]; with normalize it is
    then divided by its maximum (when that is positive)."""
    g = np.asarray(g, dtype=np.float32).copy()
    g[np.isnan(g)] = np.float32(0)
    g = np.clip(g, np.float32(0), np.float32(1))
    if normalize and g.size and g.max() > 0:
        g = (g / g.max()).astype(np.float32)
    e = np.float32(eps)
    one_m = np.float32(1) - e
    h = e + one_m * g                                # float32 ops
    hs = h * np.float32(2.0 ** quant_shift(W))       # exact scaling
    v = np.floor(hs + np.float32(0.5)).astype(np.float64)
    return np.maximum(1, v).astype(np.uint32)


def is_expectation(og, w, hw, motif: bytes):
    """Exact expectation of one importance-sampling estimate (k = 1) over
    the proposal: sum over every path P centred at p of
    (h_p / Q) * floor(X_P 2^64 / h_p) 2^-64 * Q, with X_P from the oracle's
    CheckMotif.  Returns (expectation as a Fraction, the exact count C =
    sum of X_P)."""
    Q = int(hw.S[-1])
    E = Fraction(0)
    C = 0
    orders = og.orders()
    in_eid, out_eid = orders["in_eid"], orders["out_eid"]
    for p in range(og.m):
        hp = int(hw.h[p])
        for j1 in range(int(w.a[p])):
            for j3 in range(int(w.b[p])):
                st, X = og.check_motif(motif, w.delta, int(in_eid[w.lo_in[p] + j1]),
                                       int(out_eid[p]), int(out_eid[w.lo_out[p] + j3]))
                C += X
                if X:
                    t = (X << 64) // hp
                    E += Fraction(hp, Q) * Fraction(t, 1 << 64) * Q
    return E, C
