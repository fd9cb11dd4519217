"""FP64 oracle of the learned cross-rank predictor (an addition to the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper computes every cross rank by binary search (Section 2, Steps 1-2).
The library can instead predict a rank with a small network and correct the
prediction with the bounded exponential search of ``oracle.gallop``; the
network never changes a result, only where the search starts.  This module
is the plain numpy definition of that network, its loss, its gradient and
its optimiser step, against which the GPU kernels are checked.

Model: a 2-layer perceptron 1 -> 32 (ReLU) -> 1 mapping a key to its
normalised rank r / len(X) in the target array X, i.e. a model of the
cumulative distribution of X.

Parameter vector (97 values): W1[0:32], b1[32:64], w2[64:96], b2[96].
"""
from __future__ import annotations

import numpy as np

HIDDEN = 32
NPARAM = 3 * HIDDEN + 1


def unsigned_order(keys: np.ndarray) -> np.ndarray:
    """Map keys to unsigned integers with the same order: signed integers with
    the sign bit flipped; floats by IEEE 754 totalOrder from sign and
    magnitude (negative: 2^(b-1) - 1 - magnitude, positive: 2^(b-1) +
    magnitude), returned as Python-exact uint64."""
    if keys.dtype == np.int32:
        return (keys.view(np.uint32) ^ np.uint32(0x80000000)).astype(np.uint64)
    if keys.dtype == np.int64:
        return keys.view(np.uint64) ^ np.uint64(1 << 63)
    if keys.dtype in (np.float32, np.float64):
        bits = 32 if keys.dtype == np.float32 else 64
        b = keys.view(np.uint32 if bits == 32 else np.uint64).astype(np.uint64)
        half = np.uint64(1 << (bits - 1))
        mag = b & (half - np.uint64(1))
        neg = (b & half) != 0
        return np.where(neg, (half - np.uint64(1)) - mag, half + mag)
    return keys.astype(np.uint64)


def key_bits(keys: np.ndarray) -> int:
    return 64 if keys.dtype in (np.uint64, np.int64, np.float64) else 32


def features(keys: np.ndarray) -> np.ndarray:
    """phi(key) = log2(u + 1) / bits, u the order-preserving unsigned form."""
    u = unsigned_order(keys).astype(np.float64)
    return np.log2(u + 1.0) / key_bits(keys)


def unpack(params: np.ndarray):
    p = np.asarray(params, dtype=np.float64)
    return p[0:32], p[32:64], p[64:96], p[96]


def forward(params, phi):
    """Returns (y, pre, h): output, hidden pre-activation and activation."""
    W1, b1, w2, b2 = unpack(params)
    pre = np.outer(phi, W1) + b1
    h = np.maximum(pre, 0.0)
    y = h @ w2 + b2
    return y, pre, h


def loss(params, phi, target):
    """Mean squared error of the normalised rank."""
    y, _, _ = forward(params, phi)
    d = y - target
    return float(np.mean(d * d))


def loss_and_grad(params, phi, target):
    """Loss and its gradient by the chain rule (ReLU derivative 0 at pre = 0)."""
    W1, b1, w2, b2 = unpack(params)
    y, pre, h = forward(params, phi)
    S = len(phi)
    d = y - target
    dy = 2.0 * d / S
    g = np.empty(NPARAM)
    g[64:96] = h.T @ dy
    g[96] = dy.sum()
    dh = np.outer(dy, w2) * (pre > 0.0)
    g[0:32] = dh.T @ phi
    g[32:64] = dh.sum(axis=0)
    return float(np.mean(d * d)), g


def adam_step(params, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; step >= 1.
    Returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


KNOT_MIN_GAP = 1e-6


def init_params(sample_phi_sorted: np.ndarray, sample_target: np.ndarray) -> np.ndarray:
    """Interpolating knot initialisation: hidden unit k is ReLU(phi - c_k)
    with c_k the feature of sample i_k = floor((k + 1/2) S / 32) of the sorted
    sample, and the output layer makes the network the piecewise-linear
    interpolant of the points (c_k, t_k), t_k the target of sample i_k:
    b2 = t_0, w2[k] = s_k - s_{k-1} with s_k the slope from knot k to knot
    k + 1 (0 when the two knots are closer than KNOT_MIN_GAP, and s_31 = 0:
    flat past the last knot)."""
    S = len(sample_phi_sorted)
    p = np.zeros(NPARAM)
    if S == 0:
        return p
    idx = np.minimum(((np.arange(HIDDEN) + 0.5) * S / HIDDEN).astype(np.int64), S - 1)
    c = np.asarray(sample_phi_sorted, dtype=np.float64)[idx]
    t = np.asarray(sample_target, dtype=np.float64)[idx]
    slope = np.zeros(HIDDEN)
    for k in range(HIDDEN - 1):
        gap = c[k + 1] - c[k]
        slope[k] = (t[k + 1] - t[k]) / gap if gap > KNOT_MIN_GAP else 0.0
    p[0:32] = 1.0
    p[32:64] = -c
    p[64:96] = slope - np.concatenate([[0.0], slope[:-1]])
    p[96] = t[0]
    return p


def predict_rank(params, keys: np.ndarray, length: int) -> np.ndarray:
    """Predicted rank: y * length rounded to the nearest integer (halves to
    even), clamped to [0, length]; 0 where y * length is not a number.  The
    prediction only chooses where the corrective search starts, so any value
    in [0, length] is a valid start."""
    y, _, _ = forward(params, features(keys))
    r = np.rint(np.asarray(y, dtype=np.float64) * float(length))
    r = np.where(np.isnan(r), 0.0, r)
    return np.clip(r, 0.0, float(length)).astype(np.int64)
