"""FP8 candidate pass of the precision form -- TEST INFRASTRUCTURE ONLY.

The paper searches with full-precision descriptors; the precision form is
not in it.  Its definition (the readings the design notes list) is: every
reference row and every query descriptor is scaled by the largest power of
two 2^e with max|x| * 2^e <= 448, rounded element-wise to OCP e4m3
(round to nearest, ties to even, saturating at +-448) and scaled back; the
candidate key of a pair is ||r~||^2 - 2 q~.r~ of these dequantised values;
the 4k candidates are the 4k smallest (key, reference index) pairs, which
are then re-ranked by their exact squared distance.

This module states that definition plainly in numpy (keys in float64), so
the GPU's candidate choice can be checked against it.  It shares no code
with the GPU library.
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def e4m3_round(x):
    """Nearest OCP e4m3 value of every element (ties to the even
    significand), saturating at +-448; returned as float64.

    e4m3: 1 sign bit, 4 exponent bits (bias 7), 3 significand bits; normal
    values 2^(E) * (1 + m/8) for E = -6..8 (E = 8 stops at 1.75, 448),
    subnormals m * 2^-9.  The spacing of representable values is therefore
    2^(E - 3) in binade E >= -6 and 2^-9 below 2^-6."""
    x = np.asarray(x, np.float64)
    a = np.abs(x)
    _, ex = np.frexp(a)                  # a = f * 2^ex, f in [0.5, 1)
    binade = np.maximum(ex - 1, -6)
    ulp = np.ldexp(1.0, binade - 3)
    q = np.rint(a / ulp) * ulp           # rint: round half to even
    q = np.minimum(q, E4M3_MAX)
    return np.copysign(q, x)


def scale_exponent(m):
    """Largest integer e with m * 2^e <= 448 (m > 0), clamped to [-120, 120];
    0 for m == 0.  Element-wise over an array of row maxima."""
    m = np.asarray(m, np.float64)
    out = np.zeros(m.shape, np.int64)
    for i, v in np.ndenumerate(m):
        if not v > 0:
            continue
        _, ex = np.frexp(v)              # v < 2^ex
        e = 9 - int(ex)                  # v * 2^(9 - ex) < 512
        while np.ldexp(v, e) > E4M3_MAX:
            e -= 1
        out[i] = max(-120, min(120, e))
    return out


def dequantised(X):
    """Rows of X (float32/64 [n, d]) as their per-row-scaled e4m3 values,
    scaled back (float64)."""
    X = np.asarray(X, np.float64)
    e = scale_exponent(np.max(np.abs(X), axis=1))
    return np.ldexp(e4m3_round(np.ldexp(X, e[:, None])), -e[:, None])


def keys(Q, R):
    """Candidate keys ||r~||^2 - 2 q~.r~ of every (query, reference) pair,
    float64 [n_q, n_refs]."""
    Qd, Rd = dequantised(Q), dequantised(R)
    rr = np.einsum("ij,ij->i", Rd, Rd)
    return rr[None, :] - 2.0 * (Qd @ Rd.T)


def candidates(Q, R, n_cand: int):
    """The n_cand smallest (key, index) pairs of every query: (indices
    [n_q, n_cand] in that order, keys [n_q, n_refs])."""
    K = keys(Q, R)
    idx = np.arange(K.shape[1])
    out = np.empty((K.shape[0], n_cand), np.int64)
    for i in range(K.shape[0]):
        out[i] = np.lexsort((idx, K[i]))[:n_cand]
    return out, K
