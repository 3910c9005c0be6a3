"""Oracle: max-convolution and its p-norm estimate, FP64 on CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Serang, arXiv 1511.05690, Sec. 1 and Sec. 2.1.
  * The max-convolution of nonnegative vectors x (length n) and y (length
    m) is z[t] = max_i x[i] y[t - i], t = 0 .. n + m - 2 (the maximum of the
    list u^(t) of products).
  * The p-norm estimate: with every element raised to p, the sum over the
    same list is an ordinary convolution, (x^p * y^p)[t]; its 1/p-th power
    bounds the max from above and converges to it as p grows (Sec. 1).
  * Scaling (Sec. 2.1 for the ring call, used the same way here): x' = x /
    max x, y' = y / max y, so every term lies in [0, 1]; the result is
    multiplied back by max x max y.
  * Selection: per index, the largest p of the family whose ring result is
    at least tau; the paper's tau for FFT convolution is 1e-12.  Here the
    ring (the ordinary convolution) is numpy's direct convolution, which is
    the plain definition (the GPU uses FFT convolution, the paper's H).
  * Reading: no stable p -> the smallest p of the family (index 255), as in
    the product.
"""

import numpy as np

PSTAR_NONE = 255
TAU_FFT = 1e-12


def exact_maxconv(x, y):
    """z[t] = max_i x[i] y[t - i] (the definition), batched over a leading
    axis."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    b, n = x.shape
    m = y.shape[1]
    z = np.zeros((b, n + m - 1))
    for i in range(n):
        z[:, i:i + m] = np.maximum(z[:, i:i + m], x[:, i:i + 1] * y)
    return z


def maxconv_estimate(x, y, P, tau=TAU_FFT):
    """The p-norm estimate of the max-convolution (Sec. 1): per batch item
    and index t, S_p[t] = (x'^p * y'^p)[t] for p in P (direct convolution),
    p* the largest p with S_p[t] >= tau, z[t] = max x max y S_{p*}^(1/p*).
    Returns dict z, pstar_idx (uint8, 255 = none stable), S (len(P), b, L)."""
    P = [int(p) for p in P]
    if any(p <= 0 for p in P) or any(P[i] >= P[i + 1] for i in range(len(P) - 1)):
        raise ValueError("P must be strictly ascending positive integers")
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    b, n = x.shape
    m = y.shape[1]
    rx = x.max(axis=1)
    ry = y.max(axis=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        xs = np.where(rx[:, None] > 0, x / rx[:, None], 0.0)
        ys = np.where(ry[:, None] > 0, y / ry[:, None], 0.0)
    S = np.stack([np.stack([np.convolve(xs[i] ** p, ys[i] ** p) for i in range(b)]) for p in P])
    idx = np.full((b, n + m - 1), PSTAR_NONE, dtype=np.uint8)
    for q in range(len(P)):
        idx[S[q] >= tau] = q
    qi = np.where(idx == PSTAR_NONE, 0, idx).astype(np.int64)
    Ssel = np.take_along_axis(S, qi[None], axis=0)[0]
    psel = np.asarray(P, dtype=np.float64)[qi]
    root = np.where(Ssel > 0, np.power(np.where(Ssel > 0, Ssel, 1.0), 1.0 / psel), 0.0)
    z = rx[:, None] * ry[:, None] * root
    return {"z": z, "pstar_idx": idx, "S": S, "rx": rx, "ry": ry}
