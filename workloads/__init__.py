"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method (no scaling, no powers, no
transform): it only draws matrices and graphs with numpy's PCG64
``default_rng(seed)``.  Both the oracle and the GPU path receive the same
arrays from here.

Workloads (the paper publishes no dataset; its APSP instances are random
dense graphs, Sec. 3 Table 1, so every input here is synthetic):

  uniform_product    A, B with i.i.d. entries in (0, 1]   (1 - U[0, 1))
  lognormal_product  A, B = exp(N(0, sigma^2)) clipped to (0, clip], FP32
  gradient_case      a batch of uniform products plus G ~ N(0, 1), FP32
  er_graph           directed Erdos-Renyi graph, U[0, wmax) weights, FP32,
                     +inf = no edge, diagonal 0
  rgg_graph          random geometric graph in the unit square, weight =
                     scale * Euclidean length, FP32, +inf = no edge
  dense_graph        complete digraph with U[lo, hi) weights (the shape of
                     the paper's Table 1 instances)
  crossed_product    log-normal A, B whose inner index halves are scaled by a
                     large and a small factor in opposite order (every term
                     is about big * small, the row and column maxima about
                     big): scales beyond FP32 with moderate products
  wide_scale_product FP64 log-normal A, B with rows of A and columns of B
                     scaled by 10^(+-decades)
  maxconv_vectors    b pairs of nonnegative vectors (x of length n, y of
                     length m) for the max-convolution of Sec. 1: "uniform"
                     (1 - U[0, 1)), "lognormal" (exp(N(0, 2^2))), "sparse"
                     (uniform with 70 % zeros), "distribution" (Dirichlet(1)
                     rows: probability vectors, the operands of max-product
                     inference)
"""

import numpy as np

SEED_BASE = 1000


def rng_for(seed):
    return np.random.default_rng(seed)


def uniform_product(m, k, n, seed, dtype=np.float64, batch=None):
    rng = rng_for(seed)
    sa = (m, k) if batch is None else (batch, m, k)
    sb = (k, n) if batch is None else (batch, k, n)
    A = (1.0 - rng.random(sa)).astype(dtype)
    B = (1.0 - rng.random(sb)).astype(dtype)
    return A, B


def lognormal_product(m, k, n, seed, sigma=2.0, clip=1e6, dtype=np.float32):
    rng = rng_for(seed)
    A = np.minimum(np.exp(rng.normal(0.0, sigma, size=(m, k))), clip).astype(dtype)
    B = np.minimum(np.exp(rng.normal(0.0, sigma, size=(k, n))), clip).astype(dtype)
    return A, B


def gradient_case(batch, m, k, n, seed, dtype=np.float32):
    rng = rng_for(seed)
    A = (1.0 - rng.random((batch, m, k))).astype(dtype)
    B = (1.0 - rng.random((batch, k, n))).astype(dtype)
    G = rng.standard_normal((batch, m, n)).astype(dtype)
    return A, B, G


def er_graph(n, prob, wmax, seed):
    rng = rng_for(seed)
    edge = rng.random((n, n)) < prob
    w = rng.uniform(0.0, wmax, size=(n, n))
    W = np.where(edge, w, np.inf).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


def rgg_graph(n, radius, scale, seed):
    from scipy.spatial import cKDTree

    rng = rng_for(seed)
    pts = rng.random((n, 2))
    pairs = cKDTree(pts).query_pairs(radius, output_type="ndarray")
    W = np.full((n, n), np.inf, dtype=np.float32)
    if len(pairs):
        i, j = pairs[:, 0], pairs[:, 1]
        d = (scale * np.sqrt(((pts[i] - pts[j]) ** 2).sum(axis=1))).astype(np.float32)
        W[i, j] = d
        W[j, i] = d
    np.fill_diagonal(W, 0.0)
    return W


def dense_graph(n, lo, hi, seed):
    rng = rng_for(seed)
    W = rng.uniform(lo, hi, size=(n, n)).astype(np.float32)
    np.fill_diagonal(W, 0.0)
    return W


# The five workloads of the benchmark configuration list, by number.
#   1  256^2 uniform FP64 product, P = {1..64}, FP64 path
#   2  ER APSP n=2048, p=0.05, U[0,10) weights, s=1, 11 squarings, FP64 path
#   3  8192^2 log-normal FP32 product, P = {1..128}, BF16-split and FP64 paths
#   4  64 x 512^3 uniform FP32 products with G ~ N(0,1), fixed p=16 and
#      P = {1..64}, BF16-split forward + backward
#   5  RGG APSP n=16384, radius 0.02, weight 100 x length, s=0.35,
#      14 squarings, P = {1..128}, BF16-split path
def maxconv_vectors(b, n, m, seed, kind="uniform", dtype=np.float64):
    rng = rng_for(seed)

    def draw(length):
        if kind == "uniform":
            v = 1.0 - rng.random((b, length))
        elif kind == "lognormal":
            v = np.exp(rng.normal(0.0, 2.0, (b, length)))
        elif kind == "sparse":
            v = (1.0 - rng.random((b, length))) * (rng.random((b, length)) >= 0.7)
        elif kind == "distribution":
            v = rng.dirichlet(np.ones(length), size=b) if length else np.zeros((b, 0))
        else:
            raise ValueError(kind)
        return v.astype(dtype)

    return draw(n), draw(m)


def pfamily(pmax):
    p, out = 1, []
    while p <= pmax:
        out.append(p)
        p *= 2
    return out


def config(i):
    seed = SEED_BASE + i
    if i == 1:
        A, B = uniform_product(256, 256, 256, seed)
        return {"A": A, "B": B, "P": pfamily(64), "path": "fp64"}
    if i == 2:
        return {"W": er_graph(2048, 0.05, 10.0, seed), "s": 1.0, "T": 11,
                "P": pfamily(512), "path": "fp64"}
    if i == 3:
        A, B = lognormal_product(8192, 8192, 8192, seed)
        return {"A": A, "B": B, "P": pfamily(128), "path": "bf16"}
    if i == 4:
        A, B, G = gradient_case(64, 512, 512, 512, seed)
        return {"A": A, "B": B, "G": G, "P": pfamily(64), "P_fixed": [16], "path": "bf16"}
    if i == 5:
        return {"W": rgg_graph(16384, 0.02, 100.0, seed), "s": 0.35, "T": 14,
                "P": pfamily(128), "path": "bf16"}
    raise ValueError(i)


def crossed_product(m, k, n, seed, big, small, dtype):
    """A's first half of the inner index is `big`, its second `small`; B the
    other way round.  Every term is about big * small, while r_i c_j is
    about big^2."""
    rng = np.random.default_rng(seed)
    h = k // 2
    A = np.exp(rng.normal(0.0, 1.0, (m, k)))
    B = np.exp(rng.normal(0.0, 1.0, (k, n)))
    A[:, :h] *= big
    A[:, h:] *= small
    B[:h] *= small
    B[h:] *= big
    return A.astype(dtype), B.astype(dtype)


def wide_scale_product(m, k, n, seed, decades):
    """FP64 log-normal A, B with row i of A scaled by 10^(+-decades) and
    column j of B by 10^(+-decades), signs at random."""
    rng = np.random.default_rng(seed)
    A = np.minimum(np.exp(rng.normal(0.0, 1.5, (m, k))), 1e6)
    B = np.minimum(np.exp(rng.normal(0.0, 1.5, (k, n))), 1e6)
    A *= (10.0 ** (decades * rng.choice([-1.0, 1.0], m)))[:, None]
    B *= (10.0 ** (decades * rng.choice([-1.0, 1.0], n)))[None, :]
    return A, B
