"""Oracle: all-pairs shortest paths through the (x, max) semiring, FP64 on CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Serang, arXiv 1511.05690, Sec. 2.2.
  * Nonnegative weights map to (x, max) by W' = exp(-W): sums of weights
    become products and min becomes max; distances come back as -log.
    Reading: a scale s > 0 is allowed, W' = exp(-s W) and d = -log(E) / s,
    which keeps long paths inside the floating-point range (the paper's
    discussion of long paths, Sec. 4).  s = 1 is the paper's transform.
  * A missing edge (+inf weight) maps to 0; a vertex reaches itself at
    distance 0, so the diagonal maps to 1.
  * The distance matrix is reached by log2(n) products on the semiring
    (Sec. 1, the A^n recursion; Sec. 2.2).  Reading: with the diagonal held
    at 1, T = ceil(log2 n) squarings X <- X (x) X cover every path of up to
    2^T >= n - 1 hops.
  * Reading for the estimate: after every squaring the diagonal is set back
    to 1 and every entry is clamped to <= 1 (exact values never exceed 1 for
    nonnegative weights; without the pin the estimate's diagonal, which is
    >= 1, would compound).
  * Floyd-Warshall is the exact comparison the paper uses (Sec. 3, Table 1);
    Dijkstra gives exact rows from sampled sources.
"""

import heapq
import math

import numpy as np

from .pnorm import exact_maxtimes, pnorm_estimate


def default_squarings(n):
    """T = ceil(log2 n) squarings (0 for n <= 1)."""
    return 0 if n <= 1 else int(math.ceil(math.log2(n)))


def to_maxtimes(W, s=1.0):
    """Sec. 2.2: W' = exp(-s W); +inf (no edge) -> 0; diagonal -> 1."""
    W = np.asarray(W, dtype=np.float64)
    X = np.exp(-s * W)
    n = W.shape[-1]
    X[..., np.arange(n), np.arange(n)] = 1.0
    return X


def to_distances(X, s=1.0):
    """Sec. 2.2 inverse transform: d = -log(E) / s; E = 0 -> +inf."""
    X = np.asarray(X, dtype=np.float64)
    with np.errstate(divide="ignore"):
        D = -np.log(X) / s + 0.0
    return D


def apsp_by_squaring(W, s, T, product):
    """X_0 = exp(-s W); T times: X <- product(X, X), X_ii <- 1, X <- min(X, 1);
    D = -log(X) / s.  Returns (D, X)."""
    X = to_maxtimes(W, s)
    n = X.shape[-1]
    if T is None:
        T = default_squarings(n)
    for _ in range(T):
        X = product(X, X)
        X[..., np.arange(n), np.arange(n)] = 1.0
        X = np.minimum(X, 1.0)
    return to_distances(X, s), X


def apsp_exact_squaring(W, s=1.0, T=None):
    """The same squaring loop with the exact product of Alg. 2 (Alg. 1 after the
    transform).  Equals Floyd-Warshall when T >= ceil(log2 n)."""
    return apsp_by_squaring(W, s, T, exact_maxtimes)


def apsp_estimate(W, s, P, tau, T=None, projection=None):
    """APSP estimate: the repeated squaring with the p-norm product (Alg. 5) at each
    squaring (projection "r1": the r = 1 projection of Sec. 1 in place of
    the plain root).  Returns dict D, X, pstar_idx_last (p* index of the
    last squaring)."""
    last = {}

    def product(X, Y):
        out = pnorm_estimate(X, Y, P, tau, projection=projection)
        last["idx"] = out["pstar_idx"]
        return out["C"]

    D, X = apsp_by_squaring(W, s, T, product)
    return {"D": D, "X": X, "pstar_idx_last": last.get("idx")}


def floyd_warshall(W):
    """Exact APSP by Floyd-Warshall in FP64: D = W, D_ii = 0, then for every
    intermediate vertex k: D <- min(D, D[:, k] + D[k, :])."""
    D = np.array(W, dtype=np.float64, copy=True)
    n = D.shape[0]
    D[np.arange(n), np.arange(n)] = 0.0
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    return D


def dijkstra(W, sources):
    """Exact single-source distances from each vertex in ``sources`` by
    Dijkstra's algorithm with a binary heap; W dense, +inf = no edge.
    Returns an array (len(sources), n) in FP64."""
    W = np.asarray(W)
    n = W.shape[0]
    off = ~np.eye(n, dtype=bool)
    rows, cols = np.nonzero(np.isfinite(W) & off)
    wts = W[rows, cols].astype(np.float64)
    start = np.searchsorted(rows, np.arange(n + 1))
    out = np.full((len(sources), n), np.inf)
    for si, src in enumerate(sources):
        dist = out[si]
        dist[src] = 0.0
        heap = [(0.0, int(src))]
        done = np.zeros(n, dtype=bool)
        while heap:
            d, u = heapq.heappop(heap)
            if done[u]:
                continue
            done[u] = True
            for e in range(start[u], start[u + 1]):
                v = cols[e]
                nd = d + wts[e]
                if nd < dist[v]:
                    dist[v] = nd
                    heapq.heappush(heap, (nd, int(v)))
    return out


def affine_fit(D_est, sources, exact_rows):
    """Sec. 4: an affine model between a few exact distances and the
    estimated ones.  Least squares d_exact = a d_est + b over the pairs
    (sources[q], v), v != sources[q], where both distances are finite:
    a = sum (x - mean x)(y - mean y) / sum (x - mean x)^2, b = mean y -
    a mean x.  Readings (the paper gives no formula): ordinary least squares
    on distances; no pairs -> (1, 0); all x equal -> a = 1.  Returns (a, b)."""
    D_est = np.asarray(D_est, dtype=np.float64)
    exact_rows = np.asarray(exact_rows, dtype=np.float64)
    xs, ys = [], []
    for q, s in enumerate(sources):
        x = D_est[s].copy()
        y = exact_rows[q].copy()
        keep = np.isfinite(x) & np.isfinite(y)
        keep[s] = False
        xs.append(x[keep])
        ys.append(y[keep])
    x = np.concatenate(xs) if xs else np.zeros(0)
    y = np.concatenate(ys) if ys else np.zeros(0)
    if x.size == 0:
        return 1.0, 0.0
    mx, my = x.mean(), y.mean()
    sxx = np.sum((x - mx) ** 2)
    a = np.sum((x - mx) * (y - my)) / sxx if sxx > 0 else 1.0
    return float(a), float(my - a * mx)


def affine_apply(D, a, b):
    """D <- max(0, a D + b) on every finite off-diagonal entry (distances are
    nonnegative; +inf and the zero diagonal stay)."""
    D = np.array(D, dtype=np.float64, copy=True)
    n = D.shape[0]
    m = np.isfinite(D) & ~np.eye(n, dtype=bool)
    D[m] = np.maximum(0.0, a * D[m] + b)
    return D
