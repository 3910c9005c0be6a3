"""Oracle: the top k values of x_i + y_j and their indices, FP64 on CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper: Serang, arXiv 1511.05690, Sec. 2.3 (algorithm E for x' times y',
and the index recovery that follows it).
  * The additive problem maps to (x, max) by x' = e^x, y' = e^y.  Scaled as
    in Sec. 2.1: x' = e^(x - max x), y' = e^(y - max y), every term in (0, 1].
  * For every p in the family, sigma^(p)[m] = sum over i + j = m of
    (x'_i y'_j)^p, the ordinary convolution of x'^p and y'^p (numpy's direct
    convolution here, the plain definition of the ring result; the paper
    computes it by FFT).
  * psi[m] is the estimate of the largest term of diagonal m from its norm
    sequence: the root sigma^(p*)^(1/p*) at the largest p with
    sigma^(p) >= tau (the same rule as the product and the max-convolution).
    Diagonals where no p is stable have no estimate (psi = 0, never popped
    while anything else is left).
  * NormQueue: k times, take the diagonal m* with the largest psi (the first
    one on ties), report it, subtract psi^p from every sigma^(p)[m*] and
    estimate psi[m*] again from what is left.
  * Values are reported in the additive space: max x + max y + log(psi).
  * Index recovery: a second run on y reversed gives, rank by rank, the
    anti-diagonal m2 = i + (n - 1 - j) of the same value; with m1 = i + j,
    i = (m1 + m2 - n + 1) / 2 and j = m1 - i (the pair is reported only when
    that is an integer pair inside the n x n grid).

The paired queue (xy_topk_paired) is the refinement that the Discussion
proposes: the two runs pop in lockstep, so the pair (i, j) of a rank is
known before the norms are updated; when that pair is accurate its exact
value x_i + y_j is reported and its scaled value v = x'_i y'_j, not the
estimate, is subtracted from both runs' norms.  Reading of "accurate" (the
paper leaves it open): (i, j) is an integer pair inside the grid that no
earlier rank reported (a reported pair is gone from both norms; the two runs
can meet in it again once their diagonals are popped again), and v is
at least the smallest maximum that the norm admits on each of the two
diagonals, psi len^(-1/p*) (a vector of len entries with p-norm psi has a
largest entry of at least psi len^(-1/p); len = number of grid pairs on the
diagonal; none when the diagonal has no stable p).  Otherwise the rank is
reported as by the plain queue (run 0's estimate, i = j = -1) and each run
subtracts its own estimate.
"""

import numpy as np

TAU_FFT = 1e-12


def exact_topk_xy(x, y, k):
    """The k largest x_i + y_j (brute force over all pairs), descending, with
    their indices (ties in the order of i, then j)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    s = (x[:, None] + y[None, :]).ravel()
    order = np.argsort(-s, kind="stable")[:k]
    return s[order], order // y.size, order % y.size


def _estimate(col, P, tau):
    """psi (scaled space) and the family index used, from one diagonal's
    sigma column; (0, -1) when no p is stable."""
    for q in range(len(P) - 1, -1, -1):
        if col[q] >= tau:
            return col[q] ** (1.0 / P[q]), q
    return 0.0, -1


def ring_results(x, y, P):
    """The ring results of Sec. 2.3 for one pair of lists: sigma (|P| x
    (n + m - 1)), sigma^(p) = x'^p * y'^p by direct convolution, with the
    scale-backs max x and max y."""
    P = [int(p) for p in P]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx, my = x.max(), y.max()
    xs = np.exp(x - mx)
    ys = np.exp(y - my)
    return np.stack([np.convolve(xs ** p, ys ** p) for p in P]), mx, my


def norm_queue(x, y, P, k, tau=TAU_FFT):
    """Algorithm E of Sec. 2.3 on one pair of lists (x and y may differ in
    length here).  Returns dict values (k, additive space), diag (k, m*),
    sigma (|P| x (n + m - 1), before any pop)."""
    sigma, mx, my = ring_results(x, y, P)
    return queue_pops(sigma, mx, my, P, k, tau)


def queue_pops(sigma, mx, my, P, k, tau=TAU_FFT):
    """The k pops of algorithm E (Sec. 2.3) from given ring results sigma
    (|P| x L) of lists whose maxima were mx and my: the same steps as
    norm_queue, on whatever ring results the caller holds (the tests feed
    it FFT-rounded ones to find how deep a pop sequence is insensitive to
    the ring results' rounding)."""
    P = [int(p) for p in P]
    sigma = np.asarray(sigma, dtype=np.float64)
    work = sigma.copy()
    L = work.shape[1]
    psi = np.zeros(L)
    for m in range(L):
        psi[m], _ = _estimate(work[:, m], P, tau)
    values = np.zeros(k)
    diag = np.zeros(k, dtype=np.int64)
    for r in range(k):
        m = int(np.argmax(psi))
        a = psi[m]
        values[r] = mx + my + (np.log(a) if a > 0 else -np.inf)
        diag[r] = m
        # psi may exceed 1 (the norm bounds the max from above): psi^p can
        # overflow to inf for large p, leaving -inf, which is not stable
        with np.errstate(over="ignore"):
            for q, p in enumerate(P):
                work[q, m] -= a ** p
        psi[m], _ = _estimate(work[:, m], P, tau)
    return {"values": values, "diag": diag, "sigma": sigma}


def xy_topk_estimate(x, y, P, k, tau=TAU_FFT):
    """Top k of x_i + y_j by the NormQueue with index recovery (x and y of
    the same length n).  Returns dict values, diag (i + j), anti
    (i + n - 1 - j, from the run on y reversed), i, j (-1 where the two runs
    do not give an integer pair in the grid)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    if y.size != n:
        raise ValueError("x and y must have the same length")
    a = norm_queue(x, y, P, k, tau)
    b = norm_queue(x, y[::-1], P, k, tau)
    s = a["diag"] + b["diag"] - (n - 1)
    i = np.where(s % 2 == 0, s // 2, -1)
    j = np.where(i >= 0, a["diag"] - i, -1)
    ok = (i >= 0) & (i < n) & (j >= 0) & (j < n)
    return {"values": a["values"], "diag": a["diag"], "anti": b["diag"],
            "i": np.where(ok, i, -1), "j": np.where(ok, j, -1)}


def _diag_len(m, n):
    """Number of pairs (i, j) of the n x n grid with i + j = m (the same
    count for an anti-diagonal of the run on y reversed)."""
    return min(m, 2 * n - 2 - m) + 1


def _min_admitted(a, q, m, n, P):
    """Smallest largest entry that a diagonal m with estimate a (root at
    p = P[q]) admits: a len^(-1/p).  A diagonal with no stable p (q < 0) has
    no estimate to judge a pair by: +inf, so no pair on it is accurate."""
    return a * _diag_len(m, n) ** (-1.0 / P[q]) if q >= 0 else np.inf


def xy_topk_paired(x, y, P, k, tau=TAU_FFT):
    """Top k of x_i + y_j by the paired NormQueue (Discussion): the runs on
    y and on y reversed pop together; an accurate pair (see the module
    docstring) is reported exactly and subtracted exactly from both.
    Returns dict values, diag (run 0), anti (run 1), i, j (-1 on ranks whose
    pair was not accurate), accepted (bool per rank)."""
    P = [int(p) for p in P]
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = x.size
    if y.size != n:
        raise ValueError("x and y must have the same length")
    mx, my = x.max(), y.max()
    xs = np.exp(x - mx)
    ys = np.exp(y - my)
    work = [np.stack([np.convolve(xs ** p, ys ** p) for p in P]),
            np.stack([np.convolve(xs ** p, ys[::-1] ** p) for p in P])]
    L = 2 * n - 1
    psi = [np.zeros(L), np.zeros(L)]
    pq = [np.full(L, -1), np.full(L, -1)]
    for t in range(2):
        for m in range(L):
            psi[t][m], pq[t][m] = _estimate(work[t][:, m], P, tau)
    out = {"values": np.zeros(k), "diag": np.zeros(k, dtype=np.int64), "anti": np.zeros(k, dtype=np.int64),
           "i": np.full(k, -1, dtype=np.int64), "j": np.full(k, -1, dtype=np.int64),
           "accepted": np.zeros(k, dtype=bool)}
    reported = set()
    for r in range(k):
        m1 = int(np.argmax(psi[0]))
        m2 = int(np.argmax(psi[1]))
        a = (psi[0][m1], psi[1][m2])
        out["diag"][r], out["anti"][r] = m1, m2
        ok = False
        s = m1 + m2 - (n - 1)
        if s % 2 == 0 and 0 <= s // 2 < n and 0 <= m1 - s // 2 < n:
            i, j = s // 2, m1 - s // 2
            v = np.exp((x[i] - mx) + (y[j] - my))
            ok = (i, j) not in reported
            for t, m in ((0, m1), (1, m2)):
                ok = ok and v >= _min_admitted(a[t], pq[t][m], m, n, P)
        if ok:
            out["values"][r] = x[i] + y[j]
            out["i"][r], out["j"][r] = i, j
            out["accepted"][r] = True
            reported.add((i, j))
            sub = (v, v)
        else:
            out["values"][r] = mx + my + (np.log(a[0]) if a[0] > 0 else -np.inf)
            sub = a
        with np.errstate(over="ignore"):
            for t, m in ((0, m1), (1, m2)):
                for q, p in enumerate(P):
                    work[t][q, m] -= sub[t] ** p
                psi[t][m], pq[t][m] = _estimate(work[t][:, m], P, tau)
    return out
