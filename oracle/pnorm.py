"""Oracle: exact (max, x) matrix product and its p-norm ring estimate, FP64 on CPU.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Paper: Serang, arXiv 1511.05690.
  * Alg. 2 (Sec. 2.2): the naive (x, max) product R_ij = max_k X_ik * Y_kj.
  * Alg. 3 (Sec. 2.2): the same loops with + in place of max (an ordinary
    matrix product); numpy's BLAS matmul stands in for it, which Sec. 2.1
    allows for any H that returns the same numbers as G.
  * Sec. 1 (max via the Chebyshev norm): max_k u_k = lim_p ||u||_p, and
    ||u||_p^p of u_k = A_ik B_kj is (A^p B^p)_ij because (ab)^p = a^p b^p
    (Sec. 2.1, distributivity argument).
  * Sec. 2.1, scaled call H'(I, p): inputs are divided by their maximum
    before the power so that the only numerical hazard left is underflow.
  * Sec. 1 and Alg. 5: the family P = {1, 2, 4, ...}; at every output index
    only the p whose ring result is >= tau count as stable, and the estimate
    is taken from that stable sequence.
  * Sec. 1, error bound: ||u||_inf <= ||u||_p <= len(u)^(1/p) ||u||_inf; and
    the optional division by len(u)^(1/p) that centres the error.

Readings where the paper is silent or garbled (each is also listed in the
design notes of the repository):
  R1  Scaling: the printed H' multiplies the ring result by one global max
      and never takes its 1/p root.  Read as: per-row max r_i of A and
      per-column max c_j of B; the estimate is r_i c_j S_p^(1/p).  The p-norm
      is positively homogeneous, so this is the same number with less
      underflow.
  R2  estimateMaxFromNormPowerSequence is the plain rule: the stable entry
      with the largest p, rooted: S_{p*}^(1/p*).
  R3  Stability is S_p >= tau (not >).
  R4  No stable p at all: use the smallest p of the family and mark the
      entry with index PSTAR_NONE (255).  If every term is 0 the estimate
      is exactly 0.
  R5  A zero row of A (zero column of B) has r = 0 (c = 0); its scaled row
      is 0 and its outputs are 0.  An empty inner dimension (k = 0) gives
      all-zero output with index PSTAR_NONE.
  R6  The r = 1 projection (Sec. 1, projecting the unique values of u onto
      one value alpha): the paper's form uses the evenly spaced norms p*/2
      and p*.  Read with the next smaller p of the family, p_lo, as the
      lower norm: model u as h copies of alpha, S_p = h alpha^p, so
      alpha = (S_{p*} / S_{p_lo})^(1/(p* - p_lo)); for a powers-of-two
      family p_lo = p*/2 and this is (S_{p*} / S_{p*/2})^(2/p*).  Where p*
      is the smallest p, no p is stable, or S_{p_lo} is 0, the plain root
      is used.
  R7  The r = 2 projection (Sec. 1, onto two values): the paper's 2r
      evenly spaced norms are read as q, 2q, 3q, 4q with 4q = p* (the
      largest stable p of the family P; the selection never picks one of
      the added norms 3q).  The estimate is the largest of the two
      projected values, i.e. of the positive roots x = alpha^q of the
      null-space polynomial.  Where p* is not a multiple of 4 with p*/4 and
      p*/2 in P, a norm is 0, the Hankel matrix is numerically of rank 1,
      or no root is real and positive, the r = 1 projection (R6) is used
      instead.
      Rank 1, from the rounding of the norms: each norm S_kq is a sum of K
      nonnegative terms whose powers come from p*-fold products, so its
      relative rounding is at most eps = (K + 4 p* + L) u (u = 2^-53;
      L = max_k |ln S_kq| covers the rounding of the logarithms that
      normalise the norms).  A relative perturbation eps of the Hankel
      matrix moves its null vector by about eps / rho (rho = sigma_2 /
      sigma_1) and the projected value alpha = x^(1/q) by about
      eps / (q rho).  The projection is used where that is at most
      delta = 2.5e-6, a quarter of the FP64 path's stated accuracy 1e-5,
      i.e. where rho > theta = eps / (q delta); below, rounding decides
      the root and the r = 1 projection (well conditioned: a ratio of two
      norms) is used.
  R8  Inner-index balancing (the Discussion's remark on scaling a problem
      into a bounded range; the paper gives no formula).  The product is
      unchanged when column k of A is multiplied by d_k > 0 and row k of B
      divided by it, since each term A_ik B_kj is; only the scales r_i, c_j
      and hence which p are stable change.  Read as: d_k = sqrt(b_k / a_k)
      with a_k = max_i A_ik and b_k = max_j B_kj (d_k = 1 where either is
      0), which makes the largest entry of column k of A D equal to the
      largest entry of row k of D^-1 B, and makes the balanced estimate
      independent of any inner-index rescaling of the inputs.  The
      estimate is then the plain one of (A D, D^-1 B).
"""

import numpy as np

PSTAR_NONE = 255


def _f64(x):
    return np.asarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# O-1: exact product (Alg. 2)
# --------------------------------------------------------------------------
def exact_maxtimes(A, B):
    """Alg. 2: R_ij = max_k A_ik * B_kj with R starting at 0 (the identity of
    max on nonnegative reals).  Batched over leading dimensions.

    The loop over k is kept (ascending, as in Alg. 2); i and j are
    vectorised.  max is exact, so the result does not depend on any order.
    """
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape[-2:]
    k2, n = B.shape[-2:]
    if k != k2:
        raise ValueError("inner dimensions differ")
    batch = np.broadcast_shapes(A.shape[:-2], B.shape[:-2])
    R = np.zeros(batch + (m, n))
    for kk in range(k):
        R = np.maximum(R, A[..., :, kk:kk + 1] * B[..., kk:kk + 1, :])
    return R


def exact_maxtimes_loops(A, B):
    """Alg. 2 written as its three nested loops in pure Python (tiny inputs
    only).  A second, independent formulation of exact_maxtimes."""
    A = _f64(A)
    B = _f64(B)
    m, k = A.shape
    n = B.shape[1]
    R = [[0.0] * n for _ in range(m)]
    for i in range(m):
        for j in range(n):
            for kk in range(k):
                R[i][j] = max(R[i][j], float(A[i, kk]) * float(B[kk, j]))
    return np.array(R, dtype=np.float64).reshape(m, n)


# --------------------------------------------------------------------------
# O-2 .. O-6: the p-norm estimate (Alg. 5 with the scaled call H')
# --------------------------------------------------------------------------
def scale_factors(A, B):
    """Reading R1 of Sec. 2.1's H': r_i = max_k A_ik, c_j = max_k B_kj."""
    A = _f64(A)
    B = _f64(B)
    r = np.max(A, axis=-1, initial=0.0)
    c = np.max(B, axis=-2, initial=0.0)
    return r, c


def _scaled(A, B):
    r, c = scale_factors(A, B)
    with np.errstate(divide="ignore", invalid="ignore"):
        Ap = np.where(r[..., :, None] > 0, A / r[..., :, None], 0.0)
        Bp = np.where(c[..., None, :] > 0, B / c[..., None, :], 0.0)
    return Ap, Bp, r, c


def norm_power_sequence(A, B, P):
    """First loop of Alg. 5: for every p in P, raise the scaled inputs to p
    and call the ring product (Alg. 3) on them.

    Returns S (len(P), ..., m, n) with S[q] = (A'^p) @ (B'^p), p = P[q],
    i.e. S[q]_ij = ||u||_p^p for u_k = A'_ik B'_kj; plus r and c.
    """
    A = _f64(A)
    B = _f64(B)
    Ap, Bp, r, c = _scaled(A, B)
    S = [np.power(Ap, p) @ np.power(Bp, p) for p in P]
    return np.stack(S), r, c


def select_pstar(S, tau):
    """Alg. 5, second loop, with readings R2-R4: the index q of the largest
    p whose ring result is >= tau; PSTAR_NONE where no p qualifies.
    P is ascending, so the last qualifying q seen is the largest p."""
    idx = np.full(S.shape[1:], PSTAR_NONE, dtype=np.uint8)
    for q in range(S.shape[0]):
        idx[S[q] >= tau] = q
    return idx


def _root(S, P, idx):
    """S_{p*}^(1/p*) per entry (the 1/p root of Sec. 1), with the smallest
    p of the family where idx is PSTAR_NONE (R4); 0 where S is 0."""
    P = np.asarray(P, dtype=np.int64)
    q = np.where(idx == PSTAR_NONE, 0, idx).astype(np.int64)
    Ssel = np.take_along_axis(S, q[None], axis=0)[0]
    psel = P[q].astype(np.float64)
    root = np.where(Ssel > 0, np.power(np.where(Ssel > 0, Ssel, 1.0), 1.0 / psel), 0.0)
    return root, psel, Ssel


def _project_r1(S, P, idx, root):
    """Reading R6 of the r = 1 projection (Sec. 1): per entry with stable
    index q > 0, alpha = (S_{P[q]} / S_{P[q-1]})^(1/(P[q] - P[q-1])); the
    plain root ``root`` elsewhere."""
    P = np.asarray(P, dtype=np.int64)
    q = idx.astype(np.int64)
    use = (idx != PSTAR_NONE) & (q > 0)
    qh = np.where(use, q, 0)
    ql = np.where(use, q - 1, 0)
    Sh = np.take_along_axis(S, qh[None], axis=0)[0]
    Sl = np.take_along_axis(S, ql[None], axis=0)[0]
    use &= Sl > 0
    expo = 1.0 / (P[qh] - P[ql]).astype(np.float64).clip(min=1)
    with np.errstate(divide="ignore", invalid="ignore"):
        alpha = np.power(np.where(use, Sh / np.where(use, Sl, 1.0), 1.0), expo)
    return np.where(use, alpha, root)


def r2_aux_powers(P):
    """The extra norms the r = 2 projection needs (Sec. 1: 2r evenly spaced
    norms q, 2q, 3q, 4q with 4q = p*): 3p/4 for every p of P with p/4 and
    p/2 in P, where 3p/4 is not in P itself.  Ascending."""
    Ps = set(int(p) for p in P)
    return sorted({3 * p // 4 for p in Ps if p % 4 == 0 and p // 4 in Ps and p // 2 in Ps} - Ps)


R2_DELTA = 2.5e-6
U64 = 2.0 ** -53


def r2_threshold(k, pstar, lmax):
    """Reading R7: the rank-1 threshold theta on sigma_2 / sigma_1 for inner
    length k, p* = 4q and L = max |ln S| of the four norms."""
    q = pstar // 4
    return (k + 4.0 * pstar + lmax) * U64 / (q * R2_DELTA)


def _project_r2(S, P, idx, fallback, S_aux, aux, k, info=None):
    """The r = 2 projection of Sec. 1 (reading R7): with p* = P[q] = 4t and
    the ring results S_t, S_2t, S_3t, S_4t, a null vector g of the Hankel
    matrix [[S_t, S_2t, S_3t], [S_2t, S_3t, S_4t]] (taken from the SVD) gives
    the polynomial g0 + g1 x + g2 x^2 whose roots are the projected values
    alpha^t; the estimate is the largest positive root to the power 1/t.
    The norms are first divided by c^k (c = (S_4t / S_t)^(1/3)), which only
    scales the roots by c.  Where the four norms are not all positive and
    available, the Hankel matrix has rank below 2 (sigma_2 <= 1e-8
    sigma_1: one distinct value, or so close to one that rounding in the
    norms, would decide the roots: sigma_2 / sigma_1 <= r2_threshold), or
    the roots are complex or not positive, ``fallback`` (the r = 1
    projection) is used.  k is the inner length of the product.  With a
    dict ``info``, per entry: rho (sigma_2 / sigma_1), theta, and alt, the
    value the other rank decision gives (the projected root where the
    threshold chose the fallback, the fallback where it chose the root;
    NaN where the decision had no alternative)."""
    P = [int(p) for p in P]
    pos = {p: ("P", i) for i, p in enumerate(P)}
    pos.update({p: ("A", i) for i, p in enumerate(aux)})
    out = np.array(fallback, dtype=np.float64, copy=True)
    shp = idx.shape
    flat_idx = idx.reshape(-1)
    flatS = S.reshape(S.shape[0], -1)
    flatA = S_aux.reshape(S_aux.shape[0], -1) if len(aux) else None
    flat_out = out.reshape(-1)
    fb = np.asarray(fallback, dtype=np.float64).reshape(-1)
    rho_a = np.full(flat_idx.size, np.nan)
    theta_a = np.full(flat_idx.size, np.nan)
    alt_a = np.full(flat_idx.size, np.nan)
    for e in range(flat_idx.size):
        q = int(flat_idx[e])
        if q == PSTAR_NONE:
            continue
        ps = P[q]
        if ps % 4:
            continue
        t = ps // 4
        need = [t, 2 * t, 3 * t, 4 * t]
        if any(p not in pos for p in need):
            continue
        vals = []
        for p in need:
            kind, i = pos[p]
            vals.append(flatS[i, e] if kind == "P" else flatA[i, e])
        Sk = np.array(vals, dtype=np.float64)
        if np.any(Sk <= 0):
            continue
        lS = np.log(Sk)
        logc = (lS[3] - lS[0]) / 3.0
        tk = np.exp(lS - np.arange(1, 5) * logc)
        H = np.array([[tk[0], tk[1], tk[2]], [tk[1], tk[2], tk[3]]])
        _, sv, Vh = np.linalg.svd(H)
        g0, g1, g2 = Vh[-1]
        if g2 == 0:
            continue
        disc = g1 * g1 - 4 * g2 * g0
        if disc < 0:
            continue
        roots = [(-g1 + np.sqrt(disc)) / (2 * g2), (-g1 - np.sqrt(disc)) / (2 * g2)]
        ymax = max(roots)
        if not ymax > 0:
            continue
        root_val = np.exp((np.log(ymax) + logc) / t)
        rho = sv[1] / sv[0]
        theta = r2_threshold(k, ps, np.abs(lS).max())
        rho_a[e], theta_a[e] = rho, theta
        if rho > theta:
            flat_out[e] = root_val
            alt_a[e] = fb[e]
        else:
            alt_a[e] = root_val
    if info is not None:
        info["rho"] = rho_a.reshape(shp)
        info["theta"] = theta_a.reshape(shp)
        info["alt"] = alt_a.reshape(shp)
    return out


def balance_factors(A, B):
    """Reading R8: d_k = sqrt(b_k / a_k), a_k = max_i A_ik (over the rows of
    A), b_k = max_j B_kj (over the columns of B); 1 where a_k or b_k is 0.
    Batched over leading dimensions: shape (..., k)."""
    A = _f64(A)
    B = _f64(B)
    a = np.max(A, axis=-2, initial=0.0)
    b = np.max(B, axis=-1, initial=0.0)
    ok = (a > 0) & (b > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(ok, np.sqrt(np.where(ok, b, 1.0) / np.where(ok, a, 1.0)), 1.0)


def balanced(A, B):
    """(A D, D^-1 B, d) with d from balance_factors (reading R8)."""
    A = _f64(A)
    B = _f64(B)
    d = balance_factors(A, B)
    return A * d[..., None, :], B / d[..., :, None], d


def pnorm_estimate(A, B, P, tau, norm_correct=False, projection=None, balance=False):
    """The p-norm estimate of the (max, x) product (Alg. 5, Sec. 2.1-2.2).

    C_ij = r_i c_j S_{p*}^(1/p*), p* = max{p in P : S_p[i, j] >= tau}.
    With norm_correct, C is divided by k^(1/p*) (Sec. 1, centred error).
    With projection="r1" the max is taken from the r = 1 projection of the
    norm sequence instead of the plain root (Sec. 1; reading R6).
    With balance, the estimate of the balanced pair (A D, D^-1 B) (reading
    R8); r and c are then those of the balanced pair, and d is returned.

    Returns a dict: C, pstar_idx (uint8, index into P, 255 = none stable),
    r, c, S (the whole norm power sequence), pstar (the p used per entry).
    """
    P = [int(p) for p in P]
    if any(p <= 0 for p in P) or any(P[i] >= P[i + 1] for i in range(len(P) - 1)):
        raise ValueError("P must be strictly ascending positive integers")
    if projection not in (None, "r1", "r2"):
        raise ValueError("projection must be None, 'r1' or 'r2'")
    if projection and norm_correct:
        raise ValueError("norm_correct applies to the plain root only")
    A = _f64(A)
    B = _f64(B)
    k = A.shape[-1]
    d = None
    if balance:
        A, B, d = balanced(A, B)
    S, r, c = norm_power_sequence(A, B, P)
    idx = select_pstar(S, tau)
    root, psel, _ = _root(S, P, idx)
    out_aux = {}
    if projection in ("r1", "r2"):
        root = _project_r1(S, P, idx, root)
    if projection == "r2":
        aux = r2_aux_powers(P)
        S_aux = norm_power_sequence(A, B, aux)[0] if aux else np.zeros((0,) + S.shape[1:])
        info = {}
        root = _project_r2(S, P, idx, root, S_aux, aux, k, info)
        rc = r[..., :, None] * c[..., None, :]
        out_aux = {"S_aux": S_aux, "aux": aux, "k": k, "r2_rho": info["rho"], "r2_theta": info["theta"],
                   "C_alt": rc * info["alt"]}
    C = r[..., :, None] * c[..., None, :] * root
    if norm_correct and k > 0:
        C = C / np.power(float(k), 1.0 / psel)
    out = {"C": C, "pstar_idx": idx, "pstar": psel, "r": r, "c": c, "S": S}
    if d is not None:
        out["d"] = d
    out.update(out_aux)
    return out


def pnorm_estimate_rows(A, B, P, tau, rows, norm_correct=False, projection=None, balance=False):
    """The estimate restricted to output rows ``rows``: row i of C depends
    only on row i of A (through r_i and A'_i) and on all of B, so this is
    pnorm_estimate(A[rows], B).  Balancing (R8) takes its factors from the
    whole of A and B first."""
    A = _f64(A)
    d = None
    if balance:
        A, B, d = balanced(A, B)
    out = pnorm_estimate(A[..., rows, :], B, P, tau, norm_correct=norm_correct, projection=projection)
    if d is not None:
        out["d"] = d
    return out


def pnorm_forward_fixed(A, B, P, pstar_idx, balance=False):
    """C_ij = (sum_k A_ik^p B_kj^p)^(1/p) with p = P[pstar_idx[i, j]] given
    per entry (PSTAR_NONE -> P[0]); the forward with p* frozen, for finite
    differences of the gradient.  With balance, formed from the balanced
    pair (reading R8; the same function, scaled so that it does not
    underflow where the inner index carries a scaling)."""
    if balance:
        A, B, _ = balanced(A, B)
    S, r, c = norm_power_sequence(A, B, P)
    root, _, _ = _root(S, P, np.asarray(pstar_idx, dtype=np.uint8))
    return r[..., :, None] * c[..., None, :] * root


# --------------------------------------------------------------------------
# O-10: analytic gradient with p* frozen
# --------------------------------------------------------------------------
def pnorm_grad(A, B, G, P, pstar_idx, balance=False):
    """Gradient of L = sum(G * C) for the estimate with p = p*_ij frozen per
    entry.  The paper only notes that the p-norm rings are continuous and
    differentiable (Sec. 4); the derivative follows from
    C_ij = (sum_k A_ik^p B_kj^p)^(1/p):
        dC_ij/dA_ik = C_ij^(1-p) A_ik^(p-1) B_kj^p
    Written with the scaled quantities A' = A/r, B' = B/c, C' = C/(r_i c_j)
    the powers of r and c cancel and nothing overflows:
        dL/dA_ik = sum_p A'_ik^(p-1) sum_{j: p*_ij = p} G_ij c_j C'_ij^(1-p) B'_kj^p
        dL/dB_kj = sum_p B'_kj^(p-1) sum_{i: p*_ij = p} A'_ik^p G_ij r_i C'_ij^(1-p)
    Entries whose S is 0 contribute nothing.
    With balance (reading R8) the same formula is evaluated on the balanced
    pair (A D, D^-1 B), whose scaled quantities stay in range where the
    inner index of the inputs carries a scaling, and taken back by the chain
    rule: dL/dA_ik = d_k dL/d(AD)_ik, dL/dB_kj = dL/d(D^-1 B)_kj / d_k.  The
    function C with p* frozen does not depend on d, so d is a constant here.
    """
    A = _f64(A)
    B = _f64(B)
    G = _f64(G)
    if balance:
        Ab, Bb, d = balanced(A, B)
        gA, gB = pnorm_grad(Ab, Bb, G, P, pstar_idx)
        return gA * d[..., None, :], gB / d[..., :, None]
    P = [int(p) for p in P]
    Ap, Bp, r, c = _scaled(A, B)
    idx = np.asarray(pstar_idx, dtype=np.uint8)
    q_used = np.where(idx == PSTAR_NONE, 0, idx)
    S = np.stack([np.power(Ap, p) @ np.power(Bp, p) for p in P])
    root, psel, Ssel = _root(S, P, idx)  # root = C'
    dA = np.zeros(np.broadcast_shapes(A.shape, G.shape[:-1] + (A.shape[-1],)))
    dB = np.zeros(np.broadcast_shapes(B.shape, G.shape[:-2] + B.shape[-2:]))
    for q, p in enumerate(P):
        mask = (q_used == q) & (root > 0)
        if not mask.any():
            continue
        with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
            w = np.where(mask, np.power(np.where(mask, root, 1.0), 1.0 - p), 0.0)
        GtA = G * c[..., None, :] * w
        GtB = G * r[..., :, None] * w
        Bpp = np.power(Bp, p)
        App = np.power(Ap, p)
        dA = dA + np.power(Ap, p - 1) * (GtA @ np.swapaxes(Bpp, -1, -2))
        dB = dB + np.power(Bp, p - 1) * (np.swapaxes(App, -1, -2) @ GtB)
    return dA, dB
