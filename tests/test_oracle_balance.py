"""Pins of the oracle's inner-index balancing (reading R8 of oracle/pnorm.py:
the Discussion's remark on scaling a problem into a bounded range).

The mathematics fixes: each term A_ik B_kj, hence the exact (max, x) product
(Alg. 2) and every p-norm of the terms, is unchanged by A -> A D,
B -> D^-1 B; the norm bound exact <= C <= k^(1/p*) exact (Sec. 1) still
holds; the chosen d makes the largest entry of column k of A D equal to the
largest entry of row k of D^-1 B, so the balanced estimate does not depend
on any rescaling of the inner index, and balancing twice changes nothing.
A two-term case has a closed form in which balancing lifts p* from 1 to
the largest p."""

import math

import numpy as np

import oracle
from workloads import lognormal_product

P128 = [1, 2, 4, 8, 16, 32, 64, 128]
TAU = 1e-30


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _inner_scaled(seed, m=40, k=50, n=30, decades=8):
    rng = np.random.default_rng(seed)
    U = 1.0 - rng.random((m, k))
    V = 1.0 - rng.random((k, n))
    s = 10.0 ** rng.uniform(-decades, decades, k)
    return U, V, s


def test_two_term_closed_form():
    """A = [1, 1e-20], B = [1e-20; 1].  Unbalanced: r = c = 1, both terms are
    1e-20, S_p = 2e-20p, so p* = 1 at tau = 1e-30 and C = 2e-20 (twice the
    maximum).  Balanced: a = [1, 1e-20], b = [1e-20, 1], d = [1e-10, 1e10];
    A D = [1e-10, 1e-10], D^-1 B = [1e-10; 1e-10], r = c = 1e-10, the scaled
    terms are both 1, S_p = 2 for every p, p* = 128 and
    C = 1e-20 2^(1/128)."""
    A = np.array([[1.0, 1e-20]])
    B = np.array([[1e-20], [1.0]])
    plain = oracle.pnorm_estimate(A, B, P128, TAU)
    assert plain["pstar_idx"][0, 0] == 0
    assert math.isclose(plain["C"][0, 0], 2e-20, rel_tol=1e-15)
    bal = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
    np.testing.assert_allclose(bal["d"], [1e-10, 1e10], rtol=1e-15)
    assert bal["pstar_idx"][0, 0] == 7
    assert math.isclose(bal["C"][0, 0], 1e-20 * 2.0 ** (1.0 / 128), rel_tol=1e-14)
    # the scaled terms are 1 to a few ulps; the p-th power grows that p-fold
    np.testing.assert_allclose(bal["S"][:, 0, 0], 2.0, rtol=1e-13)


def test_balanced_maxima_are_equal_per_inner_index():
    A, B = lognormal_product(37, 53, 29, seed=1)
    A = np.stack([A, A[::-1] * 7.0]).astype(np.float64)
    B = np.stack([B, B[:, ::-1] / 3.0]).astype(np.float64)
    A[0, :, 5] = 0.0   # a zero column of A
    B[1, 9, :] = 0.0   # a zero row of B
    Ab, Bb, d = oracle.balanced(A, B)
    assert d.shape == (2, 53)
    assert d[0, 5] == 1.0 and d[1, 9] == 1.0
    ca = Ab.max(axis=-2)
    rb = Bb.max(axis=-1)
    ok = (A.max(axis=-2) > 0) & (B.max(axis=-1) > 0)
    assert _rel(ca[ok], rb[ok]).max() <= 1e-15
    # the geometric mean of the two maxima
    gm = np.sqrt(A.max(axis=-2) * B.max(axis=-1))
    assert _rel(ca[ok], gm[ok]).max() <= 1e-15


def test_exact_product_and_terms_unchanged():
    A, B = lognormal_product(30, 41, 25, seed=2)
    Ab, Bb, _ = oracle.balanced(A, B)
    E = oracle.exact_maxtimes(A, B)
    assert _rel(oracle.exact_maxtimes(Ab, Bb), E).max() <= 4e-16
    # every p-norm power of the terms is unchanged (before the scaling by r, c)
    for p in (1, 3, 8):
        s0 = np.power(A.astype(np.float64), p) @ np.power(B.astype(np.float64), p)
        s1 = np.power(Ab, p) @ np.power(Bb, p)
        assert _rel(s1, s0).max() <= 1e-13


def test_norm_bound_holds_balanced():
    for seed, (m, k, n) in enumerate([(20, 1, 15), (33, 64, 17), (50, 300, 40)]):
        A, B = lognormal_product(m, k, n, seed=10 + seed)
        ref = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
        E = oracle.exact_maxtimes(A, B)
        stable = ref["pstar_idx"] != oracle.PSTAR_NONE
        C = ref["C"]
        assert (C[stable] >= E[stable] * (1 - 1e-12)).all()
        bound = E * np.power(float(k), 1.0 / ref["pstar"])
        assert (C[stable] <= bound[stable] * (1 + 1e-12)).all()
        if k == 1:
            assert _rel(C, E).max() <= 1e-14  # one term: the norm is the term


def test_invariant_under_inner_rescaling():
    """The balanced estimate of (A E, E^-1 B) is that of (A, B) for any
    positive diagonal E: the balancing undoes E."""
    A, B = lognormal_product(45, 60, 35, seed=3)
    A = A.astype(np.float64)
    B = B.astype(np.float64)
    e = 10.0 ** np.random.default_rng(4).uniform(-20, 20, 60)
    r0 = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
    r1 = oracle.pnorm_estimate(A * e[None, :], B / e[:, None], P128, TAU, balance=True)
    np.testing.assert_array_equal(r1["pstar_idx"], r0["pstar_idx"])
    assert _rel(r1["C"], r0["C"]).max() <= 1e-12
    assert _rel(r1["d"] * e, r0["d"]).max() <= 1e-15


def test_pstar_rises_on_inner_scaled_inputs():
    """Inputs U diag(s), diag(s)^-1 V with s over 16 decades: unbalanced, r_i
    and c_j are set by different inner indices and the scaled terms are
    tiny, so p* is small and the estimate is far off; balanced, the estimate
    is that of the balanced (U, V), with a large p* and a small error."""
    U, V, s = _inner_scaled(5)
    A, B = U * s[None, :], V / s[:, None]
    E = oracle.exact_maxtimes(A, B)
    plain = oracle.pnorm_estimate(A, B, P128, TAU)
    bal = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
    ref_uv = oracle.pnorm_estimate(U, V, P128, TAU, balance=True)
    np.testing.assert_array_equal(bal["pstar_idx"], ref_uv["pstar_idx"])
    assert _rel(bal["C"], ref_uv["C"]).max() <= 1e-12
    p_plain = np.where(plain["pstar_idx"] == oracle.PSTAR_NONE, 0, plain["pstar"])
    assert bal["pstar"].min() > p_plain.max()
    assert _rel(bal["C"], E).max() < 0.1 < _rel(plain["C"], E).max()


def test_balancing_twice_changes_nothing():
    A, B = lognormal_product(25, 35, 20, seed=6)
    Ab, Bb, _ = oracle.balanced(A, B)
    d2 = oracle.balance_factors(Ab, Bb)
    assert np.abs(d2 - 1.0).max() <= 4e-16


def test_already_balanced_inputs_unchanged():
    """Every column of A and row of B with maximum 1: d = 1 exactly and the
    balanced estimate is the plain one bit for bit."""
    rng = np.random.default_rng(7)
    A = 1.0 - rng.random((20, 30))
    B = 1.0 - rng.random((30, 15))
    A[rng.integers(0, 20, 30), np.arange(30)] = 1.0
    B[np.arange(30), rng.integers(0, 15, 30)] = 1.0
    assert (oracle.balance_factors(A, B) == 1.0).all()
    r0 = oracle.pnorm_estimate(A, B, P128, TAU)
    r1 = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
    np.testing.assert_array_equal(r1["C"], r0["C"])


def test_rows_take_the_factors_from_the_whole_inputs():
    A, B = lognormal_product(60, 40, 30, seed=8)
    rows = np.array([3, 17, 59])
    full = oracle.pnorm_estimate(A, B, P128, TAU, balance=True)
    part = oracle.pnorm_estimate_rows(A, B, P128, TAU, rows, balance=True)
    np.testing.assert_array_equal(part["C"], full["C"][rows])
    np.testing.assert_array_equal(part["d"], full["d"])


def _fd_directional(A, B, G, P, idx, dirA, dirB, h):
    """Central difference of L = sum(G C) along (dirA, dirB), p* frozen, on
    the balanced forward (the factors are recomputed at each point; C with
    p* frozen does not depend on them)."""
    lp = (G * oracle.pnorm_forward_fixed(A + h * dirA, B + h * dirB, P, idx, balance=True)).sum()
    lm = (G * oracle.pnorm_forward_fixed(A - h * dirA, B - h * dirB, P, idx, balance=True)).sum()
    return (lp - lm) / (2 * h)


def test_balanced_gradient_equals_plain_where_both_are_in_range():
    """On uniform inputs (no inner scaling) both forms are accurate: the
    balanced gradient is the plain one to rounding."""
    rng = np.random.default_rng(90)
    A = 1.0 - rng.random((12, 17))
    B = 1.0 - rng.random((17, 9))
    G = rng.standard_normal((12, 9))
    P = [1, 2, 4, 8, 16, 32, 64]
    idx = oracle.pnorm_estimate(A, B, P, 1e-290, balance=True)["pstar_idx"]
    g0 = oracle.pnorm_grad(A, B, G, P, idx)
    g1 = oracle.pnorm_grad(A, B, G, P, idx, balance=True)
    for a, b in zip(g1, g0):
        assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_balanced_gradient_finite_differences_on_inner_scaled_inputs():
    """Inner-scaled inputs (6 decades) at p* = 64: the plain scaled form
    underflows (C' ~ 1e-6, C'^63 below FP64), the balanced one matches
    central differences (h relative to each coordinate's scale) and Euler's
    identity."""
    U, V, s = _inner_scaled(91, m=10, k=14, n=8, decades=3)
    A, B = U * s[None, :], V / s[:, None]
    rng = np.random.default_rng(92)
    G = rng.standard_normal((10, 8))
    P = [1, 2, 4, 8, 16, 32, 64]
    ref = oracle.pnorm_estimate(A, B, P, 1e-290, balance=True)
    idx = ref["pstar_idx"]
    assert (idx == 6).all()
    gA, gB = oracle.pnorm_grad(A, B, G, P, idx, balance=True)
    assert np.isfinite(gA).all() and np.isfinite(gB).all() and np.abs(gA).max() > 0
    for t in range(6):
        dA = rng.standard_normal(A.shape) * A
        dB = rng.standard_normal(B.shape) * B
        fd = _fd_directional(A, B, G, P, idx, dA, dB, 1e-6)
        an = (gA * dA).sum() + (gB * dB).sum()
        assert abs(fd - an) <= 1e-6 * (abs(an) + np.abs(G * ref["C"]).sum())
    GC = G * ref["C"]
    np.testing.assert_allclose((A * gA).sum(1), GC.sum(1), rtol=1e-10, atol=1e-12 * np.abs(GC).sum())
    np.testing.assert_allclose((B * gB).sum(0), GC.sum(0), rtol=1e-10, atol=1e-12 * np.abs(GC).sum())
