"""Pins of the oracle's r = 1 projection (Sec. 1: the norm sequence projected
onto one unique value; reading R6 of oracle/pnorm.py).  Each pin comes from
the paper's analysis or from the mathematics, not from the oracle's formula:

* tied top terms: the projection is exact (h copies of one value are
  recovered exactly), where the plain root is h^(1/p*) too large;
* the paper's worst case: v = (1, lam, ..., lam) with lam = 1/(sqrt(k) + 1)
  attains the stated minimum ratio 2 (sqrt(k) - 1) / (k - 1) of
  ||v||_2^2 / ||v||_1, so the estimate is exactly that ratio^(2/p*) times the
  max;
* on random inputs exact * ratio^(2/p*) <= C <= exact, and C <= plain;
* positive row / column scaling commutes with the estimate;
* APSP on a 2-node chain: the two tied terms (k = i and k = j) no longer
  bias the distance, which stays exactly w.
"""

import numpy as np
import pytest

import oracle
from oracle.apsp import apsp_estimate

TAU = 1e-290
P = [1, 2, 4, 8, 16, 32, 64]


def worst_ratio(k):
    return 2.0 * (np.sqrt(k) - 1.0) / (k - 1.0)


def test_tied_top_terms_exact():
    rng = np.random.default_rng(11)
    m, k, n, h = 6, 40, 5, 4
    A = np.zeros((m, k))
    B = np.zeros((k, n))
    for i in range(m):
        A[i, rng.choice(k, h, replace=False)] = 1.0
    # every column of B is 1 on the union of the rows' supports, so each
    # entry has h tied unit terms and zeros
    B[np.any(A > 0, axis=0), :] = 1.0
    A *= rng.uniform(0.5, 3.0, (m, 1))
    B *= rng.uniform(0.5, 3.0, (1, n))
    E = oracle.exact_maxtimes(A, B)
    out = oracle.pnorm_estimate(A, B, P, TAU, projection="r1")
    np.testing.assert_allclose(out["C"], E, rtol=1e-13)
    plain = oracle.pnorm_estimate(A, B, P, TAU)
    np.testing.assert_allclose(plain["C"], E * h ** (1.0 / 64), rtol=1e-13)


@pytest.mark.parametrize("k", [2, 9, 100, 1000])
@pytest.mark.parametrize("p", [2, 16, 64])
def test_paper_worst_case_attained(k, p):
    """u = v * M with v^(p/2) = (1, lam, ..., lam), lam = 1/(sqrt(k)+1):
    the r = 1 estimate is M * (2 (sqrt(k)-1)/(k-1))^(2/p) (Sec. 1)."""
    lam = 1.0 / (np.sqrt(k) + 1.0)
    v = np.full(k, lam ** (2.0 / p))
    v[0] = 1.0
    M = 3.5
    A = (v * M)[None, :]
    B = np.ones((k, 1))
    out = oracle.pnorm_estimate(A, B, [p // 2, p], TAU, projection="r1")
    assert out["pstar"][0, 0] == p
    np.testing.assert_allclose(out["C"][0, 0], M * worst_ratio(k) ** (2.0 / p), rtol=1e-12)


@pytest.mark.parametrize("lam", [0.05, 0.4, 0.9])
@pytest.mark.parametrize("k", [2, 7])
def test_two_value_ratio(lam, k):
    """Sec. 1: with w = (u / max)^(p*/2) = (1, lam, ..., lam) the r = 1
    estimate is max * ((1 + (k-1) lam^2) / (1 + (k-1) lam))^(2/p*); over
    the family {1, ..., 64} every entry here is stable at p* = 64, whose
    evenly spaced lower norm is 32."""
    p = 64
    u = np.full(k, lam ** (2.0 / p))
    u[0] = 1.0
    M = 0.75
    out = oracle.pnorm_estimate((u * M)[None, :], np.ones((k, 1)), P, TAU, projection="r1")
    assert out["pstar"][0, 0] == p
    ratio = (1 + (k - 1) * lam ** 2) / (1 + (k - 1) * lam)
    np.testing.assert_allclose(out["C"][0, 0], M * ratio ** (2.0 / p), rtol=1e-12)


def test_random_bounds_and_below_plain():
    rng = np.random.default_rng(12)
    for trial in range(4):
        m, k, n = 30, 200, 25
        A = rng.random((m, k)) ** (1 + 3 * trial)
        B = rng.random((k, n))
        E = oracle.exact_maxtimes(A, B)
        r1 = oracle.pnorm_estimate(A, B, P, TAU, projection="r1")
        plain = oracle.pnorm_estimate(A, B, P, TAU)
        ps = r1["pstar"]
        lo = E * worst_ratio(k) ** (2.0 / ps)
        assert np.all(r1["C"] <= E * (1 + 1e-12))
        assert np.all(r1["C"] >= lo * (1 - 1e-12))
        assert np.all(r1["C"] <= plain["C"] * (1 + 1e-12))
        assert np.array_equal(r1["pstar_idx"], plain["pstar_idx"])


def test_homogeneity():
    rng = np.random.default_rng(13)
    A = rng.random((12, 50))
    B = rng.random((50, 9))
    d1 = rng.uniform(0.1, 10, 12)
    d2 = rng.uniform(0.1, 10, 9)
    a = oracle.pnorm_estimate(A, B, P, TAU, projection="r1")
    b = oracle.pnorm_estimate(d1[:, None] * A, B * d2[None, :], P, TAU, projection="r1")
    np.testing.assert_allclose(b["C"], d1[:, None] * a["C"] * d2[None, :], rtol=1e-12)
    assert np.array_equal(a["pstar_idx"], b["pstar_idx"])


def test_smallest_p_falls_back_to_plain():
    """p* at the smallest p has no lower norm: the plain root is used."""
    A = np.array([[1.0, 1e-200]])
    B = np.array([[1e-200], [1.0]])
    # S_1 = 2e-200 (stable), S_2 = 2e-400 = 0 (not stable) -> p* = 1
    r1 = oracle.pnorm_estimate(A, B, [1, 2], TAU, projection="r1")
    plain = oracle.pnorm_estimate(A, B, [1, 2], TAU)
    assert r1["pstar_idx"][0, 0] == 0
    assert r1["C"][0, 0] == plain["C"][0, 0]


@pytest.mark.parametrize("w", [0.5, 2.0, 7.25])
def test_apsp_chain_unbiased(w):
    """W = [[0, w], [inf, 0]]: after every squaring X_01 has the two tied
    terms X_00 X_01 = X_01 X_11 = e^{-s w}; the r = 1 estimate keeps it, so
    d_01 = w exactly, while the plain root shrinks it by ln 2 / (s p*) per
    squaring (Sec. 2.2)."""
    W = np.array([[0.0, w], [np.inf, 0.0]])
    out = apsp_estimate(W, 1.0, [1, 2, 4, 8, 16, 32, 64, 128, 256, 512], TAU, T=3, projection="r1")
    np.testing.assert_allclose(out["D"][0, 1], w, rtol=1e-12)
    assert np.isinf(out["D"][1, 0]) and out["D"][0, 0] == 0 and out["D"][1, 1] == 0
    plain = apsp_estimate(W, 1.0, [1, 2, 4, 8, 16, 32, 64, 128, 256, 512], TAU, T=3)
    assert plain["D"][0, 1] < w - 1e-4


def test_rejects_bad_projection():
    with pytest.raises(ValueError):
        oracle.pnorm_estimate(np.ones((2, 2)), np.ones((2, 2)), P, TAU, projection="r3")
    with pytest.raises(ValueError):
        oracle.pnorm_estimate(np.ones((2, 2)), np.ones((2, 2)), P, TAU, norm_correct=True, projection="r1")
