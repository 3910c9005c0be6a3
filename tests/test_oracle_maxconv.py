"""Pins of the oracle's max-convolution (Sec. 1).  From the definition and
the mathematics, not the oracle's formula:

* the exact max-convolution equals a brute-force double loop, and a
  one-hot x shifts y;
* the estimate lies in [exact, min(n, m)^(1/p*) exact] (the p-norm bound of
  Sec. 1 over the list of at most min(n, m) products);
* one-hot inputs are exact; all-ones inputs attain the bound exactly at
  every index (count^(1/p*), count the number of overlapping products);
* a closed form for the selection: x = (1, e), y = (1, e) gives the middle
  index S_p = 2 e^p, so p* is the largest p with 2 e^p >= tau;
* scaling x and y by positive constants scales z by their product with the
  same p*.
"""

import itertools

import numpy as np
import pytest

import oracle

P = [1, 2, 4, 8, 16, 32, 64]


def test_exact_matches_brute_force():
    rng = np.random.default_rng(51)
    x = rng.random((3, 7))
    y = rng.random((3, 5))
    z = oracle.exact_maxconv(x, y)
    for b, t in itertools.product(range(3), range(11)):
        best = max((x[b, i] * y[b, t - i] for i in range(7) if 0 <= t - i < 5), default=0.0)
        assert z[b, t] == best
    e = np.zeros(6)
    e[2] = 1.0
    np.testing.assert_array_equal(oracle.exact_maxconv(e, y[0])[0, 2:7], y[0])


def test_bounds_on_random_inputs():
    rng = np.random.default_rng(52)
    x = rng.random((4, 40)) ** 2
    y = rng.random((4, 25))
    E = oracle.exact_maxconv(x, y)
    out = oracle.maxconv_estimate(x, y, P)
    ps = np.asarray(P, dtype=float)[out["pstar_idx"]]
    assert np.all(out["z"] >= E * (1 - 1e-12))
    assert np.all(out["z"] <= E * 25 ** (1.0 / ps) * (1 + 1e-12))


def test_one_hot_exact_and_all_ones_tight():
    y = np.array([0.3, 0.9, 0.5])
    x = np.zeros(5)
    x[1] = 2.0
    out = oracle.maxconv_estimate(x, y, P)
    np.testing.assert_allclose(out["z"][0], oracle.exact_maxconv(x, y)[0], rtol=1e-13)
    n, m = 6, 4
    out = oracle.maxconv_estimate(np.ones(n), np.ones(m), P)
    cnt = np.array([min(t + 1, n, m, n + m - 1 - t) for t in range(n + m - 1)], dtype=float)
    np.testing.assert_allclose(out["z"][0], cnt ** (1.0 / 64), rtol=1e-13)
    assert np.all(out["pstar_idx"] == P.index(64))


@pytest.mark.parametrize("e", [1e-3, 1e-2, 0.3])
def test_selection_closed_form(e):
    x = np.array([1.0, e])
    y = np.array([1.0, e])
    out = oracle.maxconv_estimate(x, y, P)
    want = max(q for q, p in enumerate(P) if 2 * e ** p >= 1e-12)
    assert out["pstar_idx"][0, 1] == want
    p = P[want]
    np.testing.assert_allclose(out["z"][0, 1], (2 * e ** p) ** (1.0 / p), rtol=1e-12)


def test_homogeneity():
    rng = np.random.default_rng(53)
    x = rng.random((2, 30))
    y = rng.random((2, 20))
    a = oracle.maxconv_estimate(x, y, P)
    b = oracle.maxconv_estimate(3.5 * x, 0.2 * y, P)
    np.testing.assert_allclose(b["z"], 0.7 * a["z"], rtol=1e-12)
    assert np.array_equal(a["pstar_idx"], b["pstar_idx"])
