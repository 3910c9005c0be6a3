"""Pins of the oracle's exact product and p-norm estimate (CPU only).

Each test checks the oracle against something other than itself: brute
force, a library routine in a special case, a closed form, an invariant the
paper states, or a hand-derived golden value (tests/golden/).
"""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import exact_c
from workloads import lognormal_product, uniform_product

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
P64 = [1, 2, 4, 8, 16, 32, 64]


# ---------------------------------------------------------------- exact (Alg. 2)
@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (7, 1, 4), (8, 8, 8), (5, 6, 1)])
def test_exact_vectorised_matches_triple_loop(shape):
    m, k, n = shape
    rng = np.random.default_rng(11)
    A = rng.random((m, k))
    B = rng.random((k, n))
    np.testing.assert_array_equal(oracle.exact_maxtimes(A, B), oracle.exact_maxtimes_loops(A, B))


def test_exact_identity_and_permutation():
    rng = np.random.default_rng(12)
    A = rng.random((6, 6))
    I = np.eye(6)  # identity of (x, max): 1 on the diagonal, 0 elsewhere
    np.testing.assert_array_equal(oracle.exact_maxtimes(A, I), A)
    np.testing.assert_array_equal(oracle.exact_maxtimes(I, A), A)
    perm = rng.permutation(6)
    Pm = np.eye(6)[perm]
    np.testing.assert_array_equal(oracle.exact_maxtimes(Pm, A), A[perm])


def test_exact_homogeneity_and_zero_row():
    rng = np.random.default_rng(13)
    A = rng.random((5, 7))
    B = rng.random((7, 4))
    d1 = rng.random(5) + 0.5
    d2 = rng.random(4) + 0.5
    lhs = oracle.exact_maxtimes(d1[:, None] * A, B * d2[None, :])
    rhs = d1[:, None] * oracle.exact_maxtimes(A, B) * d2[None, :]
    np.testing.assert_allclose(lhs, rhs, rtol=1e-15)
    A[2] = 0.0
    assert np.all(oracle.exact_maxtimes(A, B)[2] == 0.0)


def test_exact_c_matches_numpy():
    rng = np.random.default_rng(14)
    A = rng.random((37, 53))
    B = rng.random((53, 29))
    ref = oracle.exact_maxtimes(A, B)
    np.testing.assert_array_equal(exact_c.exact_maxtimes_c(A, B), ref)
    rows = np.array([36, 0, 5, 5, 20])
    np.testing.assert_array_equal(exact_c.exact_maxtimes_c(A, B, rows), ref[rows])
    Af, Bf = A.astype(np.float32), B.astype(np.float32)
    np.testing.assert_array_equal(exact_c.exact_maxtimes_c(Af, Bf),
                                  oracle.exact_maxtimes(Af.astype(np.float64), Bf.astype(np.float64)))


# ------------------------------------------------------- estimate (Alg. 5, H')
def test_single_p1_is_ordinary_matmul():
    """P = {1}: the ring result is the ordinary product (Alg. 3), and the
    restored scale makes C exactly A @ B (a library routine)."""
    rng = np.random.default_rng(21)
    A = rng.random((9, 13)) * 7.0
    B = rng.random((13, 6)) * 0.3
    out = oracle.pnorm_estimate(A, B, [1], tau=1e-290)
    np.testing.assert_allclose(out["C"], A @ B, rtol=1e-13)
    assert np.all(out["pstar_idx"] == 0)


def test_single_p2_is_root_of_squared_matmul():
    rng = np.random.default_rng(22)
    A = rng.random((4, 11)) * 3.0
    B = rng.random((11, 5)) * 2.0
    out = oracle.pnorm_estimate(A, B, [2], tau=1e-290)
    np.testing.assert_allclose(out["C"], np.sqrt((A * A) @ (B * B)), rtol=1e-13)


def test_all_ones_attains_the_bound():
    """u is k equal values: ||u||_p = k^(1/p) ||u||_inf, the bound of Sec. 1
    is tight; the ÷k^(1/p*) correction gives back exactly the max."""
    k = 37
    A = np.ones((3, k))
    B = np.ones((k, 4))
    out = oracle.pnorm_estimate(A, B, P64, tau=1e-290)
    np.testing.assert_allclose(out["C"], k ** (1.0 / 64), rtol=1e-14)
    assert np.all(out["pstar_idx"] == len(P64) - 1)
    corr = oracle.pnorm_estimate(A, B, P64, tau=1e-290, norm_correct=True)
    np.testing.assert_allclose(corr["C"], 1.0, rtol=1e-14)


def test_one_hot_rows_are_exact():
    rng = np.random.default_rng(23)
    k = 16
    A = np.zeros((8, k))
    A[np.arange(8), rng.integers(0, k, 8)] = rng.random(8) + 0.1
    B = rng.random((k, 5))
    out = oracle.pnorm_estimate(A, B, P64, tau=1e-290)
    np.testing.assert_allclose(out["C"], oracle.exact_maxtimes(A, B), rtol=1e-14)


def test_golden_two_term_example():
    """Hand-derived closed form (tests/golden/two_term.json): u = (eps, eps)
    gives S_p = 2 eps^p; the threshold lands exactly on one p."""
    with open(os.path.join(GOLDEN, "two_term.json")) as f:
        cases = json.load(f)["cases"]
    for case in cases:
        A = np.array(case["A"], dtype=np.float64)
        B = np.array(case["B"], dtype=np.float64)
        out = oracle.pnorm_estimate(A, B, case["P"], tau=float.fromhex(case["tau_hex"]))
        assert int(out["pstar_idx"][0, 0]) == case["pstar_idx"], case["name"]
        np.testing.assert_allclose(out["C"][0, 0], float.fromhex(case["C_hex"]), rtol=1e-15)


def test_no_stable_p_uses_smallest_p():
    eps = 1e-20
    A = np.array([[1.0, eps]])
    B = np.array([[eps], [1.0]])
    out = oracle.pnorm_estimate(A, B, [1, 2, 4], tau=1e-3)
    assert out["pstar_idx"][0, 0] == oracle.PSTAR_NONE
    np.testing.assert_allclose(out["C"][0, 0], 2 * eps, rtol=1e-15)


def test_zero_rows_cols_and_empty_inner():
    rng = np.random.default_rng(24)
    A = rng.random((4, 6))
    B = rng.random((6, 3))
    A[1] = 0.0
    B[:, 2] = 0.0
    out = oracle.pnorm_estimate(A, B, P64, tau=1e-30)
    assert np.all(out["C"][1] == 0.0) and np.all(out["C"][:, 2] == 0.0)
    assert np.all(out["pstar_idx"][1] == oracle.PSTAR_NONE)
    e = oracle.pnorm_estimate(np.zeros((2, 0)), np.zeros((0, 3)), P64, tau=1e-30)
    assert e["C"].shape == (2, 3) and np.all(e["C"] == 0.0)
    assert np.all(e["pstar_idx"] == oracle.PSTAR_NONE)


@pytest.mark.parametrize("gen", ["uniform", "lognormal"])
def test_bound_exact_le_estimate_le_k_root(gen):
    """Sec. 1: ||u||_inf <= ||u||_p* <= k^(1/p*) ||u||_inf."""
    if gen == "uniform":
        A, B = uniform_product(40, 33, 27, seed=31)
    else:
        A, B = lognormal_product(40, 33, 27, seed=32)
        A, B = A.astype(np.float64), B.astype(np.float64)
    for tau in (1e-290, 1e-30, 1e-8):
        out = oracle.pnorm_estimate(A, B, [1, 2, 4, 8, 16, 32, 64, 128], tau)
        E = oracle.exact_maxtimes(A, B)
        k = A.shape[1]
        assert np.all(out["C"] >= E * (1 - 1e-12))
        assert np.all(out["C"] <= E * k ** (1.0 / out["pstar"]) * (1 + 1e-12))


def test_norm_sequence_is_monotone():
    """||u||_2p <= ||u||_p: S_{2p}^(1/(2p)) <= S_p^(1/p)."""
    A, B = lognormal_product(20, 50, 15, seed=33)
    P = [1, 2, 4, 8, 16, 32, 64, 128]
    S, _, _ = oracle.norm_power_sequence(A, B, P)
    for q in range(len(P) - 1):
        ok = S[q + 1] >= 1e-290  # outside the underflow range
        lo = S[q + 1][ok] ** (1.0 / P[q + 1])
        hi = S[q][ok] ** (1.0 / P[q])
        assert np.all(lo <= hi * (1 + 1e-12))


def test_homogeneity_keeps_pstar():
    A, B = lognormal_product(12, 30, 9, seed=34)
    rng = np.random.default_rng(35)
    d1 = np.exp(rng.normal(0, 3, 12))
    d2 = np.exp(rng.normal(0, 3, 9))
    P = [1, 2, 4, 8, 16, 32, 64, 128]
    a = oracle.pnorm_estimate(A, B, P, 1e-30)
    b = oracle.pnorm_estimate(d1[:, None] * A, B * d2[None, :], P, 1e-30)
    np.testing.assert_array_equal(a["pstar_idx"], b["pstar_idx"])
    np.testing.assert_allclose(b["C"], d1[:, None] * a["C"] * d2[None, :], rtol=1e-12)


def test_inner_permutation_invariance():
    A, B = uniform_product(10, 24, 8, seed=36)
    perm = np.random.default_rng(37).permutation(24)
    a = oracle.pnorm_estimate(A, B, P64, 1e-290)
    b = oracle.pnorm_estimate(A[:, perm], B[perm], P64, 1e-290)
    np.testing.assert_allclose(a["C"], b["C"], rtol=1e-13)
    np.testing.assert_array_equal(a["pstar_idx"], b["pstar_idx"])


def test_batched_equals_per_item_and_rows_helper():
    A, B = uniform_product(6, 9, 5, seed=38, batch=3)
    out = oracle.pnorm_estimate(A, B, P64, 1e-30)
    for b in range(3):
        one = oracle.pnorm_estimate(A[b], B[b], P64, 1e-30)
        np.testing.assert_allclose(out["C"][b], one["C"], rtol=1e-15)
    rows = np.array([4, 1])
    part = oracle.pnorm_estimate_rows(A[0], B[0], P64, 1e-30, rows)
    full = oracle.pnorm_estimate(A[0], B[0], P64, 1e-30)
    np.testing.assert_array_equal(part["C"], full["C"][rows])


def test_large_p_approaches_max():
    """lim_p ||u||_p = ||u||_inf (Sec. 1): with p = 1024 and distinct maxima
    the estimate is within k^(1/1024) of exact."""
    A, B = uniform_product(7, 64, 7, seed=39)
    out = oracle.pnorm_estimate(A, B, [1024], 1e-300)
    E = oracle.exact_maxtimes(A, B)
    assert np.max(out["C"] / E - 1) <= 64 ** (1 / 1024) - 1 + 1e-12


def test_rejects_bad_family():
    A = np.ones((2, 2))
    with pytest.raises(ValueError):
        oracle.pnorm_estimate(A, A, [2, 1], 1e-30)
    with pytest.raises(ValueError):
        oracle.pnorm_estimate(A, A, [0, 1], 1e-30)


def test_error_bound_formula_value():
    """The bound k^(1/p) - 1 of Sec. 1 at k = 256, p = 64 (about 9.05e-2)."""
    assert math.isclose(256 ** (1 / 64) - 1, 0.0905077326652577, rel_tol=1e-12)
