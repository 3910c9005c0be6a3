"""Pins of the oracle's r = 2 projection (Sec. 1: the norm sequence
projected onto two unique values; reading R7 of oracle/pnorm.py).  Each pin
comes from the method's definition or the mathematics, not from the
oracle's formula:

* two distinct term values (any counts): the projection is exact, where the
  plain root and the r = 1 projection are not;
* one distinct value (ties): the Hankel matrix has rank 1, the r = 1
  projection is used, which is exact there;
* positive row / column scaling commutes with the estimate;
* the projected value equals the largest root that numpy's polynomial
  solver (np.roots) finds for the null-space polynomial of the 2 x 3
  Hankel matrix, itself checked to vanish on that matrix;
* the added norms are 3p/4 for the p with p/4 and p/2 in the family.
"""

import numpy as np
import pytest

import oracle
from oracle.pnorm import r2_aux_powers

TAU = 1e-290
P = [1, 2, 4, 8, 16, 32, 64]


def test_aux_powers():
    assert r2_aux_powers(P) == [3, 6, 12, 24, 48]
    assert r2_aux_powers([1, 2, 4]) == [3]
    assert r2_aux_powers([1, 4, 16]) == []
    assert r2_aux_powers([2, 4, 8, 12]) == [6]  # 12 = 3*16/4 would need 16


@pytest.mark.parametrize("n1,n2", [(1, 1), (1, 5), (3, 40), (10, 2)])
@pytest.mark.parametrize("a1,a2", [(0.9, 0.6), (0.97, 0.2), (0.5, 0.45)])
def test_two_values_exact(n1, n2, a1, a2):
    """u = (a1 x n1, a2 x n2) scaled by M: the estimate is M a1 exactly
    (a1 > a2); p* = 64 is stable for all of these."""
    M = 2.5
    u = np.array([a1] * n1 + [a2] * n2)
    A = (u * M)[None, :]
    B = np.ones((u.size, 1))
    out = oracle.pnorm_estimate(A, B, P, TAU, projection="r2")
    assert out["pstar_idx"][0, 0] == P.index(64)
    # scaled terms are u / a1 (row max), so the projected max is 1 -> M a1
    np.testing.assert_allclose(out["C"][0, 0], M * a1, rtol=1e-9)
    r1 = oracle.pnorm_estimate(A, B, P, TAU, projection="r1")["C"][0, 0]
    plain = oracle.pnorm_estimate(A, B, P, TAU)["C"][0, 0]
    if n1 > 1:  # tied top terms inflate the plain root by n1^(1/64)
        assert abs(plain - M * a1) > 1e-6 * M * a1
    assert abs(out["C"][0, 0] - M * a1) <= abs(r1 - M * a1) + 1e-12


def test_ties_fall_back_to_r1():
    h = 7
    A = np.full((1, h), 0.3)
    B = np.ones((h, 1))
    out = oracle.pnorm_estimate(A, B, P, TAU, projection="r2")
    np.testing.assert_allclose(out["C"][0, 0], 0.3, rtol=1e-12)


def test_homogeneity():
    rng = np.random.default_rng(41)
    A = rng.random((6, 30))
    B = rng.random((30, 5))
    d1 = rng.uniform(0.2, 5, 6)
    d2 = rng.uniform(0.2, 5, 5)
    a = oracle.pnorm_estimate(A, B, P, TAU, projection="r2")
    b = oracle.pnorm_estimate(d1[:, None] * A, B * d2[None, :], P, TAU, projection="r2")
    np.testing.assert_allclose(b["C"], d1[:, None] * a["C"] * d2[None, :], rtol=1e-9)


def test_matches_np_roots_on_random_entries():
    rng = np.random.default_rng(42)
    A = rng.random((5, 40)) ** 3
    B = rng.random((40, 4))
    out = oracle.pnorm_estimate(A, B, P, TAU, projection="r2")
    r1 = oracle.pnorm_estimate(A, B, P, TAU, projection="r1")["C"]
    aux = out["aux"]
    used = 0
    for i in range(5):
        for j in range(4):
            ps = P[out["pstar_idx"][i, j]]
            t = ps // 4
            Sk = []
            for p in (t, 2 * t, 3 * t, 4 * t):
                Sk.append(out["S"][P.index(p), i, j] if p in P else out["S_aux"][aux.index(p), i, j])
            H = np.array([[Sk[0], Sk[1], Sk[2]], [Sk[1], Sk[2], Sk[3]]])
            g = np.linalg.svd(H)[2][-1]
            assert np.allclose(H @ g, 0, atol=1e-12 * np.abs(H).max())
            rts = np.roots([g[2], g[1], g[0]])
            rts = rts[np.isreal(rts)].real
            rts = rts[rts > 0]
            if rts.size == 0:
                np.testing.assert_allclose(out["C"][i, j], r1[i, j], rtol=1e-12)
                continue
            alpha = rts.max() ** (1.0 / t)
            np.testing.assert_allclose(out["C"][i, j], out["r"][i] * out["c"][j] * alpha, rtol=1e-7)
            used += 1
    assert used >= 10


def test_rejects_r2_with_norm_correct():
    with pytest.raises(ValueError):
        oracle.pnorm_estimate(np.ones((2, 2)), np.ones((2, 2)), P, TAU, norm_correct=True, projection="r2")
