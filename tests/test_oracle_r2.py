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


def _two_value_norms(gamma, h2, P_all):
    """Closed-form norms of u = (1, then h2 copies of 1 - gamma): S_p = 1 +
    h2 (1 - gamma)^p, for every power in P_all."""
    return {p: 1.0 + h2 * (1.0 - gamma) ** p for p in P_all}


def _normalised_rho(Sq):
    """sigma_2 / sigma_1 of [[t1, t2, t3], [t2, t3, t4]], t_k = S_kq / c^k,
    c = (S_4q / S_q)^(1/3): the rank quantity of reading R7, formed here by
    plain division (not the oracle's logarithms)."""
    c = (Sq[3] / Sq[0]) ** (1.0 / 3.0)
    t = [Sq[k] / c ** (k + 1) for k in range(4)]
    sv = np.linalg.svd(np.array([[t[0], t[1], t[2]], [t[1], t[2], t[3]]]), compute_uv=False)
    return sv[1] / sv[0]


def _project_closed_form(gamma, h2=1.0, k=2):
    """The oracle's r = 2 projection (p* = 64, q = 16) on the closed-form
    norms; returns (output, r = 1 value, rho, theta)."""
    aux = r2_aux_powers(P)
    Sd = _two_value_norms(gamma, h2, P + aux)
    S = np.array([Sd[p] for p in P]).reshape(len(P), 1)
    S_aux = np.array([Sd[p] for p in aux]).reshape(len(aux), 1)
    idx = np.array([P.index(64)], dtype=np.uint8)
    r1 = (Sd[64] / Sd[32]) ** (1.0 / 32)
    info = {}
    out = oracle.pnorm._project_r2(S, P, idx, np.array([r1]), S_aux, aux, k, info)
    Sq = [Sd[16], Sd[32], Sd[48], Sd[64]]
    return out[0], r1, _normalised_rho(Sq), oracle.pnorm.r2_threshold(k, 64, max(abs(np.log(v)) for v in Sq))


def test_rank_threshold_switches_once_at_theta():
    """Two values 1 and 1 - gamma (one term each): far above the threshold
    the projection returns the largest value 1, far below (near ties) the r = 1
    value; over a sweep of gamma it switches once, where the rank quantity
    sigma_2 / sigma_1 (formed independently above) crosses theta."""
    gammas = np.logspace(-9, -1, 161)
    side = []
    for g in gammas:
        out, r1, rho, theta = _project_closed_form(g)
        if rho > theta * 1.01:
            # the projection recovers the largest value, to the accuracy the
            # threshold guarantees against the rounding of the norms
            assert abs(out - 1.0) <= oracle.pnorm.R2_DELTA, (g, out)
            side.append(1)
        elif rho < theta * 0.99:
            assert out == r1, (g, out, r1)
            side.append(0)
    side = np.array(side)
    assert side[0] == 0 and side[-1] == 1
    assert (np.diff(side) >= 0).all()  # one switch


def test_threshold_bounds_the_rounding_of_the_projection():
    """The reading's claim: with every norm perturbed by a relative error of
    at most eps = (K + 4 p* + L) 2^-53, an entry above the threshold keeps
    its projected value within 4 delta = 1e-5 of the largest value (near
    ties, the worst case for the root).  Just below the threshold the same
    perturbations move it by more than delta, which is why it falls back."""
    rng = np.random.default_rng(17)
    aux = r2_aux_powers(P)
    k = 2
    worst_above, worst_below = 0.0, 0.0
    for g in np.logspace(-6, -2, 60):
        Sd = _two_value_norms(g, 1.0, P + aux)
        Sq = [Sd[16], Sd[32], Sd[48], Sd[64]]
        eps = (k + 4 * 64 + max(abs(np.log(v)) for v in Sq)) * 2.0 ** -53
        rho = _normalised_rho(Sq)
        theta = oracle.pnorm.r2_threshold(k, 64, max(abs(np.log(v)) for v in Sq))
        for _ in range(20):
            Sp = {p: v * (1.0 + eps * rng.uniform(-1, 1)) for p, v in Sd.items()}
            S = np.array([Sp[p] for p in P]).reshape(len(P), 1)
            S_aux = np.array([Sp[p] for p in aux]).reshape(len(aux), 1)
            idx = np.array([P.index(64)], dtype=np.uint8)
            info = {}
            oracle.pnorm._project_r2(S, P, idx, np.array([0.0]), S_aux, aux, k, info)
            alt = info["alt"][0]
            val = np.nan
            if rho > 1.05 * theta:
                val = oracle.pnorm._project_r2(S, P, idx, np.array([0.0]), S_aux, aux, k)[0]
                worst_above = max(worst_above, abs(val - 1.0))
            elif rho < theta / 1.05 and np.isfinite(alt):
                worst_below = max(worst_below, abs(alt - 1.0))
    assert worst_above <= 4 * oracle.pnorm.R2_DELTA, worst_above
    assert worst_below > oracle.pnorm.R2_DELTA, worst_below
