"""Pins of the oracle's top k of x_i + y_j (Sec. 2.3, algorithm E and the
index recovery).  From the definition and the mathematics, not from the
oracle's own formulas:

* the brute-force top k equals a double loop and a sort;
* lists whose diagonals hold one term each (x of length 1) are popped
  exactly, in value order;
* a near one-hot x (one element, the rest 60 below it) makes every diagonal
  one dominant term: values and indices are exact, and so on the mirror
  case with y near one-hot;
* k = 1 is the largest value of the max-convolution estimate (Sec. 1) of
  e^x and e^y, and it bounds the true maximum from above;
* on well separated random lists the estimate finds the true top k and its
  indices (the behaviour Sec. 3 reports for uniform lists);
* shifting x and y by constants shifts the values and keeps the indices;
  the run on y reversed gives the same values (the order of y does not
  matter, the premise of the index recovery).

The paired queue (Discussion: both runs in lockstep, exact values where the
pair is accurate):

* on an input where every rank's pair is accurate it returns the
  brute-force top k to the bit, indices included;
* accepted ranks are grid pairs on both popped diagonals with the exact
  value x_i + y_j, no pair twice (also deep into an exhausted queue), and
  rank 0 pops what each plain run pops first;
* the acceptance threshold psi len^(-1/p*) never exceeds a diagonal's true
  largest term on exact ring results (the norm inequality), and a diagonal
  of equal terms attains it.
"""

import itertools

import numpy as np
import pytest

import oracle
from oracle.xy_topk import exact_topk_xy, norm_queue, queue_pops, ring_results, xy_topk_estimate
from xy_robust import fft_ring_results, robust_depth

# 24 powers up to 4096, as in Sec. 3 (|P| = 24, p*_max = 4096)
P24 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096]


def test_exact_matches_brute_force():
    rng = np.random.default_rng(81)
    x = rng.normal(size=7)
    y = rng.normal(size=5)
    v, i, j = exact_topk_xy(x, y, 9)
    pairs = sorted(((x[a] + y[b], a, b) for a, b in itertools.product(range(7), range(5))),
                   key=lambda t: -t[0])[:9]
    np.testing.assert_array_equal(v, [p[0] for p in pairs])
    np.testing.assert_array_equal(i, [p[1] for p in pairs])
    np.testing.assert_array_equal(j, [p[2] for p in pairs])


def test_single_term_diagonals_are_exact():
    rng = np.random.default_rng(82)
    y = rng.uniform(0, 3, 20)
    r = norm_queue([0.7], y, P24, 12)
    order = np.argsort(-y)[:12]
    np.testing.assert_allclose(r["values"], 0.7 + y[order], rtol=0, atol=1e-12)
    np.testing.assert_array_equal(r["diag"], order)


def test_near_one_hot_exact_with_indices():
    rng = np.random.default_rng(83)
    n, k = 32, 16
    x = np.full(n, -60.0)
    x[5] = 1.5
    y = rng.uniform(0, 3, n)
    r = xy_topk_estimate(x, y, P24, k)
    v, i, j = exact_topk_xy(x, y, k)
    np.testing.assert_allclose(r["values"], v, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(r["i"], i)
    np.testing.assert_array_equal(r["j"], j)
    # the mirror: y near one-hot
    r = xy_topk_estimate(y, x, P24, k)
    v, i, j = exact_topk_xy(y, x, k)
    np.testing.assert_allclose(r["values"], v, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(r["i"], i)
    np.testing.assert_array_equal(r["j"], j)


def test_first_pop_is_the_max_convolution_estimate():
    rng = np.random.default_rng(84)
    x = rng.uniform(0, 5, 50)
    y = rng.uniform(0, 5, 50)
    r = norm_queue(x, y, P24, 1)
    mc = oracle.maxconv_estimate(np.exp(x), np.exp(y), P24)
    assert abs(r["values"][0] - np.log(mc["z"].max())) <= 1e-12
    true_max = x.max() + y.max()
    assert true_max - 1e-12 <= r["values"][0] <= true_max + np.log(50) / P24[0]


def test_well_separated_lists_find_the_true_top_k():
    rng = np.random.default_rng(85)
    x = rng.uniform(0, 40, 64)
    y = rng.uniform(0, 40, 64)
    r = xy_topk_estimate(x, y, P24, 16)
    v, i, j = exact_topk_xy(x, y, 16)
    np.testing.assert_allclose(r["values"], v, rtol=0, atol=1e-4)
    np.testing.assert_array_equal(r["i"], i)
    np.testing.assert_array_equal(r["j"], j)


def test_shift_invariance_and_order_of_y():
    rng = np.random.default_rng(86)
    x = rng.uniform(0, 10, 40)
    y = rng.uniform(0, 10, 40)
    a = xy_topk_estimate(x, y, P24, 10)
    b = xy_topk_estimate(x + 3.25, y - 1.5, P24, 10)
    np.testing.assert_allclose(b["values"], a["values"] + 1.75, rtol=0, atol=1e-9)
    np.testing.assert_array_equal(a["diag"], b["diag"])
    np.testing.assert_array_equal(a["i"], b["i"])
    rev = norm_queue(x, y[::-1], P24, 10)
    np.testing.assert_allclose(rev["values"], a["values"], rtol=0, atol=1e-6)


def test_no_stable_power_and_validation():
    # the stability test is S >= tau (Sec. 1): a ring result equal to tau counts
    r = norm_queue([0.0], [0.0], [1, 2], 1, tau=1.0)
    assert r["values"][0] == 0.0 and r["diag"][0] == 0
    # tau above every ring result: nothing is stable, every value is -inf
    r = norm_queue([0.0, 0.0], [0.0, 0.0], [1, 2], 2, tau=10.0)
    assert np.isneginf(r["values"]).all()
    try:
        xy_topk_estimate([0.0, 1.0], [0.0], [1], 1)
    except ValueError:
        pass
    else:
        raise AssertionError("unequal lengths must be rejected")


# ---- the paired queue (Discussion) ----------------------------------------

from oracle.xy_topk import _diag_len, _estimate, _min_admitted, xy_topk_paired  # noqa: E402


def test_paired_every_rank_accepted_is_the_exact_top_k():
    # spread 40, n = 256, k = 64: every rank's pair is accurate, so the
    # sequence is the brute-force top k to the bit, indices included
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 40, 256)
    y = rng.uniform(0, 40, 256)
    r = xy_topk_paired(x, y, P24, 64)
    v, i, j = exact_topk_xy(x, y, 64)
    assert r["accepted"].all()
    np.testing.assert_array_equal(r["values"], v)
    np.testing.assert_array_equal(r["i"], i)
    np.testing.assert_array_equal(r["j"], j)


def test_paired_accepted_ranks_are_grid_pairs_of_both_diagonals():
    rng = np.random.default_rng(4)
    n, k = 256, 64
    x = rng.uniform(0, 10, n)
    y = rng.uniform(0, 10, n)
    r = xy_topk_paired(x, y, P24, k)
    acc = r["accepted"]
    assert 0 < acc.sum() < k  # this input has both kinds of rank
    i, j = r["i"][acc], r["j"][acc]
    np.testing.assert_array_equal(i + j, r["diag"][acc])
    np.testing.assert_array_equal(i + n - 1 - j, r["anti"][acc])
    np.testing.assert_array_equal(r["values"][acc], x[i] + y[j])
    assert len(set(zip(i.tolist(), j.tolist()))) == acc.sum()  # no pair twice
    assert (r["i"][~acc] == -1).all() and (r["j"][~acc] == -1).all()
    # rank 0 pops what each plain run pops first
    a = norm_queue(x, y, P24, 1)
    b = norm_queue(x, y[::-1], P24, 1)
    assert r["diag"][0] == a["diag"][0] and r["anti"][0] == b["diag"][0]


def test_min_admitted_bounds_every_diagonal_maximum():
    # ||u||_inf >= ||u||_p len^(-1/p): on exact ring results the threshold
    # never exceeds a diagonal's true largest term
    rng = np.random.default_rng(5)
    n = 40
    x = rng.normal(0, 2, n)
    y = rng.normal(0, 2, n)
    xs, ys = np.exp(x - x.max()), np.exp(y - y.max())
    sig = np.stack([np.convolve(xs ** p, ys ** p) for p in P24])
    for m in range(2 * n - 1):
        a, q = _estimate(sig[:, m], P24, 1e-12)
        i = np.arange(max(0, m - n + 1), min(m, n - 1) + 1)
        assert i.size == _diag_len(m, n)
        true_max = (xs[i] * ys[m - i]).max()
        assert _min_admitted(a, q, m, n, P24) <= true_max * (1 + 1e-12)
        assert a >= true_max * (1 - 1e-12)


def test_min_admitted_is_attained_by_a_constant_diagonal():
    # the bound is tight: a diagonal of len equal terms v has p-norm
    # v len^(1/p), and the threshold gives v back
    n = 9
    for m in (0, 3, 8, 12):
        ln = _diag_len(m, n)
        for q, p in enumerate(P24):
            a = 0.75 * ln ** (1.0 / p)
            np.testing.assert_allclose(_min_admitted(a, q, m, n, P24), 0.75, rtol=1e-13)
    assert _min_admitted(0.0, -1, 4, n, P24) == np.inf


def test_paired_deep_queue_reports_no_pair_twice():
    # past the accurate ranks the two runs pop the same two diagonals again
    # and meet in the pair they already reported: it must not come back
    rng = np.random.default_rng(1000)
    x = rng.uniform(0, 8, 17)
    y = rng.uniform(0, 8, 17)
    r = xy_topk_paired(x, y, P24, 289)
    acc = r["accepted"]
    pairs = set(zip(r["i"][acc].tolist(), r["j"][acc].tolist()))
    assert len(pairs) == acc.sum() > 17
    np.testing.assert_array_equal(r["values"][acc], x[r["i"][acc]] + y[r["j"][acc]])


def test_paired_exhausted_queue_reports_nothing_more():
    # n = 1: one pair; rank 0 is that pair exactly, then no p is stable on
    # either run and the remaining ranks are -inf with no indices
    r = xy_topk_paired([0.25], [-1.5], P24, 3)
    assert r["values"][0] == 0.25 + -1.5 and r["i"][0] == 0 and r["j"][0] == 0
    assert r["accepted"].tolist() == [True, False, False]
    assert np.isneginf(r["values"][1:]).all() and (r["i"][1:] == -1).all()


def test_queue_pops_from_ring_results_is_the_queue():
    """Splitting the queue from its ring results changes nothing: the pops
    from ring_results equal norm_queue, and FFT ring results (numpy, exact
    up to rounding) agree with the direct convolution to rounding."""
    rng = np.random.default_rng(9650)
    x, y = rng.normal(0, 1, 300), rng.uniform(0, 2, 300)
    sigma, mx, my = ring_results(x, y, P24)
    a = norm_queue(x, y, P24, 20)
    b = queue_pops(sigma, mx, my, P24, 20)
    np.testing.assert_array_equal(a["diag"], b["diag"])
    np.testing.assert_array_equal(a["values"], b["values"])
    sf, mxf, myf = fft_ring_results(x, y, P24, 1024)
    assert (mxf, myf) == (mx, my)
    bound = 1e-12 * np.linalg.norm(sigma, axis=1, keepdims=True)
    assert (np.abs(sf - sigma) <= bound).all()


@pytest.mark.parametrize("n,seed", [(1024, 9600), (1024, 9601), (2048, 9700), (3000, 9801), (8192, 9800)])
def test_uniform_unit_lists_are_rounding_robust(n, seed):
    """The premise of the GPU's whole-sequence comparison on uniform [0, 1]
    lists: their top 128 (diagonals of both runs, values within 1e-6) is the
    same whichever of three FFT lengths computes the ring results."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0, 1, n)
    assert robust_depth(x, y, P24, 128) == 128


def test_robust_depth_is_short_where_ghosts_appear():
    """A near one-hot x leaves FFT residuals above tau once the dominant
    diagonal terms are popped (reading 20): the depth stops early there,
    and it never exceeds k."""
    rng = np.random.default_rng(9651)
    n = 512
    x = np.full(n, -60.0)
    x[17] = 2.0
    y = rng.uniform(0, 3, n)
    d = robust_depth(x, y, P24, 64)
    assert 1 <= d < 64
