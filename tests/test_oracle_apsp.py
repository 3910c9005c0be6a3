"""Pins of the oracle's APSP pieces (CPU only): Floyd-Warshall and Dijkstra
against scipy's csgraph (a library routine), the squaring loop with the
exact product against Floyd-Warshall, hop-limited brute force, closed forms
for short chains, and the one-sided bound of the estimate."""

import math

import numpy as np
import pytest
from scipy.sparse.csgraph import shortest_path

import oracle
from workloads import dense_graph, er_graph, rgg_graph


def _scipy_apsp(W):
    G = np.where(np.isfinite(W), W, 0.0).astype(np.float64)
    # csgraph reads 0 as "no edge"; nudge genuine zero-weight edges
    G[(G == 0) & np.isfinite(W)] = 1e-300
    np.fill_diagonal(G, 0.0)
    return shortest_path(G, method="D", directed=True)


@pytest.mark.parametrize("maker", [
    lambda: er_graph(60, 0.08, 10.0, seed=1),
    lambda: dense_graph(40, 1.0, 100.0, seed=2),
    lambda: rgg_graph(80, 0.2, 100.0, seed=3),
])
def test_floyd_warshall_and_dijkstra_match_scipy(maker):
    W = maker()
    ref = _scipy_apsp(W)
    fw = oracle.floyd_warshall(W)
    np.testing.assert_allclose(fw, ref, rtol=1e-12, atol=1e-250)
    src = [0, 5, len(W) - 1]
    np.testing.assert_allclose(oracle.dijkstra(W, src), ref[src], rtol=1e-12, atol=1e-250)


@pytest.mark.parametrize("n", [1, 2, 3, 17, 33, 64])
def test_exact_squaring_equals_floyd_warshall(n):
    """Transform, ceil(log2 n) exact squarings with the diagonal at 1, and
    the inverse transform give exactly the shortest distances."""
    W = er_graph(n, 0.15, 10.0, seed=40 + n)
    D, _ = oracle.apsp_exact_squaring(W, s=1.0)
    fw = oracle.floyd_warshall(W)
    fin = np.isfinite(fw)
    np.testing.assert_array_equal(np.isfinite(D), fin)
    np.testing.assert_allclose(D[fin], fw[fin], rtol=1e-12, atol=1e-12)


def test_squaring_count_limits_hops():
    """After T squarings the squaring loop covers paths of at most 2^T hops: with
    T = 1, brute-force min over one intermediate vertex."""
    W = er_graph(12, 0.3, 10.0, seed=50).astype(np.float64)
    D1, _ = oracle.apsp_exact_squaring(W, s=0.5, T=1)
    W0 = W.copy()
    np.fill_diagonal(W0, 0.0)
    two_hop = np.min(W0[:, :, None] + W0[None, :, :], axis=1)
    fin = np.isfinite(two_hop)
    np.testing.assert_array_equal(np.isfinite(D1), fin)
    np.testing.assert_allclose(D1[fin], two_hop[fin], rtol=1e-12, atol=1e-12)


def test_default_squarings():
    assert [oracle.default_squarings(n) for n in (1, 2, 3, 4, 5, 2048, 2049, 16384)] == \
        [0, 1, 2, 2, 3, 11, 12, 14]


@pytest.mark.parametrize("s,w,P,T", [(1.0, 2.0, [1, 2, 4, 8], 1), (0.35, 7.0, [1, 2, 4, 8, 16], 3),
                                     (1.0, 0.5, [1, 2, 4, 8, 16, 32, 64, 128, 256, 512], 2)])
def test_two_node_chain_closed_form(s, w, P, T):
    """W = [[0, w], [inf, 0]]: the (0, 1) entry sums the two equal terms
    X00 X01 and X01 X11, so every squaring multiplies it by 2^(1/p*):
    d01 = w - T ln2 / (s p*) (while positive); d10 = inf; d_ii = 0."""
    W = np.array([[0.0, w], [np.inf, 0.0]])
    out = oracle.apsp_estimate(W, s, P, tau=1e-290, T=T)
    pmax = P[-1]
    assert math.isclose(out["D"][0, 1], w - T * math.log(2) / (s * pmax), rel_tol=1e-12)
    assert out["D"][1, 0] == np.inf
    assert out["D"][0, 0] == 0.0 and out["D"][1, 1] == 0.0


def test_three_node_chain_closed_form():
    """0 -> 1 (a), 1 -> 2 (b).  One squaring: the 2-hop entry has a single
    nonzero term, so it is exact; the 1-hop entry picks up 2^(1/p).  Second
    squaring: (0, 2) sums (ab, 2^(2/p) ab, ab), i.e. 6^(1/p) ab."""
    a, b, p = 0.7, 1.3, 16
    W = np.array([[0.0, a, np.inf], [np.inf, 0.0, b], [np.inf, np.inf, 0.0]])
    o1 = oracle.apsp_estimate(W, 1.0, [p], tau=1e-290, T=1)
    assert math.isclose(o1["D"][0, 2], a + b, rel_tol=1e-13)
    assert math.isclose(o1["D"][0, 1], a - math.log(2) / p, rel_tol=1e-13)
    o2 = oracle.apsp_estimate(W, 1.0, [p], tau=1e-290, T=2)
    assert math.isclose(o2["D"][0, 2], a + b - math.log(6) / p, rel_tol=1e-13)


@pytest.mark.parametrize("maker,s,P", [
    (lambda: er_graph(48, 0.1, 10.0, seed=60), 1.0, [1, 2, 4, 8, 16, 32, 64]),
    (lambda: rgg_graph(64, 0.25, 100.0, seed=61), 0.1, [1, 2, 4, 8, 16, 32]),
])
def test_estimate_never_exceeds_exact_distance(maker, s, P):
    """||u||_p >= max u at every squaring and the exact product is monotone,
    so the estimated (x, max) matrix dominates the exact one and estimated
    distances never exceed the true ones; reachability is identical."""
    W = maker()
    out = oracle.apsp_estimate(W, s, P, tau=1e-290)
    fw = oracle.floyd_warshall(W)
    fin = np.isfinite(fw)
    np.testing.assert_array_equal(np.isfinite(out["D"]), fin)
    assert np.all(out["D"][fin] <= fw[fin] + 1e-9)
    assert np.all(out["D"] >= 0.0)
    assert np.all(np.diag(out["D"]) == 0.0)


def test_transform_round_trip():
    W = np.array([[0.0, 3.0, np.inf], [0.5, 0.0, 2.0], [np.inf, 1.0, 0.0]])
    X = oracle.to_maxtimes(W, s=0.35)
    assert X[0, 2] == 0.0 and np.all(np.diag(X) == 1.0)
    assert math.isclose(X[0, 1], math.exp(-1.05), rel_tol=1e-15)
    D = oracle.to_distances(X, s=0.35)
    np.testing.assert_allclose(D[np.isfinite(W)], W[np.isfinite(W)], rtol=1e-14, atol=1e-15)
    assert D[0, 2] == np.inf


def test_self_loops_do_not_change_distances():
    """A vertex reaches itself at distance 0 whatever its self-loop weight:
    the transform puts 1 on the diagonal, and the result equals
    Floyd-Warshall (which sets D_ii = 0)."""
    W = er_graph(20, 0.2, 10.0, seed=62).astype(np.float64)
    np.fill_diagonal(W, 3.0)
    D, _ = oracle.apsp_exact_squaring(W, s=1.0)
    fw = oracle.floyd_warshall(W)
    fin = np.isfinite(fw)
    np.testing.assert_allclose(D[fin], fw[fin], rtol=1e-12, atol=1e-12)
    assert np.all(np.diag(D) == 0.0)
