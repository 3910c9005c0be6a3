"""Pins of the oracle's affine correction of an APSP estimate (Sec. 4: an
affine model between a few exact distances and the estimated ones).  Each
pin comes from the definition of least squares or a library routine, not
from the oracle's formula:

* an estimate that is an exact affine image of the true distances is mapped
  back exactly (the model is recovered);
* on noisy data the fit equals numpy's least-squares solver on the same
  pairs, and its residuals satisfy the normal equations (sum zero,
  orthogonal to the estimate);
* two pairs: the line through both points;
* no usable pair (all unreachable): the identity; constant estimates:
  slope 1;
* the apply step keeps +inf and the zero diagonal and clamps at 0.
"""

import numpy as np
import pytest

import oracle
from workloads import er_graph


def _pairs(D_est, sources, rows):
    xs, ys = [], []
    for q, s in enumerate(sources):
        for v in range(D_est.shape[0]):
            if v != s and np.isfinite(D_est[s, v]) and np.isfinite(rows[q, v]):
                xs.append(D_est[s, v])
                ys.append(rows[q, v])
    return np.array(xs), np.array(ys)


def test_recovers_an_affine_image():
    W = er_graph(60, 0.1, 10.0, seed=31)
    Dt = oracle.floyd_warshall(W)
    a0, b0 = 1.37, -0.42
    D_est = Dt.copy()
    fin = np.isfinite(Dt) & ~np.eye(60, dtype=bool)
    D_est[fin] = (Dt[fin] - b0) / a0
    src = [0, 7, 33]
    rows = oracle.dijkstra(W, src)
    a, b = oracle.affine_fit(D_est, src, rows)
    assert a == pytest.approx(a0, rel=1e-12) and b == pytest.approx(b0, rel=1e-10)
    Dc = oracle.affine_apply(D_est, a, b)
    assert np.allclose(Dc[fin], Dt[fin], rtol=1e-12, atol=1e-12)
    assert np.array_equal(np.isinf(Dc), np.isinf(Dt)) and np.all(np.diag(Dc) == 0)


def test_matches_lstsq_and_normal_equations():
    rng = np.random.default_rng(32)
    W = er_graph(80, 0.08, 10.0, seed=33)
    Dt = oracle.floyd_warshall(W)
    D_est = Dt * rng.uniform(0.8, 1.1, Dt.shape) + rng.normal(0, 0.3, Dt.shape)
    np.fill_diagonal(D_est, 0.0)
    src = [1, 5, 40, 79]
    rows = oracle.dijkstra(W, src)
    a, b = oracle.affine_fit(D_est, src, rows)
    x, y = _pairs(D_est, src, rows)
    sol = np.linalg.lstsq(np.stack([x, np.ones_like(x)], 1), y, rcond=None)[0]
    assert a == pytest.approx(sol[0], rel=1e-10) and b == pytest.approx(sol[1], rel=1e-9, abs=1e-12)
    r = y - (a * x + b)
    assert abs(r.sum()) <= 1e-9 * np.abs(y).sum()
    assert abs((r * x).sum()) <= 1e-9 * np.abs(y * x).sum()


def test_two_points_line():
    W = np.array([[0.0, 2.0, np.inf], [np.inf, 0.0, 3.0], [np.inf, np.inf, 0.0]])
    D_est = np.array([[0.0, 1.0, 4.0], [np.inf, 0.0, 9.0], [np.inf, np.inf, 0.0]])
    rows = oracle.dijkstra(W, [0])  # exact: 0 -> 1 is 2, 0 -> 2 is 5
    a, b = oracle.affine_fit(D_est, [0], rows)
    # the line through (1, 2) and (4, 5): slope 1, intercept 1
    assert a == pytest.approx(1.0) and b == pytest.approx(1.0)


def test_degenerate_cases():
    W = np.full((4, 4), np.inf)
    np.fill_diagonal(W, 0.0)
    D = oracle.floyd_warshall(W)
    rows = oracle.dijkstra(W, [0, 2])
    assert oracle.affine_fit(D, [0, 2], rows) == (1.0, 0.0)
    W2 = np.array([[0.0, 1.0, 1.0], [1.0, 0.0, 1.0], [1.0, 1.0, 0.0]])
    D2 = np.array([[0.0, 2.0, 2.0], [2.0, 0.0, 2.0], [2.0, 2.0, 0.0]])
    a, b = oracle.affine_fit(D2, [0, 1], oracle.dijkstra(W2, [0, 1]))
    assert a == 1.0 and b == pytest.approx(-1.0)


def test_apply_keeps_inf_diagonal_and_clamps():
    D = np.array([[0.0, 0.5, np.inf], [3.0, 0.0, 1.0], [np.inf, 2.0, 0.0]])
    Dc = oracle.affine_apply(D, 2.0, -2.0)
    assert np.isinf(Dc[0, 2]) and np.isinf(Dc[2, 0])
    assert np.all(np.diag(Dc) == 0)
    assert Dc[0, 1] == 0.0 and Dc[1, 0] == 4.0 and Dc[1, 2] == 0.0 and Dc[2, 1] == 2.0
