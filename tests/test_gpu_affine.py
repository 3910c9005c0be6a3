"""Exact rows from a few sources (Bellman-Ford on the GPU) against the
oracle's Dijkstra, and the affine correction of the APSP estimate (Sec. 4)
against the oracle's fit on the same estimate and exact rows."""

import math

import numpy as np
import pytest

import oracle
from workloads import er_graph, rgg_graph

pytestmark = pytest.mark.gpu

P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _same(a, b, rtol):
    assert np.array_equal(np.isinf(a), np.isinf(b))
    f = np.isfinite(a)
    assert np.allclose(a[f], b[f], rtol=rtol, atol=0)


@pytest.mark.parametrize("kind", ["er", "rgg"])
def test_exact_rows_match_dijkstra(gpu_lib, kind):
    if kind == "er":
        W = er_graph(300, 0.04, 10.0, seed=911)
    else:
        n = 400
        W = rgg_graph(n, math.sqrt(8.0 / (math.pi * n)), 100.0, seed=912)
    rng = np.random.default_rng(913)
    src = rng.choice(W.shape[0], 17, replace=False).astype(np.int32)
    print(f"[exact-rows] {kind} n={W.shape[0]}", flush=True)
    D, rounds = gpu_lib.apsp_exact_rows(_dev(W), src)
    ref = oracle.dijkstra(W, src)
    _same(D.cpu().numpy(), ref, 1e-12)
    assert 1 <= rounds <= W.shape[0] - 1
    if kind == "rgg":
        assert rounds > 8  # several convergence checks


def test_exact_rows_bad_source(gpu_lib):
    W = er_graph(50, 0.1, 10.0, seed=914)
    with pytest.raises(gpu_lib.MaxTimesError):
        gpu_lib.apsp_exact_rows(_dev(W), [3, 50])


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_affine_correct_matches_oracle(gpu_lib, path):
    import torch

    n = 300
    W = er_graph(n, 0.04, 10.0, seed=915)
    P = P512 if path == "fp64" else P512[:8]
    dt = torch.float64 if path == "fp64" else torch.float32
    D = gpu_lib.apsp(_dev(W), s=1.0, P=P, path=path, out_dtype=dt)
    src = np.array([0, 17, 123, 299], dtype=np.int32)
    rows, _ = gpu_lib.apsp_exact_rows(_dev(W), src)
    D_est = D.cpu().numpy().astype(np.float64)
    a_ref, b_ref = oracle.affine_fit(D_est, src, rows.cpu().numpy())
    ab = gpu_lib.apsp_affine_correct(D, src, rows).cpu().numpy()
    print(f"[affine] {path}: a {ab[0]:.6f} b {ab[1]:.6f}", flush=True)
    assert ab[0] == pytest.approx(a_ref, rel=1e-9) and ab[1] == pytest.approx(b_ref, rel=1e-8, abs=1e-12)
    Dc_ref = oracle.affine_apply(D_est, ab[0], ab[1])
    _same(D.cpu().numpy().astype(np.float64), Dc_ref, 1e-12 if path == "fp64" else 1e-6)
    # the correction lowers the error against the exact distances
    Dt = oracle.floyd_warshall(W)
    fin = np.isfinite(Dt) & ~np.eye(n, dtype=bool)
    mse0 = np.mean((D_est[fin] - Dt[fin]) ** 2)
    mse1 = np.mean((D.cpu().numpy()[fin] - Dt[fin]) ** 2)
    assert mse1 < mse0


def test_affine_without_pairs_is_identity(gpu_lib):
    import torch

    n = 8
    W = np.full((n, n), np.inf, dtype=np.float32)
    np.fill_diagonal(W, 0.0)
    D = gpu_lib.apsp(_dev(W), s=1.0, P=P512, path="fp64", out_dtype=torch.float64)
    rows, _ = gpu_lib.apsp_exact_rows(_dev(W), [0, 3])
    before = D.clone()
    ab = gpu_lib.apsp_affine_correct(D, [0, 3], rows).cpu().numpy()
    assert ab[0] == 1.0 and ab[1] == 0.0
    assert torch.equal(before, D)
