"""GPU parity of the APSP estimate (Sec. 2.2) with the oracle's driver, and
properties at full size (reachability, zero diagonal, the one-sided bound
against exact distances)."""

import math

import numpy as np
import pytest

import oracle
from parity import TAU
from workloads import config, er_graph, rgg_graph

pytestmark = pytest.mark.gpu

P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]
P128 = [1, 2, 4, 8, 16, 32, 64, 128]


def _apsp(mt, W, s, P, path, T=-1, raw=False, out_dtype=None):
    import torch

    od = out_dtype or (torch.float64 if path == "fp64" else torch.float32)
    Wd = torch.from_numpy(np.ascontiguousarray(W)).cuda()
    D, ps = mt.apsp(Wd, s=s, P=P, path=path, n_squarings=T, raw=raw, out_dtype=od, return_pstar=True)
    return D.cpu().numpy().astype(np.float64), ps.cpu().numpy()


def _check_x(Xg, Xo, tol):
    both0 = (Xg == 0) & (Xo == 0)
    rel = np.abs(Xg - Xo) / np.maximum(Xo, 1e-300)
    rel[both0] = 0
    assert (Xg[Xo == 0] == 0).all() and (Xo[Xg == 0] == 0).all(), "reachability differs"
    assert rel.max() <= tol, f"max rel {rel.max():.3e} > {tol}"
    return rel.max()


@pytest.mark.parametrize("n", [1, 2, 3, 64, 200, 333])
def test_fp64_apsp_parity(gpu_lib, n):
    W = er_graph(n, min(1.0, 8.0 / max(n, 1)), 10.0, seed=200 + n)
    print(f"[apsp] fp64 ER n={n}", flush=True)
    ref = oracle.apsp_estimate(W, 1.0, P512, TAU["fp64"])
    X, _ = _apsp(gpu_lib, W, 1.0, P512, "fp64", raw=True)
    _check_x(X, ref["X"], 1e-5)
    D, ps = _apsp(gpu_lib, W, 1.0, P512, "fp64")
    fin = np.isfinite(ref["D"])
    assert np.array_equal(np.isfinite(D), fin)
    assert np.abs(D[fin] - ref["D"][fin]).max() <= 1e-5
    if n > 1:
        assert np.array_equal(ps, ref["pstar_idx_last"])


@pytest.mark.parametrize("n,T", [(150, 1), (300, 1), (300, 2)])
def test_bf16_apsp_parity_few_squarings(gpu_lib, n, T):
    """BF16 rounding of each squaring feeds the next; parity is checked over
    one or two squarings at the path's tolerance."""
    W = rgg_graph(n, math.sqrt(20.0 / (math.pi * n)), 100.0, seed=300 + n)
    print(f"[apsp] bf16 RGG n={n} T={T}", flush=True)
    ref = oracle.apsp_estimate(W, 0.35, P128, TAU["bf16"], T=T)
    X, _ = _apsp(gpu_lib, W, 0.35, P128, "bf16", T=T, raw=True)
    _check_x(X, ref["X"], 2e-3 * T)


@pytest.mark.parametrize("path,s,P", [("fp64", 1.0, P512), ("bf16", 0.35, P128)])
def test_apsp_properties_full_squarings(gpu_lib, path, s, P):
    W = rgg_graph(400, 0.08, 100.0, seed=17) if path == "bf16" else er_graph(400, 0.02, 10.0, seed=17)
    print(f"[apsp] properties {path}", flush=True)
    D, _ = _apsp(gpu_lib, W, s, P, path)
    fw = oracle.floyd_warshall(W)
    fin = np.isfinite(fw)
    assert np.array_equal(np.isfinite(D), fin)
    assert (np.diag(D) == 0).all() and (D >= 0).all()
    # estimate >= exact in (x, max) space  <=>  distance <= exact distance
    tol = 1e-9 if path == "fp64" else 2e-3 * 9 / s
    assert (D[fin] <= fw[fin] + tol).all()


def test_two_node_chain_closed_form_on_gpu(gpu_lib):
    W = np.array([[0.0, 0.5], [np.inf, 0.0]], dtype=np.float32)
    D, _ = _apsp(gpu_lib, W, 1.0, P512, "fp64", T=2)
    assert math.isclose(D[0, 1], float(np.float32(0.5)) - 2 * math.log(2) / 512, rel_tol=1e-12)
    assert D[1, 0] == np.inf and D[0, 0] == 0 and D[1, 1] == 0


def test_apsp_validate_flag(gpu_lib):
    import torch

    W = torch.rand(32, 32, device="cuda")
    W[3, 4] = -1.0
    with pytest.raises(gpu_lib.MaxTimesError) as e:
        gpu_lib.apsp(W, validate=True, P=[1, 2])
    assert e.value.status == 2
    W[3, 4] = float("inf")  # no edge: allowed
    gpu_lib.apsp(W, validate=True, P=[1, 2])


@pytest.mark.slow
def test_er2048_fp64_full_parity(gpu_lib):
    """ER n=2048, p=0.05, U[0,10) weights, s=1, 11 squarings, P={1..512}:
    the whole GPU run against the oracle's whole run."""
    cfg = config(2)
    print("[apsp] ER n=2048 fp64 full", flush=True)
    D, ps = _apsp(gpu_lib, cfg["W"], cfg["s"], cfg["P"], "fp64", T=cfg["T"])
    ref = oracle.apsp_estimate(cfg["W"], cfg["s"], cfg["P"], TAU["fp64"], T=cfg["T"])
    fin = np.isfinite(ref["D"])
    assert np.array_equal(np.isfinite(D), fin)
    err = np.abs(D[fin] - ref["D"][fin]).max()
    print(f"max |D_gpu - D_oracle| = {err:.3e}", flush=True)
    assert err <= 1e-5
    assert np.array_equal(ps, ref["pstar_idx_last"])


@pytest.mark.slow
def test_rgg16384_bf16_first_squaring_rows_and_properties(gpu_lib):
    """RGG n=16384, radius 0.02, s=0.35: (a) the first squaring on 128
    sampled rows against the oracle computed from W itself; (b) the full
    14-squaring run against Dijkstra from 8 sources (reachability, zero
    diagonal, estimated distance <= exact distance within the path's
    rounding)."""
    cfg = config(5)
    W, s, P = cfg["W"], cfg["s"], cfg["P"]
    n = W.shape[0]
    rows = np.random.default_rng(5005).choice(n, 128, replace=False)
    print("[apsp] RGG n=16384 bf16 first squaring", flush=True)
    X1, _ = _apsp(gpu_lib, W, s, P, "bf16", T=1, raw=True)
    X0 = oracle.to_maxtimes(W, s)
    ref = oracle.pnorm_estimate_rows(X0, X0, P, TAU["bf16"], rows)
    Xr = np.minimum(ref["C"], 1.0)
    Xr[np.arange(len(rows)), rows] = 1.0
    _check_x(X1[rows], Xr, 2e-3)
    del X0, ref
    print("[apsp] RGG n=16384 bf16 full", flush=True)
    D, _ = _apsp(gpu_lib, W, s, P, "bf16", T=cfg["T"])
    src = rows[:8]
    dj = oracle.dijkstra(W, src)
    fin = np.isfinite(dj)
    assert np.array_equal(np.isfinite(D[src]), fin)
    assert (D[src, src] == 0).all()
    assert (D[src][fin] <= dj[fin] + 0.05).all()
