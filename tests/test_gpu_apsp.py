"""GPU parity of the APSP estimate (Sec. 2.2) with the oracle's squaring loop, and
properties at full size (reachability, zero diagonal, the one-sided bound
against exact distances)."""

import math

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
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


def _step_parity(mt, W, s, P, path, t, rows=None):
    """Squaring t (Sec. 2.2 repeated squaring) on its own: the GPU's
    X^(t-1) (raw output of t - 1 squarings) goes into the oracle's estimate
    est(X^(t-1), X^(t-1)), clamped to 1 with the diagonal pinned to 1, and
    that is compared with the GPU's X^(t) (and its p*) on `rows` at the
    path's tolerance, with the band rule for p* flips.  Each squaring is
    held to the tolerance by itself; nothing is scaled with t."""
    Xp, _ = _apsp(mt, W, s, P, path, T=t - 1, raw=True)
    Xt, pst = _apsp(mt, W, s, P, path, T=t, raw=True)
    n = Xp.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    ref = oracle.pnorm_estimate_rows(Xp, Xp, P, TAU[path], rows)
    diag = np.zeros((len(rows), n), dtype=bool)
    diag[np.arange(len(rows)), rows] = True
    assert (Xt[rows][diag] == 1.0).all()
    st = compare_estimate(Xt[rows], pst[rows], ref, P, path, clamp=True, skip=diag)
    # reachability (an estimate is 0 exactly when every term is 0)
    assert np.array_equal(Xt[rows] == 0, (ref["C"] == 0) & ~diag)
    return st


@pytest.mark.parametrize("n,T", [(150, 1), (300, 2), (300, 9)])
def test_bf16_apsp_stepwise_parity(gpu_lib, n, T):
    """BF16 rounding of each squaring feeds the next, so every squaring is
    checked on the GPU's own input at the path's tolerance (2e-3)."""
    W = rgg_graph(n, math.sqrt(20.0 / (math.pi * n)), 100.0, seed=300 + n)
    for t in range(1, T + 1):
        print(f"[apsp] bf16 RGG n={n} squaring {t} of {T}", flush=True)
        print("   ", _step_parity(gpu_lib, W, 0.35, P128, "bf16", t), flush=True)


@pytest.mark.parametrize("n,T", [(64, 6), (333, 9)])
def test_fp64_apsp_stepwise_parity(gpu_lib, n, T):
    W = er_graph(n, min(1.0, 8.0 / n), 10.0, seed=210 + n)
    for t in range(1, T + 1):
        print(f"[apsp] fp64 ER n={n} squaring {t} of {T}", flush=True)
        _step_parity(gpu_lib, W, 1.0, P512, "fp64", t)


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


@pytest.fixture(scope="module")
def rgg16384():
    return config(5)


@pytest.mark.slow
@pytest.mark.parametrize("t", [1, 7, 14])
def test_rgg16384_bf16_stepwise_parity(gpu_lib, rgg16384, t):
    """RGG n = 16384, radius 0.02, s = 0.35, P = {1..128}, BF16: squarings
    t = 1, T/2 and T (T = 14) each on the GPU's own X^(t-1), 256 sampled
    rows against the oracle's estimate at the path's tolerance."""
    cfg = rgg16384
    n = cfg["W"].shape[0]
    rows = np.sort(np.random.default_rng(5005).choice(n, 256, replace=False))
    print(f"[apsp] RGG n=16384 bf16 squaring {t}", flush=True)
    print("   ", _step_parity(gpu_lib, cfg["W"], cfg["s"], cfg["P"], "bf16", t, rows), flush=True)


@pytest.mark.slow
def test_rgg16384_bf16_full_run_against_dijkstra(gpu_lib, rgg16384):
    """The full 14-squaring run against Dijkstra from 64 sources: the same
    reachability, a zero diagonal, and the estimate's (x, max) value at least
    the exact one (its distance at most the exact distance) up to the path's
    rounding, 2e-3 relative per squaring in (x, max) space."""
    cfg = rgg16384
    W, s, P, T = cfg["W"], cfg["s"], cfg["P"], cfg["T"]
    n = W.shape[0]
    src = np.sort(np.random.default_rng(5006).choice(n, 64, replace=False))
    print("[apsp] RGG n=16384 bf16 full", flush=True)
    D, _ = _apsp(gpu_lib, W, s, P, "bf16", T=T)
    dj = oracle.dijkstra(W, src)
    fin = np.isfinite(dj)
    assert np.array_equal(np.isfinite(D[src]), fin)
    assert (D[src, src] == 0).all()
    slack = -T * math.log1p(-2e-3) / s
    over = D[src][fin] - dj[fin]
    print(f"   largest excess over the exact distance {over.max():.3e} (bound {slack:.3e})", flush=True)
    assert (over <= slack).all()
