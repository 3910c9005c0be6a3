"""GPU parity of the r = 1 projection (MT_FLAG_PROJECT_R1; Sec. 1, the norm
sequence projected onto one unique value) with the oracle, for the product
on both paths and for APSP, plus the properties the projection guarantees
(exact on tied top terms, never above the exact product, the unbiased APSP
chain) and its interplay with the tile early exit."""

import math

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import er_graph, lognormal_product, rgg_graph, uniform_product

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P64 = [1, 2, 4, 8, 16, 32, 64]
P128 = P64 + [128]
P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _run(mt, A, B, P, path, **kw):
    C, ps = mt.estimate(_dev(A), _dev(B), P=P, path=path, return_pstar=True, projection="r1", **kw)
    return C.cpu().numpy(), ps.cpu().numpy()


@pytest.mark.parametrize("shape", [(1, 1, 1), (64, 64, 64), (300, 77, 130), (257, 513, 255)])
@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_r1_uniform_parity(gpu_lib, shape, path):
    m, k, n = shape
    print(f"[r1] uniform {path} {shape}", flush=True)
    A, B = uniform_product(m, k, n, seed=31 + m + k + n)
    dt = np.float64 if path == "fp64" else np.float32
    A, B = A.astype(dt), B.astype(dt)
    C, ps = _run(gpu_lib, A, B, P64, path)
    ref = oracle.pnorm_estimate(A, B, P64, TAU[path], projection="r1")
    st = compare_estimate(C, ps, ref, P64, path, projection="r1")
    assert st["flips"] == 0


@pytest.mark.parametrize("shape", [(200, 300, 100), (512, 512, 512), (129, 2050, 67)])
@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_r1_lognormal_parity(gpu_lib, shape, path):
    m, k, n = shape
    print(f"[r1] lognormal {path} {shape}", flush=True)
    A, B = lognormal_product(m, k, n, seed=500 + m)
    C, ps = _run(gpu_lib, A, B, P128, path)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path], projection="r1")
    st = compare_estimate(C, ps, ref, P128, path, projection="r1")
    print(st, flush=True)
    E = oracle.exact_maxtimes(A, B)
    # never above the exact product beyond the path's rounding
    # (C is FP32 here: the FP64 path rounds its result once to FP32)
    assert np.all(C <= E * (1 + (1.2e-7 if path == "fp64" else 4e-3)))


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_r1_tied_terms_exact(gpu_lib, path):
    rng = np.random.default_rng(7)
    m, k, n, h = 96, 300, 80, 3
    A = np.zeros((m, k))
    for i in range(m):
        A[i, rng.choice(k, h, replace=False)] = 1.0
    B = np.zeros((k, n))
    B[np.any(A > 0, axis=0), :] = 1.0
    A *= rng.uniform(0.5, 3.0, (m, 1))
    B *= rng.uniform(0.5, 3.0, (1, n))
    dt = np.float64 if path == "fp64" else np.float32
    A, B = A.astype(dt), B.astype(dt)
    C, _ = _run(gpu_lib, A, B, P64, path)
    E = oracle.exact_maxtimes(A, B)
    np.testing.assert_allclose(C, E, rtol=1e-12 if path == "fp64" else 2e-3)


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_r1_batched_and_k0(gpu_lib, path):
    A, B = uniform_product(70, 40, 90, seed=9)
    A = np.stack([A, A * 0.5, A ** 3])
    B = np.stack([B, B ** 2, B * 3.0])
    dt = np.float64 if path == "fp64" else np.float32
    A, B = A.astype(dt), B.astype(dt)
    C, ps = _run(gpu_lib, A, B, P64, path)
    ref = oracle.pnorm_estimate(A, B, P64, TAU[path], projection="r1")
    compare_estimate(C, ps, ref, P64, path, projection="r1")
    C0, ps0 = _run(gpu_lib, np.zeros((5, 0), dt), np.zeros((0, 6), dt), P64, path)
    assert (C0 == 0).all() and (ps0 == oracle.PSTAR_NONE).all()


@pytest.mark.parametrize("n", [2, 64, 200, 333])
def test_r1_fp64_apsp_parity(gpu_lib, n):
    import torch

    W = er_graph(n, min(1.0, 8.0 / n), 10.0, seed=700 + n)
    print(f"[r1] apsp fp64 ER n={n}", flush=True)
    ref = oracle.apsp_estimate(W, 1.0, P512, TAU["fp64"], projection="r1")
    Wd = _dev(W)
    X = gpu_lib.apsp(Wd, s=1.0, P=P512, path="fp64", raw=True, out_dtype=torch.float64,
                     projection="r1").cpu().numpy()
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    rel = np.abs(X - Xo) / np.maximum(Xo, 1e-300)
    assert rel.max() <= 1e-5, rel.max()
    D = gpu_lib.apsp(Wd, s=1.0, P=P512, path="fp64", out_dtype=torch.float64,
                     projection="r1").cpu().numpy()
    fin = np.isfinite(ref["D"])
    assert np.array_equal(np.isfinite(D), fin)
    assert np.abs(D[fin] - ref["D"][fin]).max() <= 1e-5


@pytest.mark.parametrize("n,T", [(150, 1), (300, 1)])
def test_r1_bf16_apsp_parity_one_squaring(gpu_lib, n, T):
    W = rgg_graph(n, math.sqrt(20.0 / (math.pi * n)), 100.0, seed=800 + n)
    print(f"[r1] apsp bf16 RGG n={n} T={T}", flush=True)
    ref = oracle.apsp_estimate(W, 0.35, P128, TAU["bf16"], T=T, projection="r1")
    X = gpu_lib.apsp(_dev(W), s=0.35, P=P128, path="bf16", n_squarings=T, raw=True,
                     projection="r1").cpu().numpy().astype(np.float64)
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    rel = np.abs(X - Xo) / np.maximum(Xo, 1e-300)
    assert rel.max() <= 2e-3 * T, rel.max()


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_r1_apsp_chain_unbiased(gpu_lib, path):
    """Two tied terms (k = i and k = j) per squaring: the r = 1 estimate keeps
    the edge weight where the plain root shrinks it by ln 2 / (s p*)."""
    import torch

    w = 2.0
    W = np.array([[0.0, w], [np.inf, 0.0]], dtype=np.float32)
    P = P512 if path == "fp64" else P128
    D = gpu_lib.apsp(_dev(W), s=1.0, P=P, path=path, n_squarings=3, out_dtype=torch.float64,
                     projection="r1").cpu().numpy()
    tol = 1e-12 if path == "fp64" else 2e-3 / 1.0
    assert abs(D[0, 1] - w) <= tol * w
    assert np.isinf(D[1, 0]) and D[0, 0] == 0 and D[1, 1] == 0


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_r1_runs_one_more_family_entry(gpu_lib, path):
    """Every entry stable at the largest p: the plain estimate stops each tile
    after that p; the projection needs the next one (p = 64, one segment on
    either path), so exactly twice the work."""
    rng = np.random.default_rng(3)
    dt = np.float64 if path == "fp64" else np.float32
    A = rng.uniform(0.9, 1.0, (300, 257)).astype(dt)
    B = rng.uniform(0.9, 1.0, (257, 290)).astype(dt)
    kname = "mt_pfamily_gemm_" + ("bf16" if path == "bf16" else "f64")
    work = {}
    for proj in (None, "r1"):
        gpu_lib.timing_reset()
        gpu_lib.timing_enable(True)
        try:
            gpu_lib.estimate(_dev(A), _dev(B), P=P128, path=path, projection=proj)
            work[proj] = gpu_lib.timing_work(kname)
        finally:
            gpu_lib.timing_enable(False)
            gpu_lib.timing_reset()
    assert work[None] > 0 and work["r1"] == 2 * work[None]


def test_r1_has_no_autograd(gpu_lib):
    import torch

    A = torch.rand(8, 8, device="cuda", requires_grad=True)
    with pytest.raises(ValueError):
        gpu_lib.estimate(A, torch.rand(8, 8, device="cuda"), projection="r1")
