"""The sparse tail: a forward tile with few undecided entries hands them to a
second kernel that runs the remaining p for each entry alone (dot products
of plane rows).  Results must match the oracle whether the tail is off, at
its default threshold, or takes every undecided entry after the first p of
the family, on both paths, with the plain root and the r = 1 projection, for
products and APSP; and a tile that hands over must not run the remaining p
densely (executed GEMM work drops)."""

import math

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import lognormal_product, rgg_graph, er_graph

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P128 = [1, 2, 4, 8, 16, 32, 64, 128]
P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]
THRESHOLDS = [0, 512, 65536]


@pytest.fixture
def tail(gpu_lib):
    """Restores the default threshold after the test."""
    old = gpu_lib.tail_threshold()
    yield gpu_lib
    gpu_lib.set_tail_threshold(old)


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("thr", THRESHOLDS)
@pytest.mark.parametrize("projection", [None, "r1"])
@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_tail_parity(tail, path, projection, thr):
    tail.set_tail_threshold(thr)
    A, B = lognormal_product(300, 1000, 290, seed=77)
    A = np.stack([A, A[::-1]])
    B = np.stack([B, B[:, ::-1]])
    print(f"[tail] {path} {projection} thr={thr}", flush=True)
    C, ps = tail.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True, projection=projection)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path], projection=projection)
    st = compare_estimate(C.cpu().numpy(), ps.cpu().numpy(), ref, P128, path, projection=projection)
    print(st, flush=True)


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_tail_takes_work_from_the_gemm(tail, path):
    """Every entry stable at p = 128 except 200 entries of the first tile,
    which need small p: with the tail on, that tile stops after p = 128 like
    all the others (GEMM work equal to a case where every entry is stable at
    p = 128) and the 200 go to the tail; with it off, that tile runs on."""
    rng = np.random.default_rng(21)
    dt = np.float64 if path == "fp64" else np.float32
    m = k = n = 512
    A0 = rng.uniform(0.9, 1.0, (m, k))
    B0 = rng.uniform(0.9, 1.0, (k, n))
    A, B = A0.copy(), B0.copy()
    # entries (i < 5, j < 40): one term B[i, j] = 1e-20 with A[i, i] = 1, all
    # other terms 1e-20 * B -> S_p ~ 512e-20p (p* = 1 in BF16, 8 in FP64);
    # entries (i < 5, j >= 40) keep the term A[i, i] B[i, j] = 1
    for i in range(5):
        A[i, :] = 1e-20
        A[i, i] = 1.0
        B[i, :] = 1.0
        B[i, :40] = 1e-20
    kname = "mt_pfamily_gemm_" + ("bf16" if path == "bf16" else "f64")

    def run(Am, Bm, thr):
        tail.set_tail_threshold(thr)
        tail.timing_reset()
        tail.timing_enable(True)
        try:
            C, ps = tail.estimate(_dev(Am.astype(dt)), _dev(Bm.astype(dt)), P=P128, path=path, return_pstar=True)
            work = tail.timing_work(kname)
        finally:
            tail.timing_enable(False)
            tail.timing_reset()
        return C.cpu().numpy(), ps.cpu().numpy(), work

    _, ps_high, w_high = run(A0, B0, 256)
    assert (ps_high == P128.index(128)).all()
    C_on, ps_on, w_on = run(A, B, 256)
    C_off, ps_off, w_off = run(A, B, 0)
    ref = oracle.pnorm_estimate(A.astype(dt), B.astype(dt), P128, TAU[path])
    assert (ref["pstar_idx"] != P128.index(128)).sum() == 200
    compare_estimate(C_on, ps_on, ref, P128, path)
    compare_estimate(C_off, ps_off, ref, P128, path)
    assert w_on == w_high
    assert w_off > w_high


@pytest.mark.parametrize("thr", [0, 65536])
def test_tail_fp64_apsp_parity(tail, thr):
    import torch

    tail.set_tail_threshold(thr)
    W = er_graph(200, 0.04, 10.0, seed=901)
    ref = oracle.apsp_estimate(W, 1.0, P512, TAU["fp64"])
    X = tail.apsp(_dev(W), s=1.0, P=P512, path="fp64", raw=True, out_dtype=torch.float64).cpu().numpy()
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    assert (np.abs(X - Xo) / np.maximum(Xo, 1e-300)).max() <= 1e-5


@pytest.mark.parametrize("thr", [0, 65536])
def test_tail_bf16_apsp_one_squaring(tail, thr):
    tail.set_tail_threshold(thr)
    n = 300
    W = rgg_graph(n, math.sqrt(20.0 / (math.pi * n)), 100.0, seed=902)
    ref = oracle.apsp_estimate(W, 0.35, P128, TAU["bf16"], T=1)
    X = tail.apsp(_dev(W), s=0.35, P=P128, path="bf16", n_squarings=1, raw=True).cpu().numpy().astype(np.float64)
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    assert (np.abs(X - Xo) / np.maximum(Xo, 1e-300)).max() <= 2e-3


def test_tail_threshold_api(tail):
    with pytest.raises(tail.MaxTimesError):
        tail.set_tail_threshold(-1)
    tail.set_tail_threshold(0)
    small = tail.workspace_size(1, 512, 64, 512, P128, path="bf16")
    tail.set_tail_threshold(256)
    big = tail.workspace_size(1, 512, 64, 512, P128, path="bf16")
    assert big - small >= 2 * 4 * 256 * 16
    assert tail.tail_threshold() == 256
