"""The forward p search may start below the largest p (Sec. 1 fixes p* as the
largest stable p; the order of the search only changes the work).  From a
start s it goes down to the smallest p, deciding every entry not stable at
s, then up from the (s-1)-th largest p for the entries stable at s whose S
does not rule out a larger p (S_p' <= S_p^(p'/p) for terms in [0, 1]).

Checks, for every start on both paths: parity with the oracle (which
searches top-down) with the sparse tail off, at its default and taking
everything; APSP; that the r = 1 projection ignores the start; and, through
the executed-flop counters, the work of clean cases: a tile with nothing
open left after the start jumps straight to the way up, and one whose only
waiting entries are few hands them to the tail at once."""

import math

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import crossed_product, lognormal_product, rgg_graph, er_graph

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P128 = [1, 2, 4, 8, 16, 32, 64, 128]
P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]
EPS = 1e-20


@pytest.fixture
def knobs(gpu_lib):
    """Restores the search start and the tail threshold after the test."""
    old_s, old_t = gpu_lib.search_start(), gpu_lib.tail_threshold()
    yield gpu_lib
    gpu_lib.set_search_start(old_s)
    gpu_lib.set_tail_threshold(old_t)


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("thr", [0, 256, 65536])
@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_every_start_parity(knobs, path, thr):
    """Log-normal terms spread p* over the family; a second batch item of
    sixth powers (a log-normal six times as wide) moves it further down; a
    third, unscaled, has r c beyond FP32 (about 1e40) with outputs near 1e25."""
    A, B = lognormal_product(300, 1000, 290, seed=78)
    A = A.astype(np.float64)
    B = B.astype(np.float64)
    Ax, Bx = crossed_product(300, 1000, 290, seed=80, big=1e20, small=1e5, dtype=np.float64)
    A = np.stack([A, (A[::-1] / A.max()) ** 6, Ax])
    B = np.stack([B, (B[:, ::-1] / B.max()) ** 6, Bx])
    if path == "bf16":
        A, B = A.astype(np.float32), B.astype(np.float32)
    knobs.set_tail_threshold(thr)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path])
    assert len(np.unique(ref["pstar_idx"])) >= 5  # several p* in play
    base = None
    for s in range(len(P128)):
        knobs.set_search_start(s)
        print(f"[search-start] {path} thr={thr} s={s}", flush=True)
        C, ps = knobs.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True)
        C, ps = C.cpu().numpy(), ps.cpu().numpy()
        compare_estimate(C, ps, ref, P128, path)
        if base is None:
            base = ps
        else:
            # the same p* as the top-down search but for entries on tau
            assert (ps != base).sum() <= 2 + 1e-3 * ps.size


def test_start_beyond_family_is_clamped(knobs):
    """A start past the smallest p starts at the smallest p."""
    A, B = lognormal_product(100, 300, 90, seed=79)
    ref = oracle.pnorm_estimate(A, B, [1, 2, 4], TAU["bf16"])
    knobs.set_search_start(31)
    C, ps = knobs.estimate(_dev(A), _dev(B), P=[1, 2, 4], path="bf16", return_pstar=True)
    compare_estimate(C.cpu().numpy(), ps.cpu().numpy(), ref, [1, 2, 4], "bf16")
    with pytest.raises(knobs.MaxTimesError):
        knobs.set_search_start(-2)
    with pytest.raises(knobs.MaxTimesError):
        knobs.set_search_start(32)


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_r1_ignores_start(knobs, path):
    A, B = lognormal_product(200, 500, 190, seed=80)
    if path == "fp64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    out = []
    for s in (0, 3):
        knobs.set_search_start(s)
        C, ps = knobs.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True, projection="r1")
        out.append((C.cpu().numpy(), ps.cpu().numpy()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def high_case(m, k, n, dtype, seed=5):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.9, 1.0, (m, k)).astype(dtype), rng.uniform(0.9, 1.0, (k, n)).astype(dtype))


def needy_case(m, k, n, dtype):
    """One term 1 (p* = 128) where i = j + 1 mod K; elsewhere S_p ~ 2 EPS^p:
    stable up to p = 8 in FP64 (S_8 ~ 2e-160 < the rise threshold of p = 8,
    0.9 (tau / 2)^(1/2) ~ 6e-146, so decided at a start of p = 8)."""
    A = np.full((m, k), EPS, dtype=dtype)
    A[np.arange(m), np.arange(m) % k] = 1.0
    B = np.full((k, n), EPS, dtype=dtype)
    B[(np.arange(n) + 1) % k, np.arange(n)] = 1.0
    return A, B


def _work(mt, A, B, path, P=P128):
    kname = "mt_pfamily_gemm_" + ("bf16" if path == "bf16" else "f64")
    mt.timing_reset()
    mt.timing_enable(True)
    try:
        C, ps = mt.estimate(_dev(A), _dev(B), P=P, path=path, return_pstar=True)
        work = mt.timing_work(kname)
    finally:
        mt.timing_enable(False)
        mt.timing_reset()
    return C.cpu().numpy(), ps.cpu().numpy(), work


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_work_of_clean_cases(knobs, path):
    m, k, n = 300, 257, 290
    dt = np.float64 if path == "fp64" else np.float32
    Ah, Bh = high_case(m, k, n, dt)
    knobs.set_tail_threshold(0)
    knobs.set_search_start(0)
    _, ps, w1 = _work(knobs, Ah, Bh, path)  # one family entry
    assert (ps == P128.index(128)).all() and w1 > 0
    # p* = 128 everywhere, start at p = 16 (entry 3): every entry waits, none
    # is open -> 16, then straight up: 32, 64, 128
    knobs.set_search_start(3)
    C, ps, w = _work(knobs, Ah, Bh, path)
    assert (ps == P128.index(128)).all()
    assert w == 4 * w1
    compare_estimate(C, ps, oracle.pnorm_estimate(Ah, Bh, P128, TAU[path]), P128, path)
    if path == "fp64":
        An, Bn = needy_case(m, k, n, dt)
        ref = oracle.pnorm_estimate(An, Bn, P128, TAU[path])
        assert np.count_nonzero(ref["pstar_idx"] == P128.index(8)) > 0.9 * An.shape[0] * Bn.shape[1]
        # start at p = 8: the p* = 8 entries are decided there, the p* = 128
        # ones wait -> a tile holding some runs 8, then 16, 32, 64, 128 (no
        # 4, 2, 1), one holding none stops after 8.  FP64 tiles are 64 x 64
        # at this size.
        knobs.set_search_start(4)
        C, ps, w = _work(knobs, An, Bn, path)
        compare_estimate(C, ps, ref, P128, path)
        bm = 64
        ii, jj = np.meshgrid(np.arange(m), np.arange(n), indexing="ij")
        diag = (ii - jj - 1) % k == 0
        tiles = [(ti, tj) for ti in range(-(-m // bm)) for tj in range(-(-n // bm))]
        runs = [5 if diag[ti * bm:(ti + 1) * bm, tj * bm:(tj + 1) * bm].any() else 1 for ti, tj in tiles]
        assert 1 in runs and 5 in runs
        assert w * len(tiles) == w1 * sum(runs)
        # with the tail on, the few waiting entries of each tile go to it
        # right after the start
        knobs.set_tail_threshold(256)
        C, ps, w = _work(knobs, An, Bn, path)
        compare_estimate(C, ps, ref, P128, path)
        assert w == w1


@pytest.mark.parametrize("s", [2, 5])
def test_fp64_apsp_parity(knobs, s):
    import torch

    knobs.set_search_start(s)
    W = er_graph(200, 0.04, 10.0, seed=903)
    ref = oracle.apsp_estimate(W, 1.0, P512, TAU["fp64"])
    X = knobs.apsp(_dev(W), s=1.0, P=P512, path="fp64", raw=True, out_dtype=torch.float64).cpu().numpy()
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    assert (np.abs(X - Xo) / np.maximum(Xo, 1e-300)).max() <= 1e-5


@pytest.mark.parametrize("s", [2, 5])
def test_bf16_apsp_one_squaring(knobs, s):
    knobs.set_search_start(s)
    n = 300
    W = rgg_graph(n, math.sqrt(20.0 / (math.pi * n)), 100.0, seed=904)
    ref = oracle.apsp_estimate(W, 0.35, P128, TAU["bf16"], T=1)
    X = knobs.apsp(_dev(W), s=0.35, P=P128, path="bf16", n_squarings=1, raw=True).cpu().numpy().astype(np.float64)
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    assert (np.abs(X - Xo) / np.maximum(Xo, 1e-300)).max() <= 2e-3


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_pilot_start(knobs, path):
    """The default start (-1): a pilot picks it for a product of >= 2^22
    outputs.  The chosen start (workspace header, third word) is a plan
    index, the p* equal those of the top-down search up to entries on tau,
    and sampled rows match the oracle."""
    import torch

    m, k, n = 2048, 1024, 2304
    A, B = lognormal_product(m, k, n, seed=81)
    if path == "fp64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    dA, dB = _dev(A), _dev(B)
    res = {}
    for s in (-1, 0):
        knobs.set_search_start(s)
        ws = torch.zeros(knobs.workspace_size(1, m, k, n, P128, path=path), dtype=torch.uint8, device="cuda")
        C, ps = knobs.estimate(dA, dB, P=P128, path=path, return_pstar=True, workspace=ws)
        torch.cuda.synchronize()
        res[s] = (C.cpu().numpy(), ps.cpu().numpy(), int(ws[8:12].view(torch.int32).item()))
    chosen = res[-1][2]
    print(f"[pilot] {path}: start {chosen}", flush=True)
    assert 0 <= chosen < len(P128)
    assert res[0][2] == 0
    assert (res[-1][1] != res[0][1]).sum() <= 2 + 1e-4 * m * n
    rows = np.arange(0, m, 97)
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU[path], rows)
    compare_estimate(res[-1][0][rows], res[-1][1][rows], ref, P128, path)
