"""A forward tile stops once every entry of it has found p* (the smaller p of
the family cannot change a decided entry, Sec. 1: p* is the largest stable
p).  Checks that the results still match the oracle and, through the
executed-flop counters of the timing facility, that the work done is one
family entry when every entry is decided at the largest p and the whole
family when some entry in every tile needs the smallest p."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P128 = [1, 2, 4, 8, 16, 32, 64, 128]
SHAPE = (300, 257, 290)
EPS = 1e-20


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def high_case(m, k, n, dtype, seed=5):
    """Every product term lies in [0.81, 1]: S_p >= tau at p = 128 for every
    entry, so p* = 128 everywhere."""
    rng = np.random.default_rng(seed)
    return (rng.uniform(0.9, 1.0, (m, k)).astype(dtype), rng.uniform(0.9, 1.0, (k, n)).astype(dtype))


def needy_case(m, k, n, dtype):
    """A_ik = 1 iff k = i mod K, B_kj = 1 iff k = (j + 1) mod K, EPS elsewhere.
    Entry (i, j) has one term 1 when i = j + 1 (mod K) and p* = 128 there;
    elsewhere two terms EPS and the rest EPS^2, so S_p ~ 2 EPS^p: stable only
    at p = 1 in BF16 (tau 1e-30) and up to p = 8 in FP64 (tau 1e-290)."""
    A = np.full((m, k), EPS, dtype=dtype)
    A[np.arange(m), np.arange(m) % k] = 1.0
    B = np.full((k, n), EPS, dtype=dtype)
    B[(np.arange(n) + 1) % k, np.arange(n)] = 1.0
    return A, B


def _run_counted(mt, A, B, path):
    kname = "mt_pfamily_gemm_" + ("bf16" if path == "bf16" else "f64")
    mt.timing_reset()
    mt.timing_enable(True)
    try:
        C, ps = mt.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True)
        work = mt.timing_work(kname)
        _, launches = mt.timing_read(kname)
    finally:
        mt.timing_enable(False)
        mt.timing_reset()
    assert launches == 1
    return C.cpu().numpy(), ps.cpu().numpy(), work


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_early_exit_work_and_parity(gpu_lib, path):
    m, k, n = SHAPE
    dt = np.float64 if path == "fp64" else np.float32
    print(f"[early-exit] {path} {SHAPE}", flush=True)
    res = {}
    for name, (A, B) in (("high", high_case(m, k, n, dt)), ("needy", needy_case(m, k, n, dt))):
        C, ps, work = _run_counted(gpu_lib, A, B, path)
        ref = oracle.pnorm_estimate(A, B, P128, TAU[path])
        st = compare_estimate(C, ps, ref, P128, path)
        assert st["flips"] == 0, (name, st)
        res[name] = (ps, work)
    ps_high, w_high = res["high"]
    ps_needy, w_needy = res["needy"]
    assert np.all(ps_high == P128.index(128))
    assert w_high > 0
    if path == "bf16":
        # needy: p* = 1 for most entries; every tile runs all 14 segments
        # (p = 1, 2, 4 split into three, 8 .. 128 one each); high: one segment
        assert np.count_nonzero(ps_needy == 0) > 0.9 * ps_needy.size
        assert w_needy == pytest.approx(14 * w_high, rel=0, abs=0)
    else:
        # needy: p* = 8 for most entries; five family entries (128 .. 8)
        assert np.count_nonzero(ps_needy == P128.index(8)) > 0.9 * ps_needy.size
        assert w_needy == pytest.approx(5 * w_high, rel=0, abs=0)


def test_timing_work_off_is_zero(gpu_lib):
    """Without timing no counters are taken."""
    A, B = high_case(64, 64, 64, np.float32)
    gpu_lib.timing_enable(False)
    gpu_lib.timing_reset()
    gpu_lib.estimate(_dev(A), _dev(B), P=P128, path="bf16")
    assert gpu_lib.timing_work("mt_pfamily_gemm") == 0.0
