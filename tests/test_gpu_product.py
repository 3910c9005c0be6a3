"""GPU parity of the p-norm (max, x) product estimate with the oracle,
through the C ABI (via the thin binding), at sizes the oracle finishes in
seconds that span several tiles and ragged tails, plus edge cases."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import lognormal_product, uniform_product

pytestmark = pytest.mark.gpu

P64 = [1, 2, 4, 8, 16, 32, 64]
P128 = P64 + [128]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# "fp64" takes the one-kernel path for products of at most 2^25
# multiply-adds (most below), "fp64_general" the general one (planes, MFMA
# GEMM, sparse tail, root pass) with the one-kernel path turned off
PATHS = ["fp64", "fp64_general", "bf16"]


def _real(path):
    return "fp64" if path.startswith("fp64") else path


def _run(mt, A, B, P, path, **kw):
    old = mt.small_product_limit()
    if path == "fp64_general":
        mt.set_small_product_limit(0)
    try:
        C, ps = mt.estimate(_dev(A), _dev(B), P=P, path=_real(path), return_pstar=True, **kw)
    finally:
        mt.set_small_product_limit(old)
    return C.cpu().numpy(), ps.cpu().numpy()


SHAPES = [(1, 1, 1), (5, 7, 3), (64, 64, 64), (300, 77, 130), (257, 513, 255), (256, 1000, 512)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("path", PATHS)
def test_uniform_parity(gpu_lib, shape, path):
    m, k, n = shape
    print(f"[parity] uniform {path} {shape}", flush=True)
    A, B = uniform_product(m, k, n, seed=m * 7 + k * 3 + n)
    dt = np.float64 if path.startswith("fp64") else np.float32
    A, B = A.astype(dt), B.astype(dt)
    C, ps = _run(gpu_lib, A, B, P64, path)
    ref = oracle.pnorm_estimate(A, B, P64, TAU[_real(path)])
    st = compare_estimate(C, ps, ref, P64, _real(path))
    assert st["flips"] == 0


@pytest.mark.parametrize("shape", [(200, 300, 100), (512, 512, 512), (129, 2050, 67)])
@pytest.mark.parametrize("path", PATHS)
def test_lognormal_parity(gpu_lib, shape, path):
    """Large dynamic range: p* spreads over the family and flips at tau
    occur; the band rule arbitrates them."""
    m, k, n = shape
    print(f"[parity] lognormal {path} {shape}", flush=True)
    A, B = lognormal_product(m, k, n, seed=100 + m)
    C, ps = _run(gpu_lib, A, B, P128, path)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[_real(path)])
    st = compare_estimate(C, ps, ref, P128, _real(path))
    print(st, flush=True)
    assert len(np.unique(ps)) >= 2


@pytest.mark.parametrize("path", PATHS)
def test_batched_parity(gpu_lib, path):
    A, B = uniform_product(70, 90, 40, seed=5, batch=3)
    dt = np.float64 if path.startswith("fp64") else np.float32
    A, B = A.astype(dt), B.astype(dt)
    print(f"[parity] batched {path}", flush=True)
    C, ps = _run(gpu_lib, A, B, P64, path)
    ref = oracle.pnorm_estimate(A, B, P64, TAU[_real(path)])
    compare_estimate(C, ps, ref, P64, _real(path))


@pytest.mark.parametrize("P", [[1], [2], [3, 5, 7], [16], [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]])
@pytest.mark.parametrize("path", PATHS)
def test_other_families(gpu_lib, P, path):
    """Single p, non-power-of-two p and a long family."""
    A, B = lognormal_product(96, 160, 80, seed=len(P) + P[-1], sigma=1.0)
    if path.startswith("fp64"):
        A, B = A.astype(np.float64), B.astype(np.float64)
    print(f"[parity] family {P} {path}", flush=True)
    C, ps = _run(gpu_lib, A, B, P, path)
    ref = oracle.pnorm_estimate(A, B, P, TAU[_real(path)])
    compare_estimate(C, ps, ref, P, _real(path))


@pytest.mark.parametrize("path", PATHS)
def test_closed_forms_on_gpu(gpu_lib, path):
    """All-ones: C = k^(1/p_max); one-hot rows: C exact; P = {1}: A @ B."""
    dt = np.float64 if path.startswith("fp64") else np.float32
    tol = 1e-12 if path.startswith("fp64") else 2e-3
    k = 300
    C, ps = _run(gpu_lib, np.ones((40, k), dt), np.ones((k, 50), dt), P64, path)
    np.testing.assert_allclose(C, k ** (1 / 64), rtol=tol)
    assert (ps == len(P64) - 1).all()
    rng = np.random.default_rng(3)
    A = np.zeros((64, 96), dt)
    A[np.arange(64), rng.integers(0, 96, 64)] = rng.random(64) + 0.1
    B = rng.random((96, 33)).astype(dt)
    C, _ = _run(gpu_lib, A, B, P64, path)
    np.testing.assert_allclose(C, oracle.exact_maxtimes(A, B), rtol=tol)
    A = rng.random((50, 70)).astype(dt)
    B = rng.random((70, 30)).astype(dt)
    C, _ = _run(gpu_lib, A, B, [1], path)
    np.testing.assert_allclose(C, A.astype(np.float64) @ B.astype(np.float64), rtol=1e-12 if path.startswith("fp64") else 5e-5)


@pytest.mark.parametrize("path", PATHS)
def test_zero_rows_and_empty_inner(gpu_lib, path):
    import torch

    dt = np.float64 if path.startswith("fp64") else np.float32
    A, B = uniform_product(33, 20, 17, seed=9)
    A, B = A.astype(dt), B.astype(dt)
    A[4] = 0
    B[:, 3] = 0
    C, ps = _run(gpu_lib, A, B, P64, path)
    assert (C[4] == 0).all() and (C[:, 3] == 0).all()
    assert (ps[4] == 255).all() and (ps[:, 3] == 255).all()
    Ce, pe = gpu_lib.estimate(torch.zeros((5, 0), dtype=torch.float32, device="cuda"),
                              torch.zeros((0, 6), dtype=torch.float32, device="cuda"),
                              P=P64, path=_real(path), return_pstar=True)
    assert (Ce.cpu().numpy() == 0).all() and (pe.cpu().numpy() == 255).all()


@pytest.mark.parametrize("path", PATHS)
def test_norm_correct_and_clamp(gpu_lib, path):
    A, B = uniform_product(80, 120, 60, seed=11)
    dt = np.float64 if path.startswith("fp64") else np.float32
    A, B = A.astype(dt), B.astype(dt)
    C, ps = _run(gpu_lib, A, B, P64, path, norm_correct=True)
    ref = oracle.pnorm_estimate(A, B, P64, TAU[_real(path)], norm_correct=True)
    compare_estimate(C, ps, ref, P64, _real(path), norm_k=120)
    C2, _ = _run(gpu_lib, A * 3, B, P64, path, clamp=True)
    assert C2.max() <= 1.0


def test_validate_flag_reports_domain_errors(gpu_lib):
    import torch

    for bad in (-1.0, float("nan"), float("inf")):
        A = torch.rand(16, 16, device="cuda")
        A[3, 5] = bad
        B = torch.rand(16, 16, device="cuda")
        with pytest.raises(gpu_lib.MaxTimesError) as e:
            gpu_lib.estimate(A, B, validate=True)
        assert e.value.status == 2
        with pytest.raises(gpu_lib.MaxTimesError):
            gpu_lib.estimate(B, A, validate=True)
    A = torch.rand(16, 16, device="cuda")
    gpu_lib.estimate(A, A, validate=True)


@pytest.mark.parametrize("path", PATHS)
def test_deterministic(gpu_lib, path):
    A, B = lognormal_product(300, 700, 260, seed=13)
    C1, p1 = _run(gpu_lib, A, B, P128, path)
    C2, p2 = _run(gpu_lib, A, B, P128, path)
    assert np.array_equal(C1.view(np.uint32), C2.view(np.uint32)) and np.array_equal(p1, p2)


def test_fp64_input_on_bf16_path_and_fp32_on_fp64_path(gpu_lib):
    A, B = uniform_product(100, 130, 90, seed=15)
    C, ps = _run(gpu_lib, A, B, P64, "bf16")  # FP64 storage, BF16 ring products
    assert C.dtype == np.float64
    compare_estimate(C, ps, oracle.pnorm_estimate(A, B, P64, TAU["bf16"]), P64, "bf16")
    Af, Bf = A.astype(np.float32), B.astype(np.float32)
    C, ps = _run(gpu_lib, Af, Bf, P64, "fp64")  # FP32 storage, FP64 ring products
    assert C.dtype == np.float32
    ref = oracle.pnorm_estimate(Af, Bf, P64, TAU["fp64"])
    stats = compare_estimate(C.astype(np.float64), ps, ref, P64, "fp64")
    assert stats["max_rel"] < 1e-6  # FP32 storage of the output


def test_timing_facility_sees_kernels(gpu_lib):
    import torch

    A = torch.rand(512, 512, device="cuda")
    gpu_lib.timing_reset()
    gpu_lib.timing_enable(True)
    try:
        gpu_lib.estimate(A, A, path="bf16")
        ms, n = gpu_lib.timing_read("mt_pfamily_gemm_bf16")
    finally:
        gpu_lib.timing_enable(False)
        gpu_lib.timing_reset()
    assert n == 1 and ms > 0


def test_timing_span_on_the_device_clock(gpu_lib):
    """The GEMM's span on the device's real-time counter: one per timed
    launch, positive, inside the launch's events and the host's wall time,
    and the work counters unchanged by it."""
    import time

    import torch

    A = torch.rand(2048, 2048, device="cuda")
    gpu_lib.estimate(A, A, path="bf16")
    torch.cuda.synchronize()
    gpu_lib.timing_reset()
    gpu_lib.timing_enable(True)
    try:
        t0 = time.perf_counter()
        for _ in range(3):
            gpu_lib.estimate(A, A, path="bf16")
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        ev_ms, ev_n = gpu_lib.timing_read("mt_pfamily_gemm_bf16")
        sp_ms, sp_n = gpu_lib.timing_span("mt_pfamily_gemm_bf16")
        work = gpu_lib.timing_work("mt_pfamily_gemm_bf16")
        none_ms, none_n = gpu_lib.timing_span("mt_rowmax")  # counts no work, records no span
    finally:
        gpu_lib.timing_enable(False)
        gpu_lib.timing_reset()
    print(f"span {sp_ms:.4f} ms, events {ev_ms:.4f} ms, wall {wall_ms:.3f} ms", flush=True)
    assert ev_n == 3 and sp_n == 3
    assert 0 < sp_ms <= ev_ms + 0.005 and sp_ms < wall_ms
    assert work >= 3 * 2.0 * 2048 ** 3  # at least one segment per launch
    assert none_n == 0 and none_ms == 0.0


@pytest.mark.parametrize("shape", [(1, 1, 1), (70, 33, 130), (3, 200, 64, 90)])
def test_exact_kernel_matches_oracle(gpu_lib, shape):
    """The exact (max, x) product kernel (Alg. 2) against the oracle."""
    import torch

    if len(shape) == 3:
        A, B = uniform_product(*shape, seed=21)
    else:
        A, B = uniform_product(*shape[1:], seed=21, batch=shape[0])
    for dt, tol in ((np.float64, 0.0), (np.float32, 6e-8)):
        Ad, Bd = torch.from_numpy(A.astype(dt)).cuda(), torch.from_numpy(B.astype(dt)).cuda()
        E = gpu_lib.exact(Ad, Bd).cpu().numpy().astype(np.float64)
        ref = oracle.exact_maxtimes(A.astype(dt), B.astype(dt))
        np.testing.assert_allclose(E, ref, rtol=tol, atol=0)
