"""The one-kernel FP64-path estimate of small products (maxtimes_estimate for
b m k n up to the small-product limit): parity with the oracle at the FP64
path's tolerance on shapes around its 32 x 32 output tile and 32-element
inner chunks (ragged edges, one element, batches, zero lines, FP32 and FP64
storage, non-doubling families, the clamp and the k^(1/p*) correction),
agreement with the general path on the same inputs, the 256^3 product as
one launch, and the flags that keep a small product on the general path."""

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


def _est(mt, A, B, P, limit=None, **kw):
    old = mt.small_product_limit()
    if limit is not None:
        mt.set_small_product_limit(limit)
    try:
        C, ps = mt.estimate(_dev(A), _dev(B), P=P, path="fp64", return_pstar=True, **kw)
    finally:
        mt.set_small_product_limit(old)
    return C.cpu().numpy(), ps.cpu().numpy()


def _launches(mt, A, B, P, **kw):
    """Library launches of one estimate, by kernel name prefix."""
    import torch

    Ad, Bd = _dev(A), _dev(B)
    mt.estimate(Ad, Bd, P=P, path="fp64", **kw)
    torch.cuda.synchronize()
    mt.timing_reset()
    mt.timing_enable(True)
    try:
        mt.estimate(Ad, Bd, P=P, path="fp64", **kw)
        torch.cuda.synchronize()
        small = mt.timing_read("mt_small_product_f64")[1]
        every = mt.timing_read("mt_")[1]
    finally:
        mt.timing_enable(False)
        mt.timing_reset()
    return small, every


SHAPES = [(1, 1, 1), (1, 5, 1), (31, 33, 33), (32, 32, 32), (33, 1, 65), (64, 96, 64), (100, 700, 70),
          (3, 257, 2)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dist", ["uniform", "lognormal"])
def test_parity_with_the_oracle(gpu_lib, shape, dist):
    m, k, n = shape
    print(f"[small] {dist} {shape}", flush=True)
    if dist == "uniform":
        A, B = uniform_product(m, k, n, seed=m + 3 * k + 7 * n)
        P = P64
    else:
        A, B = lognormal_product(m, k, n, seed=m + 5 * k + n)
        P = P128
    A, B = A.astype(np.float64), B.astype(np.float64)
    C, ps = _est(gpu_lib, A, B, P)
    ref = oracle.pnorm_estimate(A, B, P, TAU["fp64"])
    print(compare_estimate(C, ps, ref, P, "fp64"), flush=True)


def test_batched_fp32_storage_and_zero_lines(gpu_lib):
    pairs = [lognormal_product(45, 70, 38, seed=61 + i) for i in range(4)]
    A = np.stack([a for a, _ in pairs]).astype(np.float32)
    B = np.stack([b for _, b in pairs]).astype(np.float32)
    A[1, 7] = 0.0
    B[2, :, 5] = 0.0
    C, ps = _est(gpu_lib, A, B, P128)
    assert C.dtype == np.float32
    ref = oracle.pnorm_estimate(A, B, P128, TAU["fp64"])
    compare_estimate(C.astype(np.float64), ps, ref, P128, "fp64")
    assert (C[1, 7] == 0).all() and (ps[1, 7] == 255).all()
    assert (C[2, :, 5] == 0).all() and (ps[2, :, 5] == 255).all()


@pytest.mark.parametrize("P", [[1], [3, 5, 7], [2, 6, 12, 48], [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]])
def test_other_families(gpu_lib, P):
    A, B = lognormal_product(50, 90, 41, seed=len(P) + P[-1], sigma=1.0)
    A, B = A.astype(np.float64), B.astype(np.float64)
    C, ps = _est(gpu_lib, A, B, P)
    ref = oracle.pnorm_estimate(A, B, P, TAU["fp64"])
    compare_estimate(C, ps, ref, P, "fp64")


def test_norm_correct_and_clamp(gpu_lib):
    A, B = uniform_product(70, 120, 60, seed=62)
    C, ps = _est(gpu_lib, A, B, P64, norm_correct=True)
    ref = oracle.pnorm_estimate(A, B, P64, TAU["fp64"], norm_correct=True)
    compare_estimate(C, ps, ref, P64, "fp64", norm_k=120)
    C2, _ = _est(gpu_lib, A * 3, B, P64, clamp=True)
    assert C2.max() <= 1.0 and (C2 == 1.0).any()


@pytest.mark.parametrize("shape", [(64, 64, 64), (100, 700, 70), (3, 257, 2)])
def test_equals_the_general_path(gpu_lib, shape):
    """Both paths sum the same FP64 terms in different orders: the same p*
    (outside entries whose S lies within rounding of tau) and the same C to
    a few ulps of FP64."""
    m, k, n = shape
    A, B = lognormal_product(m, k, n, seed=63 + m)
    A, B = A.astype(np.float64), B.astype(np.float64)
    C1, p1 = _est(gpu_lib, A, B, P128)
    C0, p0 = _est(gpu_lib, A, B, P128, limit=0)
    same = p1 == p0
    assert same.mean() > 0.999
    rel = np.abs(C1 - C0)[same] / np.maximum(np.abs(C0[same]), 1e-300)
    print(f"   max rel diff {rel.max():.2e}, p* differ at {(~same).sum()}", flush=True)
    assert rel.max() <= 1e-12


def test_config1_product_is_one_launch(gpu_lib):
    """The 256^3 FP64 product of uniform inputs (P = {1, ..., 64}) runs as one
    library kernel; with the one-kernel path off it takes the general path's
    launches; both against the oracle on the whole output."""
    from workloads import config

    c1 = config(1)
    A, B, P = c1["A"], c1["B"], c1["P"]
    small, every = _launches(gpu_lib, A, B, P)
    assert small == 1 and every == 1
    old = gpu_lib.small_product_limit()
    gpu_lib.set_small_product_limit(0)
    try:
        small0, every0 = _launches(gpu_lib, A, B, P)
    finally:
        gpu_lib.set_small_product_limit(old)
    print(f"   launches: one-kernel {every}, general {every0}", flush=True)
    assert small0 == 0 and every0 >= 5
    ref = oracle.pnorm_estimate(A, B, P, TAU["fp64"])
    C, ps = _est(gpu_lib, A, B, P)
    compare_estimate(C, ps, ref, P, "fp64")


@pytest.mark.parametrize("flags", [{"validate": True}, {"projection": "r1"}, {"balance": True}])
def test_other_options_stay_on_the_general_path(gpu_lib, flags):
    A, B = uniform_product(40, 50, 30, seed=64)
    small, every = _launches(gpu_lib, A, B, P64, **flags)
    assert small == 0 and every >= 3
