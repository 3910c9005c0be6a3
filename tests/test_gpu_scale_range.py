"""GPU parity where the row and column scales of the scaled ring call H'
(Sec. 2.1) leave the FP32 range while the estimate r_i c_j S^(1/p*) does not.

  * FP32 inputs whose r_i c_j exceeds 3.4e38 with finite outputs (the large
    entries of a row of A meet the small entries of a column of B);
  * FP64 inputs and outputs on the BF16 path with r and c near 1e+-50;
  * the same through the sparse tail (every entry handed over after the
    first p);
  * the adjoint (Sec. 4 notes the p-norm rings are differentiable) on both.

Every case is compared with the oracle at the path's tolerance (band rule for
p* flips), as everywhere else."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import crossed_product, wide_scale_product

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P128 = [1, 2, 4, 8, 16, 32, 64, 128]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.fixture
def knobs(gpu_lib):
    old_s, old_t = gpu_lib.search_start(), gpu_lib.tail_threshold()
    yield gpu_lib
    gpu_lib.set_search_start(old_s)
    gpu_lib.set_tail_threshold(old_t)


def test_reviewers_two_term_case(gpu_lib):
    """A = [1e20, 1e5], B = [1e5; 1e20]: r c = 1e40 (beyond FP32), the true
    maximum 1e25, the estimate sqrt(2) 1e25 at p* = 2."""
    A = np.array([[1e20, 1e5]], dtype=np.float32)
    B = np.array([[1e5], [1e20]], dtype=np.float32)
    ref = oracle.pnorm_estimate(A, B, P128, TAU["bf16"])
    C, ps = gpu_lib.estimate(_dev(A), _dev(B), P=P128, path="bf16", return_pstar=True)
    C, ps = C.cpu().numpy(), ps.cpu().numpy()
    assert np.isfinite(C).all()
    assert P128[int(ref["pstar_idx"][0, 0])] == 2
    compare_estimate(C, ps, ref, P128, "bf16")


@pytest.mark.parametrize("path", ["bf16", "fp64"])
@pytest.mark.parametrize("thr", [None, 65536])
def test_fp32_scales_beyond_fp32_product(knobs, path, thr):
    A, B = crossed_product(300, 515, 290, seed=901, big=1e20, small=1e5, dtype=np.float32)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path])
    rc = ref["r"][:, None] * ref["c"][None, :]
    assert (rc > 3.4e38).mean() > 0.5 and np.isfinite(ref["C"]).all() and ref["C"].max() < 1e36
    if thr is not None:
        knobs.set_tail_threshold(thr)  # every entry goes to the sparse tail after the first p
    print(f"[scale-range] crossed fp32 {path} thr={thr}", flush=True)
    C, ps = knobs.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True)
    C, ps = C.cpu().numpy(), ps.cpu().numpy()
    assert np.isfinite(C).all()
    print(compare_estimate(C, ps, ref, P128, path), flush=True)


@pytest.mark.parametrize("path", ["bf16", "fp64"])
@pytest.mark.parametrize("thr", [None, 65536])
def test_fp64_io_scales_near_1e50(knobs, path, thr):
    A, B = wide_scale_product(260, 300, 270, seed=902, decades=50)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path])
    assert ref["r"].min() < 1e-40 and ref["r"].max() > 1e40
    if thr is not None:
        knobs.set_tail_threshold(thr)
    print(f"[scale-range] 1e+-50 fp64 I/O {path} thr={thr}", flush=True)
    C, ps = knobs.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True)
    assert C.dtype.itemsize == 8
    C, ps = C.cpu().numpy(), ps.cpu().numpy()
    assert np.isfinite(C).all() and (C > 0).all()
    print(compare_estimate(C, ps, ref, P128, path), flush=True)


def _grad_check(got, ref, tol):
    nrm = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / nrm
    assert rel <= tol, f"norm-wise relative error {rel:.3e} > {tol}"
    # row by row of the output (each row has one scale): norm-wise within the row
    rows = np.linalg.norm(got - ref, axis=-1) / np.maximum(np.linalg.norm(ref, axis=-1), 1e-300)
    assert rows.max() <= 5 * tol, f"row-wise relative error {rows.max():.3e}"
    return rel


@pytest.mark.parametrize("path", ["bf16", "fp64"])
@pytest.mark.parametrize("case", ["crossed_fp32", "wide_fp64"])
def test_gradient_with_wide_scales(gpu_lib, path, case):
    """dA and dB against the oracle's FP64 gradient with p* frozen, where r c
    leaves FP32 (crossed FP32 inputs) or r and c sit near 1e+-50 (FP64)."""
    if case == "crossed_fp32":
        A, B = crossed_product(96, 130, 80, seed=903, big=1e20, small=1e5, dtype=np.float32)
    else:
        A, B = wide_scale_product(96, 130, 80, seed=904, decades=50)
    G = np.random.default_rng(905).standard_normal((A.shape[0], B.shape[1])).astype(A.dtype)
    P = [1, 2, 4, 8, 16, 32, 64]
    print(f"[scale-range] gradient {case} {path}", flush=True)
    Ad, Bd = _dev(A), _dev(B)
    split = 4096 if path == "bf16" else None
    C, ps = gpu_lib.estimate(Ad, Bd, P=P, path=path, split_max_p=split, return_pstar=True)
    dA, dB = gpu_lib.estimate_backward(Ad, Bd, _dev(G), C, ps, P, path=path)
    ps = ps.cpu().numpy()
    dA = dA.cpu().numpy().astype(np.float64)
    dB = dB.cpu().numpy().astype(np.float64)
    assert np.isfinite(dA).all() and np.isfinite(dB).all()
    rA, rB = oracle.pnorm_grad(A, B, G, P, ps)
    tol = 2e-3 if path == "bf16" else 1e-5
    eA = _grad_check(dA, rA, tol)
    # dB: the scale is per column of B, so compare column by column
    eB = _grad_check(dB.T, rB.T, tol)
    print(f"   rel err dA {eA:.2e} dB {eB:.2e}", flush=True)
