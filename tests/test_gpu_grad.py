"""GPU parity of the hand-written adjoint (maxtimes_estimate_backward) with
the oracle's FP64 analytic gradient (p* held fixed), Euler's identity on the
GPU outputs, and the autograd wiring."""

import numpy as np
import pytest

import oracle
from parity import TAU
from workloads import config, gradient_case, lognormal_product

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-5, "bf16": 2e-3}


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _gpu_grad(mt, A, B, G, P, path):
    Ad, Bd, Gd = _dev(A), _dev(B), _dev(G)
    split = 4096 if path == "bf16" else None
    C, ps = mt.estimate(Ad, Bd, P=P, path=path, split_max_p=split, return_pstar=True)
    dA, dB = mt.estimate_backward(Ad, Bd, Gd, C, ps, P, path=path)
    return (C.cpu().numpy().astype(np.float64), ps.cpu().numpy(),
            dA.cpu().numpy().astype(np.float64), dB.cpu().numpy().astype(np.float64))


def _check(got, ref, tol):
    """Norm-wise relative error <= tol, and elementwise with an absolute
    floor of 1e-3 * max |ref| (fp64: tol * max |ref|)."""
    ref = np.asarray(ref)
    nrm = np.linalg.norm(ref)
    rel = np.linalg.norm(got - ref) / max(nrm, 1e-300)
    assert rel <= tol, f"norm-wise relative error {rel:.3e} > {tol}"
    floor = (1e-3 if tol > 1e-4 else tol) * np.abs(ref).max()
    err = np.abs(got - ref) - tol * np.abs(ref)
    assert (err <= floor).all(), f"elementwise: max excess {err.max():.3e} over floor {floor:.3e}"
    return rel


CASES = [(1, 33, 47, 29), (2, 64, 64, 64), (1, 130, 70, 257), (3, 100, 128, 90)]


@pytest.mark.parametrize("shape", CASES)
@pytest.mark.parametrize("path", ["fp64", "bf16"])
@pytest.mark.parametrize("P", [[16], [1, 2, 4, 8, 16, 32, 64]])
def test_gradient_parity_uniform(gpu_lib, shape, path, P):
    b, m, k, n = shape
    print(f"[grad] uniform {path} {shape} P={P}", flush=True)
    dt = np.float64 if path == "fp64" else np.float32
    A, B, G = gradient_case(b, m, k, n, seed=sum(shape), dtype=dt)
    if b == 1:
        A, B, G = A[0], B[0], G[0]
    C, ps, dA, dB = _gpu_grad(gpu_lib, A, B, G, P, path)
    ref = oracle.pnorm_estimate(A, B, P, TAU[path])
    assert np.array_equal(ps, ref["pstar_idx"])
    rA, rB = oracle.pnorm_grad(A, B, G, P, ref["pstar_idx"])
    eA = _check(dA, rA, TOL[path])
    eB = _check(dB, rB, TOL[path])
    print(f"   rel err dA {eA:.2e} dB {eB:.2e}", flush=True)


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_gradient_parity_spread_pstar(gpu_lib, path):
    """Moderate dynamic range: entries use several p; the adjoint runs one
    product per used p."""
    A, B = lognormal_product(90, 120, 70, seed=77, sigma=1.5)
    if path == "fp64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    G = np.random.default_rng(78).standard_normal((90, 70)).astype(A.dtype)
    P = [1, 2, 4, 8, 16, 32, 64, 128]
    C, ps, dA, dB = _gpu_grad(gpu_lib, A, B, G, P, path)
    ref = oracle.pnorm_estimate(A, B, P, TAU[path])
    same = ps == ref["pstar_idx"]
    print(f"[grad] spread {path}: p* values {np.unique(ps)}, agree {same.mean():.4f}", flush=True)
    assert same.all(), "p* differs from the oracle; the comparison needs identical p*"
    rA, rB = oracle.pnorm_grad(A, B, G, P, ref["pstar_idx"])
    _check(dA, rA, TOL[path])
    _check(dB, rB, TOL[path])


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_euler_identity_on_gpu(gpu_lib, path):
    """sum_k A_ik dA_ik = sum_j G_ij C_ij and sum_k B_kj dB_kj = sum_i G_ij C_ij."""
    A, B, G = gradient_case(2, 96, 160, 80, seed=5, dtype=np.float64 if path == "fp64" else np.float32)
    C, ps, dA, dB = _gpu_grad(gpu_lib, A, B, G, [1, 2, 4, 8, 16, 32, 64], path)
    GC = G.astype(np.float64) * C
    tol = 1e-9 if path == "fp64" else 2e-3
    scale = np.abs(GC).sum(axis=2).max()
    assert np.abs((A * dA).sum(2) - GC.sum(2)).max() <= tol * scale
    assert np.abs((B * dB).sum(1) - GC.sum(1)).max() <= tol * np.abs(GC).sum(axis=1).max()


def test_autograd_matches_backward_call(gpu_lib):
    import torch

    A, B, G = gradient_case(1, 40, 50, 30, seed=9)
    Ad = _dev(A[0]).requires_grad_(True)
    Bd = _dev(B[0]).requires_grad_(True)
    Gd = _dev(G[0])
    C = gpu_lib.estimate(Ad, Bd, P=[1, 2, 4, 8, 16], path="bf16")
    (C * Gd).sum().backward()
    C2, ps = gpu_lib.estimate(Ad.detach(), Bd.detach(), P=[1, 2, 4, 8, 16], path="bf16",
                              split_max_p=4096, return_pstar=True)
    dA, dB = gpu_lib.estimate_backward(Ad.detach(), Bd.detach(), Gd, C2, ps, [1, 2, 4, 8, 16], path="bf16")
    assert torch.equal(Ad.grad, dA) and torch.equal(Bd.grad, dB)


def test_backward_rejects_norm_correct(gpu_lib):
    import torch

    A = torch.rand(8, 8, device="cuda")
    C, ps = gpu_lib.estimate(A, A, return_pstar=True)
    with pytest.raises(gpu_lib.MaxTimesError) as e:
        gpu_lib.estimate_backward(A, A, A, C, ps, [1, 2, 4, 8, 16, 32, 64], flags=2)
    assert e.value.status == 5


@pytest.mark.slow
@pytest.mark.parametrize("which", ["fixed16", "selected"])
def test_config4_full_gradient(gpu_lib, which):
    """64 x (512 x 512) products, G ~ N(0,1): the full GPU gradient against
    the oracle's full FP64 gradient, at fixed p = 16 and with selected p*."""
    cfg = config(4)
    A, B, G = cfg["A"], cfg["B"], cfg["G"]
    P = cfg["P_fixed"] if which == "fixed16" else cfg["P"]
    print(f"[grad] config 4 {which}", flush=True)
    C, ps, dA, dB = _gpu_grad(gpu_lib, A, B, G, P, "bf16")
    ref = oracle.pnorm_estimate(A, B, P, TAU["bf16"])
    assert np.array_equal(ps, ref["pstar_idx"])
    rA, rB = oracle.pnorm_grad(A, B, G, P, ref["pstar_idx"])
    eA = _check(dA, rA, TOL["bf16"])
    eB = _check(dB, rB, TOL["bf16"])
    print(f"   rel err dA {eA:.2e} dB {eB:.2e}", flush=True)
