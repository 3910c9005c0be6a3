"""Pins of the oracle's analytic gradient (CPU only): central finite
differences with p* frozen, the single-p = 1 case (the gradient of an
ordinary matrix product), k = 1, and Euler's identity for functions that
are positively homogeneous of degree 1."""

import numpy as np
import pytest

import oracle
from workloads import gradient_case, lognormal_product, uniform_product

P64 = [1, 2, 4, 8, 16, 32, 64]


def test_p1_is_matmul_gradient():
    rng = np.random.default_rng(70)
    A = rng.random((5, 7)) + 0.1
    B = rng.random((7, 4)) + 0.1
    G = rng.standard_normal((5, 4))
    out = oracle.pnorm_estimate(A, B, [1], 1e-290)
    dA, dB = oracle.pnorm_grad(A, B, G, [1], out["pstar_idx"])
    np.testing.assert_allclose(dA, G @ B.T, rtol=1e-12)
    np.testing.assert_allclose(dB, A.T @ G, rtol=1e-12)


def test_k1_outer_product():
    """k = 1: C_ij = A_i0 B_0j for every p, so dA = G B^T and dB = A^T G."""
    rng = np.random.default_rng(71)
    A = rng.random((6, 1)) + 0.1
    B = rng.random((1, 5)) + 0.1
    G = rng.standard_normal((6, 5))
    out = oracle.pnorm_estimate(A, B, P64, 1e-290)
    np.testing.assert_allclose(out["C"], A @ B, rtol=1e-13)
    dA, dB = oracle.pnorm_grad(A, B, G, P64, out["pstar_idx"])
    np.testing.assert_allclose(dA, G @ B.T, rtol=1e-12)
    np.testing.assert_allclose(dB, A.T @ G, rtol=1e-12)


@pytest.mark.parametrize("P", [[16], P64, [1, 2, 4, 8, 16, 32, 64, 128]])
def test_euler_identity(P):
    """C is positively homogeneous of degree 1 in row i of A and in column j
    of B, so sum_k A_ik dL/dA_ik = sum_j G_ij C_ij and
    sum_k B_kj dL/dB_kj = sum_i G_ij C_ij."""
    A, B = lognormal_product(9, 14, 7, seed=72)
    A, B = A.astype(np.float64), B.astype(np.float64)
    G = np.random.default_rng(73).standard_normal((9, 7))
    out = oracle.pnorm_estimate(A, B, P, 1e-30)
    dA, dB = oracle.pnorm_grad(A, B, G, P, out["pstar_idx"])
    GC = G * out["C"]
    np.testing.assert_allclose((A * dA).sum(1), GC.sum(1), rtol=1e-10, atol=1e-12 * np.abs(GC).sum())
    np.testing.assert_allclose((B * dB).sum(0), GC.sum(0), rtol=1e-10, atol=1e-12 * np.abs(GC).sum())


@pytest.mark.parametrize("P,seed", [([16], 80), (P64, 81), ([1, 2, 4, 8, 16, 32, 64, 128], 82)])
def test_central_finite_differences(P, seed):
    """Central differences (h = 1e-6, FP64) of L = sum(G * C) with p*
    frozen, on single coordinates and on random directions."""
    A, B = uniform_product(6, 8, 5, seed=seed)
    rng = np.random.default_rng(seed + 100)
    G = rng.standard_normal((6, 5))
    out = oracle.pnorm_estimate(A, B, P, 1e-30)
    idx = out["pstar_idx"]
    dA, dB = oracle.pnorm_grad(A, B, G, P, idx)

    def L(Ax, Bx):
        return float(np.sum(G * oracle.pnorm_forward_fixed(Ax, Bx, P, idx)))

    h = 1e-6
    for (i, k) in [(0, 0), (3, 5), (5, 7), (2, 2)]:
        E = np.zeros_like(A)
        E[i, k] = h
        fd = (L(A + E, B) - L(A - E, B)) / (2 * h)
        assert abs(fd - dA[i, k]) <= 1e-6 * max(1.0, abs(dA[i, k]))
    for (k, j) in [(0, 0), (7, 4), (3, 1)]:
        E = np.zeros_like(B)
        E[k, j] = h
        fd = (L(A, B + E) - L(A, B - E)) / (2 * h)
        assert abs(fd - dB[k, j]) <= 1e-6 * max(1.0, abs(dB[k, j]))
    for _ in range(4):
        VA = rng.standard_normal(A.shape)
        VB = rng.standard_normal(B.shape)
        fd = (L(A + h * VA, B + h * VB) - L(A - h * VA, B - h * VB)) / (2 * h)
        an = float(np.sum(dA * VA) + np.sum(dB * VB))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_batched_gradient_matches_per_item():
    A, B, G = gradient_case(3, 5, 6, 4, seed=90, dtype=np.float64)
    out = oracle.pnorm_estimate(A, B, P64, 1e-30)
    dA, dB = oracle.pnorm_grad(A, B, G, P64, out["pstar_idx"])
    for b in range(3):
        o = oracle.pnorm_estimate(A[b], B[b], P64, 1e-30)
        a1, b1 = oracle.pnorm_grad(A[b], B[b], G[b], P64, o["pstar_idx"])
        np.testing.assert_allclose(dA[b], a1, rtol=1e-14)
        np.testing.assert_allclose(dB[b], b1, rtol=1e-14)


def test_zero_entries_contribute_nothing():
    A = np.array([[1.0, 0.0], [0.0, 0.0]])
    B = np.array([[0.0, 1.0], [1.0, 0.0]])
    G = np.ones((2, 2))
    out = oracle.pnorm_estimate(A, B, [4], 1e-290)
    dA, dB = oracle.pnorm_grad(A, B, G, [4], out["pstar_idx"])
    assert np.all(np.isfinite(dA)) and np.all(np.isfinite(dB))
    # row 1 of C is 0 (zero row of A); only C[0,1] = 1 is nonzero
    np.testing.assert_allclose(dA, [[1.0, 0.0], [0.0, 0.0]], atol=1e-15)
