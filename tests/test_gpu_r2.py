"""The r = 2 projection (Sec. 1; MT_FLAG_PROJECT_R2, FP64 path) against the
oracle: products, exactness on two distinct term values, APSP, and the
argument checks (BF16 path, backward)."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import lognormal_product, er_graph

pytestmark = pytest.mark.gpu

P64 = [1, 2, 4, 8, 16, 32, 64]
P512 = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("kind", ["lognormal", "uniform_cubed"])
def test_r2_product_parity(gpu_lib, kind):
    if kind == "lognormal":
        A, B = lognormal_product(120, 300, 110, seed=601)
        A, B = A.astype(np.float64), B.astype(np.float64)
    else:
        rng = np.random.default_rng(602)
        A, B = rng.random((2, 90, 257)) ** 3, rng.random((2, 257, 100))
    print(f"[r2] {kind} {A.shape}x{B.shape}", flush=True)
    C, ps = gpu_lib.estimate(_dev(A), _dev(B), P=P64, path="fp64", return_pstar=True, projection="r2")
    ref = oracle.pnorm_estimate(A, B, P64, TAU["fp64"], projection="r2")
    st = compare_estimate(C.cpu().numpy(), ps.cpu().numpy(), ref, P64, "fp64", projection="r2")
    print(st, flush=True)


def test_r2_two_values_exact(gpu_lib):
    """Each row of A has n1 terms a1 and n2 terms a2 against a column of ones
    in B: the projection returns a1 (times the scales) exactly."""
    rows = []
    want = []
    for n1, n2, a1, a2 in [(1, 3, 0.9, 0.6), (4, 20, 0.97, 0.2), (2, 2, 0.5, 0.45), (7, 1, 0.8, 0.1)]:
        u = np.zeros(32)
        u[:n1] = a1
        u[n1:n1 + n2] = a2
        rows.append(u * 3.0)
        want.append(3.0 * a1)
    A = np.array(rows)
    B = np.ones((32, 3))
    C = gpu_lib.estimate(_dev(A), _dev(B), P=P64, path="fp64", projection="r2").cpu().numpy()
    np.testing.assert_allclose(C, np.array(want)[:, None] * np.ones((1, 3)), rtol=1e-8)


def _apsp_raw(mt, W, T):
    import torch

    X, ps = mt.apsp(_dev(W), s=1.0, P=P512, path="fp64", raw=True, out_dtype=torch.float64, projection="r2",
                    n_squarings=T, return_pstar=True)
    return X.cpu().numpy(), ps.cpu().numpy()


def test_r2_apsp_stepwise_parity(gpu_lib):
    """Every squaring (Sec. 2.2) of the GPU's own X^(t-1) against the
    oracle's r = 2 estimate of it, clamped with the diagonal pinned, at the
    FP64 tolerance; entries whose rank decision sits at the threshold are
    arbitrated (tests/parity.py)."""
    W = er_graph(150, 0.05, 10.0, seed=603)
    n = W.shape[0]
    diag = np.eye(n, dtype=bool)
    T = oracle.default_squarings(n)
    flips = 0
    for t in range(1, T + 1):
        Xp, _ = _apsp_raw(gpu_lib, W, t - 1)
        Xt, pst = _apsp_raw(gpu_lib, W, t)
        ref = oracle.pnorm_estimate(Xp, Xp, P512, TAU["fp64"], projection="r2")
        assert (Xt[diag] == 1.0).all()
        st = compare_estimate(Xt, pst, ref, P512, "fp64", projection="r2", clamp=True, skip=diag)
        assert np.array_equal(Xt == 0, (ref["C"] == 0) & ~diag)
        flips += st["r2_rank_flips"]
        print(f"[r2 apsp] squaring {t}: {st}", flush=True)
    assert flips <= 1e-3 * T * n * n


def test_r2_rejections(gpu_lib):
    A = _dev(np.random.default_rng(604).random((8, 8)).astype(np.float32))
    with pytest.raises(gpu_lib.MaxTimesError) as e:
        gpu_lib.estimate(A, A, P=P64, path="bf16", projection="r2")
    assert e.value.status == 5
    with pytest.raises(ValueError):
        A64 = A.double().requires_grad_(True)
        gpu_lib.estimate(A64, A64, P=P64, path="fp64", projection="r2").sum().backward()
