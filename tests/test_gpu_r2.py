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


def test_r2_apsp_parity(gpu_lib):
    import torch

    W = er_graph(150, 0.05, 10.0, seed=603)
    ref = oracle.apsp_estimate(W, 1.0, P512, TAU["fp64"], projection="r2")
    X = gpu_lib.apsp(_dev(W), s=1.0, P=P512, path="fp64", raw=True, out_dtype=torch.float64,
                     projection="r2").cpu().numpy()
    Xo = ref["X"]
    assert (X[Xo == 0] == 0).all() and (Xo[X == 0] == 0).all()
    assert (np.abs(X - Xo) / np.maximum(Xo, 1e-300)).max() <= 1e-5


def test_r2_rejections(gpu_lib):
    A = _dev(np.random.default_rng(604).random((8, 8)).astype(np.float32))
    with pytest.raises(gpu_lib.MaxTimesError) as e:
        gpu_lib.estimate(A, A, P=P64, path="bf16", projection="r2")
    assert e.value.status == 5
    with pytest.raises(ValueError):
        A64 = A.double().requires_grad_(True)
        gpu_lib.estimate(A64, A64, P=P64, path="fp64", projection="r2").sum().backward()
