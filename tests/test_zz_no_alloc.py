"""maxtimes_estimate_noalloc: the estimate on the library's static scratch,
for callers that cannot allocate device memory.  Through the C ABI it must
give what maxtimes_estimate gives on a caller workspace (the same kernels on
the same inputs: bit for bit), on two calls in a row with the second smaller
(the scratch keeps the first call's contents), and both agree with the
oracle at the path's tolerance."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import lognormal_product

pytestmark = pytest.mark.gpu

P128 = [1, 2, 4, 8, 16, 32, 64, 128]


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("path,big,small", [
    ("bf16", (1, 1024, 1024, 1024), (1, 300, 257, 190)),
    ("fp64", (2, 256, 512, 384), (1, 129, 70, 33)),
])
def test_noalloc_equals_workspace_call_twice(gpu_lib, path, big, small):
    import torch

    mt = gpu_lib
    for t, (b, m, k, n) in enumerate((big, small)):
        print(f"[noalloc] {path} call {t} b={b} m={m} k={k} n={n}", flush=True)
        assert mt.workspace_size(b, m, k, n, P128, path=path) <= mt.NOALLOC_SCRATCH_BYTES
        A, B = lognormal_product(b * m, k, n * b, seed=600 + 7 * t + m)
        if b > 1:
            A = A.reshape(b, m, k)
            B = np.stack([B[:, i * n:(i + 1) * n] for i in range(b)])
        if path == "fp64":
            A, B = A.astype(np.float64), B.astype(np.float64)
        Ad, Bd = _dev(A), _dev(B)
        C0, ps0 = mt.estimate(Ad, Bd, P=P128, path=path, return_pstar=True)
        C1, ps1 = mt.estimate_noalloc(Ad, Bd, P=P128, path=path)
        torch.cuda.synchronize()
        assert torch.equal(ps0, ps1)
        assert torch.equal(C0, C1)
        ref = oracle.pnorm_estimate(A, B, P128, TAU[path])
        print(compare_estimate(C1.cpu().numpy(), ps1.cpu().numpy(), ref, P128, path), flush=True)


def test_noalloc_rejects_a_product_beyond_the_scratch(gpu_lib):
    import torch

    mt = gpu_lib
    A = torch.ones(2048, 2048, dtype=torch.float32, device="cuda")
    assert mt.workspace_size(1, 2048, 2048, 2048, P128, path="bf16") > mt.NOALLOC_SCRATCH_BYTES
    with pytest.raises(mt.MaxTimesError) as e:
        mt.estimate_noalloc(A, A, P=P128, path="bf16")
    assert e.value.status == 3 and "static scratch" in str(e.value)
    # a fitting call afterwards still works
    A2, B2 = lognormal_product(64, 96, 80, seed=77)
    C, ps = mt.estimate_noalloc(_dev(A2), _dev(B2), P=P128, path="bf16")
    ref = oracle.pnorm_estimate(A2, B2, P128, TAU["bf16"])
    compare_estimate(C.cpu().numpy(), ps.cpu().numpy(), ref, P128, "bf16")
