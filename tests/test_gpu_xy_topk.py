"""GPU parity of the top k of x + y (Sec. 2.3: algorithm E, the NormQueue and
the index recovery) against the oracle.

The ring results sigma^(p) (FFT on the GPU, direct convolution in the
oracle) are compared entry by entry within the FFT bound delta_p of the
max-convolution tests.  The pops subtract psi^p from sigma^(p), a
cancellation that turns 1e-15 differences of sigma into different later pops
on some inputs (the accumulation of error Sec. 3 reports), so the whole pop
sequence (values within 1e-6, diagonals and indices exactly) is compared on
inputs and depths whose sequence does not depend on rounding (checked on the
CPU by running the oracle's algorithm on numpy FFT ring results of three
lengths, which give the same sequence; `test_oracle_xy_topk.py`): uniform
lists on [0, 1] to rank 128.
Elsewhere the FFT's absolute rounding of small ring results leaves residuals
above tau after a diagonal is popped, whose roots then compete with the true
values (near one-hot lists show it within a few ranks), so there the first
pop is compared.  (That numpy's FFT at three lengths gives the same
sequence is necessary, not sufficient: on normal lists, n = 1024, whose
first 15 ranks are the same under numpy's three FFTs, the GPU's coarser
FFT rounding re-popped a diagonal at rank 13; `xy_robust`.)  The value
tolerance covers
the FFT rounding of a ring result near tau divided by p* (the numpy FFT run
differs from the direct one by up to 6e-9 on these inputs).  On any input the first pop,
the largest diagonal estimate, is compared.
"""

import math

import numpy as np
import pytest

import oracle
from oracle.xy_topk import exact_topk_xy, norm_queue, xy_topk_estimate

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
P24 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096]


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _sigma_gpu(mt, x, y, P):
    """sigma of both runs from the workspace of a k = 0 call (its documented
    layout)."""
    import torch

    n = x.size
    need = mt.xy_topk_workspace_size(n, 0, P)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    lib = mt.load_library()
    import ctypes

    o = mt._options(P, "fp64", None, None, 0)
    xd, yd = _dev(x), _dev(y)
    st = lib.xy_topk_estimate(mt._ptr(xd), mt._ptr(yd), mt._dtype_code(xd), n, 0, ctypes.byref(o), None, None,
                              None, None, mt._ptr(ws), need, mt._stream(xd.device))
    assert st == 0
    L = 2 * n - 1
    return ws[: 2 * len(P) * L * 8].view(torch.float64).reshape(2, len(P), L).cpu().numpy()


@pytest.mark.parametrize("n", [1, 5, 64, 700, 1024, 2048, 2049, 3000, 8192])
def test_ring_results_within_fft_bound(gpu_lib, n):
    """Lists up to n = 2048 transform in LDS; longer ones (to 8192) through
    global buffers."""
    rng = np.random.default_rng(9100 + n)
    x = rng.normal(0, 2, n)
    y = rng.uniform(-3, 3, n)
    sg = _sigma_gpu(gpu_lib, x, y, P24)
    N = max(16, 1 << math.ceil(math.log2(2 * n - 1))) if n > 1 else 16
    xs = np.exp(x - x.max())
    for run, yy in enumerate((y, y[::-1])):
        ys = np.exp(yy - yy.max())
        for q, p in enumerate(P24):
            ref = np.convolve(xs ** p, ys ** p)
            delta = 40.0 * math.log2(N) * U * np.linalg.norm(xs ** p) * np.linalg.norm(ys ** p)
            err = np.abs(sg[run, q] - ref)
            assert (err <= delta).all(), (run, p, err.max(), delta)


def _compare_sequence(mt, x, y, k, atol=1e-6):
    v, i, j, d = mt.xy_topk(_dev(x), _dev(y), k, P24, return_diag=True)
    ref = xy_topk_estimate(x, y, P24, k)
    np.testing.assert_array_equal(d.cpu().numpy(), ref["diag"])
    np.testing.assert_allclose(v.cpu().numpy(), ref["values"], rtol=0, atol=atol)
    np.testing.assert_array_equal(i.cpu().numpy(), ref["i"])
    np.testing.assert_array_equal(j.cpu().numpy(), ref["j"])
    return v.cpu().numpy(), i.cpu().numpy(), j.cpu().numpy()


def test_near_one_hot_first_pop_is_exact(gpu_lib):
    """One dominant term per diagonal: the first pop is the true maximum with
    its indices (deeper pops of such lists leave FFT residual ghosts)."""
    rng = np.random.default_rng(9200)
    n = 512
    x = np.full(n, -60.0)
    x[17] = 2.0
    y = rng.uniform(0, 3, n)
    v, i, j = _compare_sequence(gpu_lib, x, y, 1)
    ev, ei, ej = exact_topk_xy(x, y, 1)
    np.testing.assert_allclose(v, ev, rtol=0, atol=1e-6)
    np.testing.assert_array_equal(i, ei)
    np.testing.assert_array_equal(j, ej)


@pytest.mark.parametrize("n,seed,k", [(1024, 9600, 128), (1024, 9601, 128), (2048, 9700, 128), (3000, 9801, 128),
                                      (8192, 9800, 128)])
def test_uniform_unit_lists_full_sequence(gpu_lib, n, seed, k):
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, 1, n)
    y = rng.uniform(0, 1, n)
    v, i, j = _compare_sequence(gpu_lib, x, y, k)
    ev, ei, ej = exact_topk_xy(x, y, k)
    print(n, k, "indices found", int(((i == ei) & (j == ej)).sum()), "of", k, flush=True)


@pytest.mark.parametrize("n", [1024, 8192])
@pytest.mark.parametrize("dist", ["normal", "uniform40", "exponential"])
def test_first_pop_any_input(gpu_lib, dist, n):
    rng = np.random.default_rng(9400)
    if dist == "normal":
        x, y = rng.normal(0, 1, n), rng.normal(0, 1, n)
    elif dist == "uniform40":
        x, y = rng.uniform(0, 40, n), rng.uniform(0, 40, n)
    else:
        x, y = rng.exponential(1, n), rng.exponential(1, n)
    v, i, j = gpu_lib.xy_topk(_dev(x), _dev(y), 1, P24)
    ref = norm_queue(x, y, P24, 1)
    assert abs(v.cpu().numpy()[0] - ref["values"][0]) <= 1e-9
    # the largest value is bounded below by the true maximum
    assert v.cpu().numpy()[0] >= x.max() + y.max() - 1e-9


def test_fp32_inputs_and_edges(gpu_lib):
    import torch

    mt = gpu_lib
    rng = np.random.default_rng(9600)
    x = rng.uniform(0, 1, 1024).astype(np.float32)
    y = rng.uniform(0, 1, 1024).astype(np.float32)
    v, i, j, d = mt.xy_topk(_dev(x), _dev(y), 64, P24, return_diag=True)
    ref = xy_topk_estimate(x.astype(np.float64), y.astype(np.float64), P24, 64)
    np.testing.assert_array_equal(d.cpu().numpy(), ref["diag"])
    np.testing.assert_allclose(v.cpu().numpy(), ref["values"], rtol=0, atol=1e-6)
    np.testing.assert_array_equal(i.cpu().numpy(), ref["i"])
    np.testing.assert_array_equal(j.cpu().numpy(), ref["j"])
    # n = 1: one diagonal with one term, then nothing stable is left
    v, i, j = mt.xy_topk(_dev(np.array([0.5])), _dev(np.array([-0.25])), 3, P24)
    ref = xy_topk_estimate([0.5], [-0.25], P24, 3)
    np.testing.assert_allclose(v.cpu().numpy()[:1], [0.25], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(np.isneginf(v.cpu().numpy()), np.isneginf(ref["values"]))
    np.testing.assert_array_equal(i.cpu().numpy(), ref["i"])
    # k = 0: nothing to pop
    v, i, j = mt.xy_topk(_dev(x), _dev(y), 0, P24)
    assert v.numel() == 0
    # lengths beyond the longest transform are rejected before launch
    with pytest.raises(mt.MaxTimesError) as e:
        mt.xy_topk(torch.zeros(8193, dtype=torch.float64, device="cuda"),
                   torch.zeros(8193, dtype=torch.float64, device="cuda"), 4, P24)
    assert e.value.status == 5


def test_queue_over_every_diagonal_matches_the_candidate_queue(gpu_lib):
    # k <= 4096 pops both runs together over the min(k, 2n - 1) candidate
    # diagonals, keeping log psi; a larger k runs one wave per run over every
    # diagonal, keeping psi.  The same pops (diagonals and indices exactly);
    # values agree to the rounding of a log, which the subtraction psi^p
    # (p up to 4096, cancelling deep in the queue) grows to about 1e-11; the
    # first pop also against the oracle
    rng = np.random.default_rng(4242)
    xn = rng.uniform(0, 8, 300)
    yn = rng.uniform(0, 8, 300)
    x, y = _dev(xn), _dev(yn)
    a = gpu_lib.xy_topk(x, y, 4097, return_diag=True)
    # k = 4096 keeps the columns in the workspace (K = 599), k = 320 in LDS
    # (K = 320), k = 200 with a lane's slots in registers (K = 200)
    for kk in (4096, 320, 200):
        b = gpu_lib.xy_topk(x, y, kk, return_diag=True)
        for u, w in zip(a[1:], b[1:]):
            np.testing.assert_array_equal(u.cpu().numpy()[:kk], w.cpu().numpy())
        va, vb = a[0].cpu().numpy()[:kk], b[0].cpu().numpy()
        fin = np.isfinite(vb)
        np.testing.assert_array_equal(np.isfinite(va), fin)
        np.testing.assert_allclose(va[fin], vb[fin], rtol=1e-10, atol=0)
    b = gpu_lib.xy_topk(x, y, 4096, return_diag=True)
    o = xy_topk_estimate(xn, yn, P24, 1)
    np.testing.assert_allclose(b[0].cpu().numpy()[0], o["values"][0], rtol=0, atol=1e-9)
    assert b[3].cpu().numpy()[0] == o["diag"][0]


def test_largest_k_at_the_largest_n(gpu_lib):
    """n = 8192, k = 4096 (the sizes of Sec. 3 with the largest k of the
    candidate queue: K = 4096 candidates per run, 160 KiB of LDS): the first
    128 ranks of uniform lists on [0, 1] against the oracle (the depth whose
    sequence does not depend on rounding), and every rank the same as a call
    with a smaller k gives (the candidates are exact at every rank)."""
    rng = np.random.default_rng(9800)
    x = rng.uniform(0, 1, 8192)
    y = rng.uniform(0, 1, 8192)
    print("[xy] plain n=8192 k=4096", flush=True)
    v, i, j, d = gpu_lib.xy_topk(_dev(x), _dev(y), 4096, P24, return_diag=True)
    v, i, j, d = (t.cpu().numpy() for t in (v, i, j, d))
    ref = xy_topk_estimate(x, y, P24, 128)
    np.testing.assert_array_equal(d[:128], ref["diag"])
    np.testing.assert_allclose(v[:128], ref["values"], rtol=0, atol=1e-6)
    np.testing.assert_array_equal(i[:128], ref["i"])
    np.testing.assert_array_equal(j[:128], ref["j"])
    v2, i2, j2, d2 = (t.cpu().numpy() for t in gpu_lib.xy_topk(_dev(x), _dev(y), 1000, P24, return_diag=True))
    np.testing.assert_array_equal(d[:1000], d2)
    np.testing.assert_array_equal(i[:1000], i2)
    np.testing.assert_allclose(v[:1000], v2, rtol=1e-12, atol=0)
