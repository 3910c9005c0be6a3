"""GPU parity of the max-convolution (Sec. 1, ring kernel H = FFT
convolution with tau = 1e-12, Sec. 2.1) against the oracle.

The oracle forms S_p by direct convolution (the plain definition of the ring
result); the GPU by FFT in FP64.  The two differ by the FFT's rounding, which
is absolute, not relative: per index and p the tests allow

    delta_p = 40 log2(N) u ||x'^p||_2 ||y'^p||_2,   u = 2^-53,

the normwise error bound of a radix-2 FFT (about 6.7 log2(N) u relative in
the 2-norm per transform with accurate twiddles) taken over the forward
transform, the product and the inverse, with a factor of 3 to spare, and
bounding each index by the 2-norm of the error.  The bar:

  * same p* on both sides: |z_gpu - z_ref| <= rx ry ((S + delta)^(1/p) -
    max(S - delta, 0)^(1/p)) + 1e-13 z_ref (+ one FP32 rounding for FP32
    output), S the oracle's ring result at that p;
  * different p*: the oracle's S at the larger of the two lies within delta
    of tau, the GPU value matches the oracle's estimate at the GPU's p* by the
    rule above, and at most 1 % (+ 2) of the indices flip;
  * the exact max-convolution is bit-exact (products rounded once, exact max).
"""

import math

import numpy as np
import pytest

import oracle
from workloads import maxconv_vectors

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
P = [1, 2, 4, 8, 16, 32, 64]


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def fft_delta(x, y, P):
    """delta_p per batch row (len(P) x b), from the inputs alone."""
    x = np.atleast_2d(np.asarray(x, dtype=np.float64))
    y = np.atleast_2d(np.asarray(y, dtype=np.float64))
    L = x.shape[1] + y.shape[1] - 1
    logN = max(1, math.ceil(math.log2(L))) if L > 1 else 1
    rx = x.max(axis=1, keepdims=True)
    ry = y.max(axis=1, keepdims=True)
    xs = np.where(rx > 0, x / np.where(rx > 0, rx, 1.0), 0.0)
    ys = np.where(ry > 0, y / np.where(ry > 0, ry, 1.0), 0.0)
    out = []
    for p in P:
        out.append(40.0 * logN * U * np.linalg.norm(xs ** p, axis=1) * np.linalg.norm(ys ** p, axis=1))
    return np.stack(out)


def _root_window(S, delta, p):
    hi = np.power(S + delta, 1.0 / p)
    lo = np.power(np.maximum(S - delta, 0.0), 1.0 / p)
    return hi - lo


def compare(z_gpu, ps_gpu, x, y, P, tau, fp32_out=False, max_flip_frac=0.01):
    """Check the GPU's (z, p*) against the oracle on the same inputs; returns
    statistics."""
    ref = oracle.maxconv_estimate(x, y, P, tau)
    delta = fft_delta(x, y, P)[:, :, None]  # (|P|, b, 1)
    S, q_ref = ref["S"], ref["pstar_idx"]
    rxy = (ref["rx"] * ref["ry"])[:, None]
    z_gpu = np.asarray(z_gpu, dtype=np.float64).reshape(q_ref.shape)
    ps_gpu = np.asarray(ps_gpu).reshape(q_ref.shape)
    Pa = np.asarray(P, dtype=np.float64)
    out_eps = 2.0 ** -24 if fp32_out else 0.0

    def allowed(qidx):
        qq = np.where(qidx == oracle.PSTAR_NONE, 0, qidx).astype(np.int64)
        S_at = np.take_along_axis(S, qq[None], 0)[0]
        d_at = np.take_along_axis(np.broadcast_to(delta, S.shape), qq[None], 0)[0]
        z_at = rxy * np.power(np.maximum(S_at, 0.0), 1.0 / Pa[qq])
        tol = rxy * _root_window(np.maximum(S_at, 0.0), d_at, Pa[qq]) + (1e-13 + out_eps) * z_at
        return z_at, tol

    z_at_g, tol_g = allowed(ps_gpu)
    err = np.abs(z_gpu - z_at_g)
    bad = err > tol_g
    assert not bad.any(), (f"{bad.sum()} indices off: max err {err[bad].max():.3e} "
                           f"tol {tol_g[bad].min():.3e}")
    flips = ps_gpu != q_ref
    n_flip = int(flips.sum())
    if n_flip:
        qg = np.where(ps_gpu == oracle.PSTAR_NONE, -1, ps_gpu.astype(np.int64))
        qr = np.where(q_ref == oracle.PSTAR_NONE, -1, q_ref.astype(np.int64))
        hi = np.maximum(qg, qr)
        S_hi = np.take_along_axis(S, hi[None], 0)[0]
        d_hi = np.take_along_axis(np.broadcast_to(delta, S.shape), hi[None], 0)[0]
        far = flips & (np.abs(S_hi - tau) > d_hi)
        assert not far.any(), f"{far.sum()} p* flips with S farther than delta from tau"
        assert n_flip <= max_flip_frac * q_ref.size + 2, f"too many p* flips: {n_flip} of {q_ref.size}"
    same = ~flips & (q_ref != oracle.PSTAR_NONE)
    rel = np.abs(z_gpu - ref["z"])[same] / ref["z"][same]
    return {"flips": n_flip, "max_rel_same": float(rel.max()) if rel.size else 0.0,
            "none": int((q_ref == oracle.PSTAR_NONE).sum())}


# up to n + m - 1 = 4096 in LDS; longer pairs (to 16384) through global buffers
SHAPES = [(3, 1, 1), (2, 5, 3), (4, 100, 37), (3, 257, 256), (2, 2048, 2049), (1, 4096, 1), (1, 1, 4096),
          (2, 1000, 1500), (2, 2049, 2049), (3, 3000, 2000), (1, 8192, 8193), (1, 16384, 1)]
KINDS = ["uniform", "lognormal", "sparse", "distribution"]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", KINDS)
def test_maxconv_parity(gpu_lib, shape, kind):
    b, n, m = shape
    x, y = maxconv_vectors(b, n, m, seed=7000 + n + 3 * m, kind=kind)
    z, ps = gpu_lib.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    st = compare(z.cpu().numpy(), ps.cpu().numpy(), x, y, P, oracle.TAU_FFT)
    print(kind, shape, st, flush=True)


@pytest.mark.parametrize("shape", [(4, 100, 37), (2, 2048, 2049), (2, 5000, 3000)],
                         ids=lambda s: "x".join(map(str, s)))
def test_maxconv_fp32(gpu_lib, shape):
    """FP32 input and output: the transform still runs in FP64; z is rounded
    once to FP32."""
    b, n, m = shape
    x, y = maxconv_vectors(b, n, m, seed=7100 + n, kind="lognormal", dtype=np.float32)
    z, ps = gpu_lib.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    assert z.dtype.is_floating_point and z.element_size() == 4
    compare(z.cpu().numpy(), ps.cpu().numpy(), x.astype(np.float64), y.astype(np.float64), P,
            oracle.TAU_FFT, fp32_out=True)


@pytest.mark.parametrize("shape", [(2, 7, 9), (3, 300, 300), (1, 2048, 2049), (2, 6000, 6000)],
                         ids=lambda s: "x".join(map(str, s)))
def test_fft_convolution_accuracy(gpu_lib, shape):
    """One power p = 1 and tau = 1e-300: z / (rx ry) is the FFT convolution
    itself (clamped at 0), within delta_1 of the direct convolution."""
    b, n, m = shape
    x, y = maxconv_vectors(b, n, m, seed=7200 + n, kind="uniform")
    z = gpu_lib.maxconv(_dev(x), _dev(y), [1], tau=1e-300).cpu().numpy()
    rxy = (x.max(axis=1) * y.max(axis=1))[:, None]
    direct = np.stack([np.convolve(x[i] / x[i].max(), y[i] / y[i].max()) for i in range(b)])
    delta = fft_delta(x, y, [1])[0][:, None]
    err = np.abs(z / rxy - direct)
    assert (err <= delta).all(), f"FFT error {err.max():.3e} above delta {delta.min():.3e}"
    print(shape, "max |err| / delta", float((err / delta).max()), flush=True)


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_exact_maxconv_bitexact(gpu_lib, dtype):
    x, y = maxconv_vectors(3, 300, 171, seed=7300, kind="lognormal", dtype=dtype)
    z = gpu_lib.maxconv_exact(_dev(x), _dev(y)).cpu().numpy()
    # a product of two FP32 values is exact in FP64; rounding is monotone, so
    # the FP32 max of rounded products is the rounded FP64 max
    ref = oracle.exact_maxconv(x.astype(np.float64), y.astype(np.float64)).astype(dtype)
    np.testing.assert_array_equal(z, ref)


def test_estimate_bounds_against_exact(gpu_lib):
    """E <= z <= K^(1/p*) E (Sec. 1), K the number of products at the index,
    against the GPU's exact max-convolution, widened by the FFT's rounding:
    S_gpu = (z / (rx ry))^p* lies within delta of a ring result that the
    bound brackets."""
    b, n, m = 4, 700, 500
    x, y = maxconv_vectors(b, n, m, seed=7400, kind="distribution")
    z, ps = gpu_lib.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    E = gpu_lib.maxconv_exact(_dev(x), _dev(y)).cpu().numpy()
    z, ps = z.cpu().numpy(), ps.cpu().numpy()
    t = np.arange(n + m - 1)
    K = np.minimum(np.minimum(t + 1, n + m - 1 - t), min(n, m))[None, :]
    # no stable p: the smallest p's root of max(S, 0), bracketed the same way
    qi = np.where(ps == oracle.PSTAR_NONE, 0, ps).astype(np.int64)
    p = np.asarray(P, dtype=np.float64)[qi]
    d = fft_delta(x, y, P)[qi, np.arange(b)[:, None]]
    rxy = (x.max(axis=1) * y.max(axis=1))[:, None]
    e = E / rxy
    lo = rxy * np.power(np.maximum(np.power(e, p) - d, 0.0), 1.0 / p)
    hi = rxy * np.power(K * np.power(e, p) + d, 1.0 / p)
    assert (z >= lo * (1 - 1e-13)).all()
    assert (z <= hi * (1 + 1e-13)).all()


def test_edge_cases(gpu_lib):
    import torch

    mt = gpu_lib
    P4 = [1, 2, 4, 8]
    # empty batch and empty vectors: empty results, nothing launched
    e = mt.maxconv(torch.zeros((0, 5), dtype=torch.float64, device="cuda"),
                   torch.zeros((0, 3), dtype=torch.float64, device="cuda"), P4)
    assert e.shape == (0, 7)
    e = mt.maxconv(torch.zeros(0, dtype=torch.float64, device="cuda"),
                   torch.ones(3, dtype=torch.float64, device="cuda"), P4)
    assert e.shape == (0,)
    # an all-zero operand: z = 0, no p stable
    x = np.zeros((1, 6))
    y = np.ones((1, 4))
    z, ps = mt.maxconv(_dev(x), _dev(y), P4, return_pstar=True)
    assert (z.cpu().numpy() == 0).all() and (ps.cpu().numpy() == oracle.PSTAR_NONE).all()
    # one-hot x: z is y shifted, exactly at every stable index up to the FFT
    x = np.zeros((1, 9))
    x[0, 3] = 2.5
    y = maxconv_vectors(1, 20, 20, seed=7500)[1][:, :20]
    z, ps = mt.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    compare(z.cpu().numpy(), ps.cpu().numpy(), x, y, P, oracle.TAU_FFT)
    j = int(np.argmax(y[0]))
    assert abs(z.cpu().numpy()[0, 3 + j] - 2.5 * y[0, j]) <= 1e-13 * 2.5 * y[0, j]
    # tiny and huge scales: the scaling keeps the transform in [0, 1]
    for scale in (1e-150, 1e150):
        x, y = maxconv_vectors(2, 64, 80, seed=7600, kind="uniform")
        z, ps = mt.maxconv(_dev(x * scale), _dev(y), P, return_pstar=True)
        compare(z.cpu().numpy(), ps.cpu().numpy(), x * scale, y, P, oracle.TAU_FFT)
    # one p: every stable index uses it; a custom tau moves p*
    x, y = maxconv_vectors(2, 50, 60, seed=7700, kind="lognormal")
    for tau in (1e-3, 1e-12):
        z, ps = mt.maxconv(_dev(x), _dev(y), P, tau=tau, return_pstar=True)
        compare(z.cpu().numpy(), ps.cpu().numpy(), x, y, P, tau)
    z, ps = mt.maxconv(_dev(x), _dev(y), [16], return_pstar=True)
    compare(z.cpu().numpy(), ps.cpu().numpy(), x, y, [16], oracle.TAU_FFT)


def test_large_batch_sampled_rows(gpu_lib):
    """The benchmark's shape (8192 pairs of 2048-vectors): the whole batch on
    the GPU, sampled rows against the oracle."""
    b, n, m = 8192, 2048, 2048
    x, y = maxconv_vectors(b, n, m, seed=7800, kind="distribution")
    z, ps = gpu_lib.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    z, ps = z.cpu().numpy(), ps.cpu().numpy()
    rows = np.random.default_rng(7801).choice(b, 6, replace=False)
    rows = np.concatenate([[0, b - 1], rows])
    compare(z[rows], ps[rows], x[rows], y[rows], P, oracle.TAU_FFT)


@pytest.mark.parametrize("shape", [(3, 200, 150), (2, 1024, 1024), (2, 4000, 4000)],
                         ids=lambda s: "x".join(map(str, s)))
def test_non_power_of_two_family(gpu_lib, shape):
    """p that are not powers of two take the root as exp(log S / p) and the
    powers by repeated squaring with odd steps."""
    b, n, m = shape
    P = [1, 3, 5, 7, 12, 20, 33]
    x, y = maxconv_vectors(b, n, m, seed=7900 + n, kind="lognormal")
    z, ps = gpu_lib.maxconv(_dev(x), _dev(y), P, return_pstar=True)
    st = compare(z.cpu().numpy(), ps.cpu().numpy(), x, y, P, oracle.TAU_FFT)
    print(shape, st, flush=True)
