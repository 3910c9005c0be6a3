"""Host-side emulation of how the BF16 path restores the row and column
scales (Sec. 2.1, scaled call H': the estimate is r_i c_j S^(1/p) with r_i,
c_j the maxima the inputs were divided by).

The kernels split each scale v = m 2^e with m in [0.5, 1) (frexp), multiply
the FP32 mantissas with the root, and apply e_r + e_c with one ldexp in the
output's precision.  This file emulates that arithmetic in numpy (it models
the kernel, it is not the oracle) and checks that it neither over- nor
underflows where the true value r c S^(1/p) is representable, for scales far
outside FP32, and that it is as accurate as an FP32 product.  The plain FP32
product of the scales, which the form replaces, overflows on the same
inputs (checked, so the cases really reach the hazard).
"""

import numpy as np

F32_MAX = float(np.finfo(np.float32).max)
F32_TINY = float(np.finfo(np.float32).tiny)
U32 = 2.0 ** -24


def split_scale(v):
    m, e = np.frexp(np.asarray(v, dtype=np.float64))
    return m.astype(np.float32), e.astype(np.int64)


def restore(r, c, root, out_dtype):
    """The epilogue: (m_r m_c root) in FP32, then ldexp by e_r + e_c in the
    output type."""
    mr, er = split_scale(r)
    mc, ec = split_scale(c)
    v = (mr * mc).astype(np.float32) * np.asarray(root, dtype=np.float32)
    v = v.astype(np.float32)
    return np.ldexp(v.astype(out_dtype), (er + ec).astype(np.int32))


def naive_f32(r, c, root):
    with np.errstate(over="ignore", under="ignore"):
        return np.float32(r) * np.float32(c) * np.float32(root)


def test_reviewer_case_overflows_naively_and_not_in_the_split_form():
    # A row [1e20, 1e5], B column [1e5, 1e20]: r = c = 1e20, S_2 = 2e-30
    r = float(np.float32(1e20))
    c = r
    root = np.sqrt(2.0 * (np.float32(1e5) / np.float32(1e20)) ** 2, dtype=np.float64)
    assert np.isinf(naive_f32(r, c, root))
    got = float(restore(r, c, root, np.float32))
    want = r * c * root
    assert np.isfinite(got)
    assert abs(got / want - 1.0) <= 4 * U32


def test_fp32_outputs_of_fp32_scales_beyond_fp32_product():
    rng = np.random.default_rng(11)
    n = 200000
    r = np.float32(10.0 ** rng.uniform(-37, 38, n)).astype(np.float64)
    c = np.float32(10.0 ** rng.uniform(-37, 38, n)).astype(np.float64)
    root = np.float32(10.0 ** rng.uniform(-20, 0.6, n)).astype(np.float64)
    want = r * c * root
    with np.errstate(over="ignore"):
        got = restore(r, c, root, np.float32).astype(np.float64)
    normal = (want >= F32_TINY) & (want <= F32_MAX * (1 - 4 * U32))
    assert normal.sum() > n // 4
    rel = np.abs(got[normal] / want[normal] - 1.0)
    assert rel.max() <= 4 * U32, rel.max()
    # overflow only where the value itself exceeds FP32, 0 only below its subnormals
    assert np.isinf(got[want > F32_MAX * (1 + 4 * U32)]).all()
    assert (got[want < F32_TINY * 2.0 ** -24 * 0.49] == 0).all()
    # the naive product overflows on a good share of the representable cases
    with np.errstate(over="ignore", invalid="ignore"):
        nv = np.float32(r) * np.float32(c) * np.float32(root)
    assert np.isinf(nv[normal]).sum() > 1000


def test_fp64_outputs_with_scales_far_outside_fp32():
    rng = np.random.default_rng(12)
    n = 200000
    r = 10.0 ** rng.uniform(-150, 150, n)
    c = 10.0 ** rng.uniform(-150, 150, n)
    root = rng.uniform(1e-6, 4.0, n).astype(np.float32).astype(np.float64)
    want = r * c * root
    got = restore(r, c, root, np.float64)
    rel = np.abs(got / want - 1.0)
    assert rel.max() <= 4 * U32, rel.max()
    # near 1e+-50 (the precision form's FP64 I/O): every value is finite and nonzero
    r50 = 10.0 ** rng.uniform(-50, 50, n)
    c50 = 10.0 ** rng.uniform(-50, 50, n)
    got50 = restore(r50, c50, root, np.float64)
    assert np.isfinite(got50).all() and (got50 > 0).all()


def test_zero_scale_gives_zero():
    assert restore(0.0, 1e30, 1.0, np.float32) == 0.0
    assert restore(1e30, 0.0, 1.0, np.float64) == 0.0


def test_adjoint_scaled_operand_stays_in_unit_interval():
    """The adjoint forms M / v as (M 2^-e) / m (v = m 2^e): for M <= v it is
    in [0, 1], also for FP64 entries beyond FP32 and subnormal scales."""
    rng = np.random.default_rng(13)
    v = np.concatenate([10.0 ** rng.uniform(-300, 300, 1000), [5e-324, 1e-310, 1.7e308]])
    M = v * rng.uniform(0, 1, v.shape)
    M[-3:] = v[-3:]
    m, e = np.frexp(v)
    x = np.ldexp(M, -e).astype(np.float32) * (np.float32(1.0) / m.astype(np.float32))
    assert np.isfinite(x).all() and (x >= 0).all() and (x <= 1.0 + 2 * U32).all()
    ok = M / v
    assert np.abs(x - ok)[ok > 1e-30].max() <= 4 * U32
