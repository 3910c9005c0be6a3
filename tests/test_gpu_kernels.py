"""Kernel-level checks of the product's first steps, read from the workspace
through maxtimes_workspace_map (bit-exact):

* K1: r_i = max_k A_ik and c_j = max_k B_kj (Sec. 2.1 scaling) equal numpy's
  maxima of the same values exactly (a max is exact);
* K2: every power plane equals an emulation of the plane kernel's arithmetic
  bit for bit: x = A / r (multiplied by the FP64 reciprocal of r for whole
  8-element chunks of rows whose length the vector loads allow, divided
  otherwise), powers in the path's precision (squaring when p doubles the
  previous power, binary powering otherwise), and on the BF16 path hi =
  round-to-nearest-even of the FP32 power to BF16, lo = the same rounding of
  the remainder for split p.  Padding holds zeros.

The emulation is a model of the kernel's rounding, not the oracle: the
oracle's FP64 estimate is compared with the whole product elsewhere.
"""

import numpy as np
import pytest

from workloads import lognormal_product, uniform_product

# these cases exercise the general path (planes, MFMA GEMM, sparse tail,
# search start), also at sizes the one-kernel small-product path would take
pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]


def _bf16_rne(f32):
    u = f32.astype(np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def _bf16_to_f32(h):
    return (h.astype(np.uint32) << 16).view(np.float32)


def _ipow(x, p):
    r = np.ones_like(x)
    while p:
        if p & 1:
            r = r * x
        x = x * x
        p >>= 1
    return r


def emulate_planes(src, scale, rows_pad, cols_pad, powers, split, transposed, bf16):
    """src (b, rows, cols) as the kernel walks it, scale (b, rows) FP64."""
    b, rows, cols = src.shape
    tc = np.float32 if bf16 else np.float64
    s64 = src.astype(np.float64)
    sc = scale[:, :, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        fast_val = (s64 * np.where(sc > 0, 1.0 / np.where(sc > 0, sc, 1.0), 0.0)).astype(tc)
        slow_val = np.where(sc > 0, s64 / np.where(sc > 0, sc, 1.0), 0.0).astype(tc)
    u = np.arange(cols)
    chunk_ok = (u // 8) * 8 + 8 <= cols
    if not transposed:
        chunk_ok &= (cols % 4 == 0)
    fast = chunk_ok[None, None, :] & (sc > 0)
    x = np.zeros((b, rows_pad, cols_pad), dtype=tc)
    x[:, :rows, :cols] = np.where(fast, fast_val, slow_val)
    planes = []
    prev, pw = 0, None
    for p, sp in zip(powers, split):
        pw = pw * pw if (prev > 0 and p == 2 * prev) else _ipow(x.copy(), p)
        prev = p
        if bf16:
            hi = _bf16_rne(pw)
            planes.append(hi)
            if sp:
                planes.append(_bf16_rne(pw.astype(np.float32) - _bf16_to_f32(hi)))
        else:
            planes.append(pw)
    return np.stack(planes, axis=1)


def _run_and_map(mt, A, B, P, path):
    import torch

    b, m, k = A.shape
    n = B.shape[2]
    wm = mt.workspace_map(b, m, k, n, P, path=path)
    ws = torch.zeros(mt.workspace_size(b, m, k, n, P, path=path), dtype=torch.uint8, device="cuda")
    mt.estimate(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), P=P, path=path, workspace=ws)
    return wm, ws.cpu().numpy()


CASES = [
    ("uniform", 2, 100, 70, 50),      # k % 4 != 0: every A chunk divides
    ("lognormal", 1, 257, 204, 129),  # a ragged last chunk, denormal powers
    ("lognormal", 2, 64, 256, 300),
    ("lognormal", 1, 5, 8192, 40),    # the longest rows whose maxima the plane pass takes
    ("uniform", 1, 6, 8200, 33),      # one chunk longer: separate maxima, k % 4 != 0
]


@pytest.mark.parametrize("path,P", [("bf16", [1, 2, 3, 4, 8, 16, 64]), ("fp64", [1, 2, 3, 4, 8, 32])])
@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c)))
def test_scales_and_power_planes_bit_exact(gpu_lib, case, path, P):
    kind, b, m, k, n = case
    if kind == "uniform":
        A, B = uniform_product(m, k, n, seed=9900 + m, dtype=np.float32, batch=b)
    else:
        A, B = lognormal_product(m, k, n, seed=9900 + m, sigma=3.0)
        A = np.stack([A] * b) if A.ndim == 2 else A
        B = np.stack([B] * b) if B.ndim == 2 else B
    A = np.ascontiguousarray(A.reshape(b, m, k))
    B = np.ascontiguousarray(B.reshape(b, k, n))
    A[0, 3, :] = 0.0  # a zero row: r = 0, an all-zero plane row
    wm, ws = _run_and_map(gpu_lib, A, B, P, path)

    # K1
    r = ws[wm["r"]: wm["r"] + b * m * 8].view(np.float64).reshape(b, m)
    c = ws[wm["c"]: wm["c"] + b * n * 8].view(np.float64).reshape(b, n)
    np.testing.assert_array_equal(r, A.astype(np.float64).max(axis=2))
    np.testing.assert_array_equal(c, B.astype(np.float64).max(axis=1))

    # K2
    bf16 = path == "bf16"
    et = np.uint16 if bf16 else np.float64
    np_, mp, npad, kp = wm["n_planes"], wm["m_pad"], wm["n_pad"], wm["k_pad"]
    esz = wm["elem_bytes"]
    pa = ws[wm["a_planes"]: wm["a_planes"] + b * np_ * mp * kp * esz].view(et).reshape(b, np_, mp, kp)
    pb = ws[wm["b_planes"]: wm["b_planes"] + b * np_ * npad * kp * esz].view(et).reshape(b, np_, npad, kp)
    ea = emulate_planes(A, r, mp, kp, wm["power"], wm["split"], transposed=False, bf16=bf16)
    eb = emulate_planes(np.ascontiguousarray(B.transpose(0, 2, 1)), c, npad, kp, wm["power"], wm["split"],
                        transposed=True, bf16=bf16)
    if bf16:
        np.testing.assert_array_equal(pa, ea)
        np.testing.assert_array_equal(pb, eb)
    else:
        np.testing.assert_array_equal(pa.view(np.uint64), ea.view(np.uint64))
        np.testing.assert_array_equal(pb.view(np.uint64), eb.view(np.uint64))
