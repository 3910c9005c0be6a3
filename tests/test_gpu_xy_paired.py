"""GPU parity of the paired NormQueue (the Discussion's refinement of Sec.
2.3: both runs pop in lockstep, an accurate pair is reported and subtracted
exactly) against the oracle.

Accurate ranks subtract an exact value, so the FFT rounding of the ring
results no longer grows into later pops the way it does in the plain queue;
the cases below were checked on the CPU to give the same sequence on direct
ring results (the oracle's) and on numpy FFT ones of two transform lengths
(uniform lists on [0, s], s = 1 .. 40, FP64 and FP32, both transform paths,
K = min(k, 2n - 1) up to 256 (a lane's slots in registers), 320 (in LDS) and
599 (columns in the workspace)).
Compared: the accept mask, both diagonals and the indices exactly; accepted
values bit for bit (x_i + y_j in FP64 on both sides); the other values,
estimates, within 1e-6 (the tolerance of the plain queue's tests, which the
FFT-run check stays inside: 7.2e-7 at most).
"""

import numpy as np
import pytest

from oracle.xy_topk import exact_topk_xy, xy_topk_paired

pytestmark = pytest.mark.gpu

P24 = [1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 1536, 2048, 3072, 4096]

CASES = [  # n, k, spread, seed, dtype
    (256, 64, 40, 3, np.float64),      # every rank accurate
    (256, 64, 10, 4, np.float64),      # accurate and estimated ranks
    (1000, 128, 20, 11, np.float64),
    (700, 100, 30, 13, np.float32),
    (2049, 160, 10, 14, np.float64),   # first length on the global-memory transforms
    (3000, 200, 40, 12, np.float64),
    (1500, 320, 30, 16, np.float64),   # K = 320: columns in LDS, slots in LDS
    (8192, 256, 40, 5005, np.float64),
    (8192, 256, 1, 5005, np.float64),
]


def _run(mt, x, y, k):
    import torch

    xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
    yd = torch.from_numpy(np.ascontiguousarray(y)).cuda()
    v, i, j, d = mt.xy_topk(xd, yd, k, paired=True, return_diag=True)
    torch.cuda.synchronize()
    return v.cpu().numpy(), i.cpu().numpy(), j.cpu().numpy(), d.cpu().numpy()


def _check(v, i, j, d, o):
    acc = o["accepted"]
    np.testing.assert_array_equal(i, o["i"])
    np.testing.assert_array_equal(j, o["j"])
    np.testing.assert_array_equal(d, o["diag"])
    np.testing.assert_array_equal(v[acc], o["values"][acc])
    fin = ~acc & np.isfinite(o["values"])
    np.testing.assert_allclose(v[fin], o["values"][fin], rtol=0, atol=1e-6)
    np.testing.assert_array_equal(np.isneginf(v), np.isneginf(o["values"]))


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"n{c[0]}_k{c[1]}_s{c[2]}_{c[4].__name__}")
def test_paired_matches_oracle(gpu_lib, case):
    n, k, spread, seed, dt = case
    rng = np.random.default_rng(seed)
    x = rng.uniform(0, spread, n).astype(dt)
    y = rng.uniform(0, spread, n).astype(dt)
    v, i, j, d = _run(gpu_lib, x, y, k)
    o = xy_topk_paired(x.astype(np.float64), y.astype(np.float64), P24, k)
    _check(v, i, j, d, o)


def test_paired_every_rank_accurate_is_the_exact_top_k(gpu_lib):
    rng = np.random.default_rng(3)
    x = rng.uniform(0, 40, 256)
    y = rng.uniform(0, 40, 256)
    v, i, j, _ = _run(gpu_lib, x, y, 64)
    ev, ei, ej = exact_topk_xy(x, y, 64)
    np.testing.assert_array_equal(v, ev)
    np.testing.assert_array_equal(i, ei)
    np.testing.assert_array_equal(j, ej)


def _check_properties(x, y, v, i, j, d):
    """What holds at any depth and under any rounding: an accepted rank
    (i >= 0) is a grid pair on its diagonal with the exact value, no pair
    comes twice, and other ranks carry no indices."""
    n = x.size
    acc = i >= 0
    assert ((j >= 0) == acc).all()
    assert (i[acc] < n).all() and (j[acc] < n).all()
    np.testing.assert_array_equal(i[acc] + j[acc], d[acc])
    np.testing.assert_array_equal(v[acc], x[i[acc]] + y[j[acc]])
    assert len(set(zip(i[acc].tolist(), j[acc].tolist()))) == int(acc.sum())


# depth = the ranks that come out the same on direct ring results and on
# numpy FFT ones of three transform lengths, halved for margin (past it the
# queues run into residuals at the rounding level of the transforms)
@pytest.mark.parametrize("n,k,depth", [(1, 3, 3), (2, 4, 2), (5, 30, 3), (17, 289, 12), (64, 4096, 31),
                                       (300, 4096, 89)])
def test_paired_small_and_exhausted(gpu_lib, n, k, depth):
    # k up to every pair and beyond (ranks past the last stable estimate are
    # -inf), k above 2n - 1 (every diagonal a candidate), the largest k
    rng = np.random.default_rng(700 + n)
    x = rng.uniform(0, 8, n)
    y = rng.uniform(0, 8, n)
    v, i, j, d = _run(gpu_lib, x, y, k)
    o = xy_topk_paired(x, y, P24, k)
    _check(v[:depth], i[:depth], j[:depth], d[:depth], {f: a[:depth] for f, a in o.items()})
    _check_properties(x, y, v, i, j, d)


def test_paired_equal_lists(gpu_lib):
    # x = y: every pair has its mirror on the same diagonal
    x = np.array([3.0, 1.0, 2.0, 3.0, 0.5, 2.0, 1.0, 3.0])
    v, i, j, d = _run(gpu_lib, x, x.copy(), 40)
    o = xy_topk_paired(x, x.copy(), P24, 40)
    _check(v[:5], i[:5], j[:5], d[:5], {f: a[:5] for f, a in o.items()})
    _check_properties(x, x, v, i, j, d)


def test_paired_rejects_large_k(gpu_lib):
    import torch

    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(gpu_lib.MaxTimesError, match="k <= 4096"):
        gpu_lib.xy_topk(x, x, 4097, paired=True)


def test_paired_largest_k_at_the_largest_n(gpu_lib):
    """n = 8192, k = 4096: 2 x 4096 candidates, the reported pairs and the
    estimates exceed LDS with the log lengths, which are then taken per rank.
    The first 256 ranks against the oracle (the depth the k = 256 case
    checks; candidates are exact, so ranks do not depend on k), every rank's
    properties, and the first 1000 ranks equal to a k = 1000 call (log
    lengths kept in LDS there)."""
    rng = np.random.default_rng(5005)
    x = rng.uniform(0, 40, 8192)
    y = rng.uniform(0, 40, 8192)
    print("[xy] paired n=8192 k=4096", flush=True)
    v, i, j, d = _run(gpu_lib, x, y, 4096)
    o = xy_topk_paired(x, y, P24, 256)
    _check(v[:256], i[:256], j[:256], d[:256], o)
    _check_properties(x, y, v, i, j, d)
    v2, i2, j2, d2 = _run(gpu_lib, x, y, 1000)
    np.testing.assert_array_equal(i[:1000], i2)
    np.testing.assert_array_equal(d[:1000], d2)
    np.testing.assert_array_equal(v[:1000], v2)
