"""Deferred planes on the BF16 path.

p* is the largest stable p (Sec. 1), so an entry reaches the two smallest p
of the family only when it is unstable at every larger one.  The plane
launches leave those planes out; they are written before the GEMM when the
pilot's sampled entries include such an entry, and otherwise after it, when
a GEMM tile or a sparse-tail entry has reached them, and the tiles that did
run their whole search again.

Checks, on 2048 x 512 x 2048 products (large enough for the pilot, whose
64 x 64 sample takes the rows and columns at odd multiples of 16):

* no entry needs the late planes: the same C and p* as with every plane
  written up front, bit for bit, and no tile runs again;
* a few rows off the sample need them (zero rows, whose S is 0 at every p,
  and rows whose every term is about 1e-10 after scaling, p* = 2): tiles
  reach them in the GEMM (three such rows in a tile, 768 undecided entries,
  more than the tail takes) and in the tail (one such row); those tiles run
  again, the special rows and other rows of them match the oracle, and the
  other tiles are bit-equal to the all-planes run;
* every row needs them: the pilot sees it, the planes are written before
  the GEMM and no tile runs again;
* the same rare rows with inner-index balancing (which lifts most entries
  of the crossed rows to p* = 4, leaving some at 2) and with FP64 inputs
  (the late planes take the balancing factors and the FP64 reader);
* two batch items of a ragged product, only the second with such rows: the
  marks index the batch item and partial tiles;
* the FP64 path, which defers all but the three largest p (64 x 64 tiles at
  this size): no entry below p = 32 (bit-equal, nothing runs again); zero
  rows and rows with p* = 16 off the sample, reached in the tail and, eleven
  such rows in one tile, in the GEMM; every row at p* = 16."""

import numpy as np
import pytest

import oracle
from parity import TAU, compare_estimate
from workloads import lognormal_product

pytestmark = [pytest.mark.gpu, pytest.mark.usefixtures("general_path")]

P128 = [1, 2, 4, 8, 16, 32, 64, 128]
M, K, N = 2048, 512, 2048
ZERO_ROWS = (5, 300, 301, 302)     # tile rows 0 (tail) and 1 (GEMM)
CROSSED_ROWS = (1000, 1500, 1501, 1502)  # tile rows 3 (tail) and 5 (GEMM)
SPECIAL_TILE_ROWS = (0, 1, 3, 5)


@pytest.fixture
def knobs(gpu_lib):
    old_d, old_s = gpu_lib.deferred_planes(), gpu_lib.search_start()
    gpu_lib.set_search_start(-1)
    yield gpu_lib
    gpu_lib.set_deferred_planes(old_d)
    gpu_lib.set_search_start(old_s)
    gpu_lib.timing_enable(False)
    gpu_lib.timing_reset()


def _dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _sampled_rows():
    return set(((2 * np.arange(64) + 1) * M) // 128)


def _rare(A, B):
    """B's first half of the inner index scaled by 1e-10; the crossed rows of
    A by 1e-12 on the second half (every term of theirs about 1e-10 or less
    after scaling: unstable at p = 4, stable at p = 2); the zero rows 0."""
    A, B = A.copy(), B.copy()
    h = A.shape[-1] // 2
    B[..., :h, :] *= 1e-10
    for i in CROSSED_ROWS:
        A[..., i, h:] *= 1e-12
    for i in ZERO_ROWS:
        A[..., i, :] = 0
    assert not (set(CROSSED_ROWS) | set(ZERO_ROWS)) & _sampled_rows()
    return A, B


def _run(mt, A, B, on, balance=False, path="bf16"):
    """(C, p*, work of the tiles that ran again) with deferral on or off."""
    import torch

    mt.set_deferred_planes(on)
    mt.timing_reset()
    mt.timing_enable(True)
    C, ps = mt.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True, balance=balance)
    torch.cuda.synchronize()
    rerun = mt.timing_work("mt_rerun_gemm")
    mt.timing_enable(False)
    mt.timing_reset()
    return C.cpu().numpy(), ps.cpu().numpy(), rerun


def test_no_entry_needs_late_planes(knobs):
    A, B = lognormal_product(M, K, N, seed=4201)
    print("[deferred] log-normal, no entry below p = 4", flush=True)
    C1, p1, w1 = _run(knobs, A, B, True)
    C0, p0, w0 = _run(knobs, A, B, False)
    assert w1 == 0.0 and w0 == 0.0
    np.testing.assert_array_equal(p1, p0)
    np.testing.assert_array_equal(C1.view(np.uint32), C0.view(np.uint32))
    rows = np.arange(7, M, 211)
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU["bf16"], rows)
    compare_estimate(C1[rows], p1[rows], ref, P128, "bf16")


@pytest.mark.parametrize("variant", ["fp32", "fp64_inputs", "balanced"])
def test_rare_rows_run_again(knobs, variant):
    A, B = lognormal_product(M, K, N, seed=4201)
    if variant == "fp64_inputs":
        A, B = A.astype(np.float64), B.astype(np.float64)
    A, B = _rare(A, B)
    bal = variant == "balanced"
    print(f"[deferred] rare rows, {variant}", flush=True)
    C1, p1, w1 = _run(knobs, A, B, True, balance=bal)
    C0, p0, w0 = _run(knobs, A, B, False, balance=bal)
    assert w0 == 0.0
    # the tile rows with special rows ran again (8 tiles each, at least one
    # dense p per tile): all four, or with balancing, which lifts most
    # entries of the crossed rows to p* = 4, surely the two with zero rows
    assert w1 >= (16 if bal else 32) * 2.0 * 256 * 256 * K
    special = np.zeros(M, dtype=bool)
    for t in SPECIAL_TILE_ROWS:
        special[t * 256:(t + 1) * 256] = True
    # tiles that did not run again: bit-equal to the all-planes run
    np.testing.assert_array_equal(p1[~special], p0[~special])
    np.testing.assert_array_equal(C1[~special].view(np.uint32), C0[~special].view(np.uint32))
    # the special rows and others of the tiles that ran again, and a few
    # elsewhere, against the oracle
    rows = np.array(sorted(set(ZERO_ROWS) | set(CROSSED_ROWS) | {6, 299, 777, 1499, 1535, 1800}))
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU["bf16"], rows, balance=bal)
    compare_estimate(C1[rows], p1[rows], ref, P128, "bf16")
    assert (C1[list(ZERO_ROWS)] == 0).all()
    if not bal:
        assert (p1[list(CROSSED_ROWS)] == 1).mean() > 0.99  # p* = 2


def test_every_row_needs_late_planes(knobs):
    A, B = lognormal_product(M, K, N, seed=4203)
    h = K // 2
    B[:h, :] *= 1e-10
    A[:, h:] *= 1e-12
    print("[deferred] every row crossed", flush=True)
    C1, p1, w1 = _run(knobs, A, B, True)
    assert w1 == 0.0  # written before the GEMM: nothing ran again
    assert (p1 == 1).mean() > 0.99
    rows = np.arange(3, M, 173)
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU["bf16"], rows)
    compare_estimate(C1[rows], p1[rows], ref, P128, "bf16")


def test_rare_rows_batched_ragged(knobs):
    """Two batch items of a ragged 2000 x 520 x 2100 product (partial tiles,
    a padded inner length): only the second has rows that need the late
    planes, so only its tiles with them run again; the tile marks index the
    batch item."""
    m, k, n = 2000, 520, 2100
    sampled = set(((2 * np.arange(64) + 1) * m) // 128)
    A0, B0 = lognormal_product(m, k, n, seed=4301)
    A1, B1 = lognormal_product(m, k, n, seed=4302)
    h = k // 2
    B1[:h, :] *= 1e-10
    crossed, zero = (700, 1990), (1010, 1011, 1012)
    for i in crossed:
        A1[i, h:] *= 1e-12
    for i in zero:
        A1[i, :] = 0
    assert not (set(crossed) | set(zero)) & sampled
    A, B = np.stack([A0, A1]), np.stack([B0, B1])
    print("[deferred] batched ragged rare rows", flush=True)
    C1, p1, w1 = _run(knobs, A, B, True)
    C0, p0, w0 = _run(knobs, A, B, False)
    assert w0 == 0.0 and w1 > 0.0
    special = np.zeros((2, m), dtype=bool)
    for i in crossed + zero:
        special[1, (i // 256) * 256:(i // 256 + 1) * 256] = True
    np.testing.assert_array_equal(p1[~special], p0[~special])
    np.testing.assert_array_equal(C1[~special].view(np.uint32), C0[~special].view(np.uint32))
    for bi, rows in ((0, [3, 1000, 1999]), (1, sorted(crossed + zero + (699, 1013, 1500)))):
        rows = np.array(rows)
        ref = oracle.pnorm_estimate_rows(A[bi], B[bi], P128, TAU["bf16"], rows)
        compare_estimate(C1[bi][rows], p1[bi][rows], ref, P128, "bf16")
    assert (C1[1][list(zero)] == 0).all()


@pytest.mark.parametrize("case", ["none", "rare", "every"])
def test_fp64_path(knobs, case):
    """FP64 path (tau 1e-290): the planes of p <= 16 are deferred.  Crossed
    terms of about 1e-10 underflow at p >= 32 and are stable at p = 16."""
    A, B = lognormal_product(M, K, N, seed=4203 if case == "every" else 4201)
    A, B = A.astype(np.float64), B.astype(np.float64)
    h = K // 2
    crossed, zero = (1000,) + tuple(range(1500, 1511)), (5, 300, 301, 302)
    if case == "rare":
        B[:h] *= 1e-10
        for i in crossed:
            A[i, h:] *= 1e-12
        for i in zero:
            A[i] = 0
        assert not (set(crossed) | set(zero)) & _sampled_rows()
    elif case == "every":
        B[:h] *= 1e-10
        A[:, h:] *= 1e-12
    print(f"[deferred] fp64 {case}", flush=True)
    C1, p1, w1 = _run(knobs, A, B, True, path="fp64")
    C0, p0, w0 = _run(knobs, A, B, False, path="fp64")
    assert w0 == 0.0
    special = np.zeros(M, dtype=bool)
    if case == "rare":
        for i in crossed + zero:
            special[(i // 64) * 64:(i // 64 + 1) * 64] = True
        assert w1 > 0.0
        assert (p1[list(crossed)] == 4).mean() > 0.99  # p* = 16
        assert (C1[list(zero)] == 0).all()
    else:
        assert w1 == 0.0
    if case != "every":
        np.testing.assert_array_equal(p1[~special], p0[~special])
        np.testing.assert_array_equal(C1[~special].view(np.uint64), C0[~special].view(np.uint64))
    else:
        assert (p1 == 4).mean() > 0.99
    rows = np.array(sorted({3, 741, 1300, 2047} | (set(crossed) | set(zero) | {299, 1499} if case == "rare" else set())))
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU["fp64"], rows)
    compare_estimate(C1[rows], p1[rows], ref, P128, "fp64")


def test_rare_rows_noalloc(knobs):
    """The entry point without a workspace keeps the marks and flags in its
    static scratch: the same C and p* as the workspace call, twice in a row
    (the second call finds the first call's marks and clears them)."""
    import torch

    if knobs.workspace_size(1, M, K, N, P128, path="bf16") > knobs.NOALLOC_SCRATCH_BYTES:
        pytest.skip("the product does not fit the static scratch")
    A, B = _rare(*lognormal_product(M, K, N, seed=4201))
    knobs.set_deferred_planes(True)
    dA, dB = _dev(A), _dev(B)
    C0, p0 = knobs.estimate(dA, dB, P=P128, path="bf16", return_pstar=True)
    for rep in range(2):
        print(f"[deferred] noalloc call {rep}", flush=True)
        C1, p1 = knobs.estimate_noalloc(dA, dB, P=P128, path="bf16")
        torch.cuda.synchronize()
        assert torch.equal(p0, p1)
        assert torch.equal(C0, C1)
