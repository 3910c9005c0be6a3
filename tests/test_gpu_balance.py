"""GPU parity of the inner-index balanced estimate (MT_FLAG_BALANCE: the
estimate of (A D, D^-1 B), d_k = sqrt(max_j B_kj / max_i A_ik); the
Discussion's remark on scaling into a bounded range) against the oracle's
balanced estimate, at the path's tolerance with the band rule for p* flips,
on ragged and batched shapes, through the sparse tail and the pilot's search
start, plus the closed-form two-term case, inner-scaled inputs (where p*
rises and the error against the exact product falls) and the argument
checks."""

import math

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


def _run(mt, A, B, P, path, **kw):
    C, ps = mt.estimate(_dev(A), _dev(B), P=P, path=path, return_pstar=True, balance=True, **kw)
    return C.cpu().numpy(), ps.cpu().numpy()


@pytest.fixture
def knobs(gpu_lib):
    old_s, old_t = gpu_lib.search_start(), gpu_lib.tail_threshold()
    yield gpu_lib
    gpu_lib.set_search_start(old_s)
    gpu_lib.set_tail_threshold(old_t)


def inner_scaled(m, k, n, seed, decades, batch=None):
    """U diag(s), diag(s)^-1 V: uniform U, V; log10 s uniform on [-decades, decades]."""
    rng = np.random.default_rng(seed)
    shp = () if batch is None else (batch,)
    U = 1.0 - rng.random(shp + (m, k))
    V = 1.0 - rng.random(shp + (k, n))
    s = 10.0 ** rng.uniform(-decades, decades, shp + (k,))
    return U * s[..., None, :], V / s[..., :, None]


@pytest.mark.parametrize("shape", [(1, 1, 1), (5, 7, 3), (257, 513, 255), (129, 2050, 67)])
@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_lognormal_parity(gpu_lib, shape, path):
    m, k, n = shape
    print(f"[balance] lognormal {path} {shape}", flush=True)
    A, B = lognormal_product(m, k, n, seed=300 + m + k)
    if path == "fp64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    C, ps = _run(gpu_lib, A, B, P128, path)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path], balance=True)
    print(compare_estimate(C, ps, ref, P128, path), flush=True)


@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_inner_scaled_batched_with_zero_lines(gpu_lib, path):
    """Batched inner-scaled inputs (16 decades), with a zero column of A in
    one item and a zero row of B in another (d = 1 there)."""
    A, B = inner_scaled(200, 300, 150, seed=41, decades=8, batch=3)
    A[0, :, 17] = 0.0
    B[1, 40, :] = 0.0
    dt = np.float64 if path == "fp64" else np.float32
    A, B = A.astype(dt), B.astype(dt)
    print(f"[balance] inner-scaled batched {path}", flush=True)
    C, ps = _run(gpu_lib, A, B, P128, path)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path], balance=True)
    print(compare_estimate(C, ps, ref, P128, path), flush=True)
    # against the unbalanced GPU estimate: higher p*, smaller error vs exact
    C0, ps0 = gpu_lib.estimate(_dev(A), _dev(B), P=P128, path=path, return_pstar=True)
    C0, ps0 = C0.cpu().numpy(), ps0.cpu().numpy()
    E = oracle.exact_maxtimes(A, B)
    p_bal = np.asarray(P128)[np.where(ps == 255, 0, ps)]
    p_pln = np.asarray(P128)[np.where(ps0 == 255, 0, ps0)]
    assert p_bal.mean() > 4 * p_pln.mean()
    err_bal = np.abs(C / E - 1).max()
    err_pln = np.abs(C0 / E - 1).max()
    print(f"   max rel err vs exact: balanced {err_bal:.3e}, plain {err_pln:.3e}", flush=True)
    assert err_bal < 0.1 * err_pln


def test_two_term_closed_form(gpu_lib):
    """A = [1, 1e-20], B = [1e-20; 1]: balanced, both scaled terms are 1,
    p* = 128 and C = 1e-20 2^(1/128); unbalanced p* = 1 and C = 2e-20."""
    A = np.array([[1.0, 1e-20]], dtype=np.float32)
    B = np.array([[1e-20], [1.0]], dtype=np.float32)
    C, ps = _run(gpu_lib, A, B, P128, "bf16")
    assert ps[0, 0] == 7
    a = float(np.float32(1e-20))
    assert math.isclose(float(C[0, 0]), a * 2.0 ** (1 / 128), rel_tol=2e-3)
    C0, ps0 = gpu_lib.estimate(_dev(A), _dev(B), P=P128, path="bf16", return_pstar=True)
    assert int(ps0[0, 0]) == 0


@pytest.mark.parametrize("path", ["bf16", "fp64"])
@pytest.mark.parametrize("thr,start", [(65536, None), (512, 2)])
def test_tail_and_search_start(knobs, path, thr, start):
    A, B = lognormal_product(300, 700, 280, seed=44)
    if path == "fp64":
        A, B = A.astype(np.float64), B.astype(np.float64)
    knobs.set_tail_threshold(thr)
    if start is not None:
        knobs.set_search_start(start)
    print(f"[balance] {path} tail {thr} start {start}", flush=True)
    C, ps = _run(knobs, A, B, P128, path)
    ref = oracle.pnorm_estimate(A, B, P128, TAU[path], balance=True)
    compare_estimate(C, ps, ref, P128, path)


def test_pilot_sized_product_sampled_rows(gpu_lib):
    """2048 x 512 x 2048 (the pilot picks the search start above 2^22
    outputs): 64 sampled rows against the oracle, the factors taken from the
    whole inputs."""
    A, B = lognormal_product(2048, 512, 2048, seed=45)
    rows = np.sort(np.random.default_rng(46).choice(2048, 64, replace=False))
    print("[balance] pilot-sized bf16", flush=True)
    C, ps = _run(gpu_lib, A, B, P128, "bf16")
    ref = oracle.pnorm_estimate_rows(A, B, P128, TAU["bf16"], rows, balance=True)
    compare_estimate(C[rows], ps[rows], ref, P128, "bf16")


def test_fp64_io_on_bf16_path(gpu_lib):
    A, B = inner_scaled(150, 220, 130, seed=47, decades=30)
    print("[balance] fp64 I/O bf16 path, 60 decades of inner scale", flush=True)
    C, ps = _run(gpu_lib, A, B, P128, "bf16")
    ref = oracle.pnorm_estimate(A, B, P128, TAU["bf16"], balance=True)
    compare_estimate(C, ps, ref, P128, "bf16")


@pytest.mark.parametrize("path", ["fp64", "bf16"])
def test_gradient_through_balanced_forward(gpu_lib, path):
    """The backward of a balanced forward works on the balanced pair and
    takes the result back by d (the scaled quantities of the unbalanced
    pair underflow here: C' ~ 1e-6 at p* = 64); against the oracle's
    balanced gradient at the path's tolerance."""
    A, B = inner_scaled(64, 96, 48, seed=48, decades=3)
    G = np.random.default_rng(49).standard_normal((64, 48))
    if path == "bf16":
        A, B, G = A.astype(np.float32), B.astype(np.float32), G.astype(np.float32)
    Ad = _dev(A).requires_grad_(True)
    Bd = _dev(B).requires_grad_(True)
    P = [1, 2, 4, 8, 16, 32, 64]
    print(f"[balance] gradient {path}", flush=True)
    C, ps = gpu_lib.estimate(Ad, Bd, P=P, path=path, return_pstar=True, balance=True)
    (C * _dev(G)).sum().backward()
    ps = ps.cpu().numpy()
    assert (ps == 6).mean() > 0.99
    rA, rB = oracle.pnorm_grad(A, B, G, P, ps, balance=True)
    gA = Ad.grad.cpu().numpy().astype(np.float64)
    gB = Bd.grad.cpu().numpy().astype(np.float64)
    assert np.isfinite(gA).all() and np.isfinite(gB).all()
    tol = 1e-5 if path == "fp64" else 2e-3
    eA = np.linalg.norm(gA - rA) / np.linalg.norm(rA)
    eB = np.linalg.norm(gB - rB) / np.linalg.norm(rB)
    print(f"   rel err dA {eA:.2e} dB {eB:.2e}", flush=True)
    assert eA <= tol and eB <= tol


def test_apsp_rejects_the_flag(gpu_lib):
    import torch

    W = torch.rand(16, 16, device="cuda")
    lib = gpu_lib.load_library()
    o = gpu_lib._options([1, 2, 4], "fp64", None, None, gpu_lib.FLAG_BALANCE)
    import ctypes

    n = ctypes.c_size_t(0)
    assert lib.apsp_workspace_size(16, ctypes.byref(o), ctypes.byref(n)) == 1
    del W
