"""Parity at the benchmark's full sizes, in the same launch configuration
the benchmark times: 256^2 FP64 (whole output) and 8192^2 log-normal FP32
on both paths (sampled output rows, which the oracle computes one by one)."""

import numpy as np
import pytest

import oracle
from oracle import exact_c
from parity import TAU, compare_estimate
from workloads import config

pytestmark = pytest.mark.gpu


def test_config1_256_fp64_full(gpu_lib):
    import torch

    cfg = config(1)
    A, B, P = cfg["A"], cfg["B"], cfg["P"]
    print("[full] 256^2 fp64", flush=True)
    C, ps = gpu_lib.estimate(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), P=P,
                             path="fp64", return_pstar=True)
    C, ps = C.cpu().numpy(), ps.cpu().numpy()
    ref = oracle.pnorm_estimate(A, B, P, TAU["fp64"])
    st = compare_estimate(C, ps, ref, P, "fp64")
    E = oracle.exact_maxtimes(A, B)
    err = np.abs(C / E - 1).max()
    print(st, "max rel err vs exact", err, flush=True)
    assert st["max_rel"] < 1e-12
    assert err <= 256 ** (1 / 64) - 1 + 1e-9


@pytest.fixture(scope="module")
def config3():
    import torch

    cfg = config(3)
    A, B = cfg["A"], cfg["B"]
    rows = np.sort(np.random.default_rng(3003).choice(A.shape[0], 64, replace=False))
    return cfg, torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(), rows


@pytest.mark.slow
@pytest.mark.parametrize("path", ["bf16", "fp64"])
def test_config3_8192_sampled_rows(gpu_lib, config3, path):
    cfg, Ad, Bd, rows = config3
    A, B, P = cfg["A"], cfg["B"], cfg["P"]
    print(f"[full] 8192^2 {path}", flush=True)
    C, ps = gpu_lib.estimate(Ad, Bd, P=P, path=path, return_pstar=True)
    Cr = C[torch_index(rows)].cpu().numpy()
    pr = ps[torch_index(rows)].cpu().numpy()
    del C, ps
    ref = oracle.pnorm_estimate_rows(A, B, P, TAU[path], rows)
    st = compare_estimate(Cr, pr, ref, P, path)
    E = exact_c.exact_maxtimes_c(A, B, rows)
    err = np.abs(Cr / E - 1)
    print(st, f"rel err vs exact: max {err.max():.3e} median {np.median(err):.3e}", flush=True)


def torch_index(rows):
    import torch

    return torch.from_numpy(rows).cuda()
