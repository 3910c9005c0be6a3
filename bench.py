#!/usr/bin/env python3
"""Benchmark of the p-norm (max, x) product estimate on one MI355X.

Workload (the configuration the metric compares the BF16 and FP64 paths
on): C ~ max_k A_ik B_kj for A, B of 8192 x 8192, entries exp(N(0, 2^2))
clipped to (0, 1e6], stored FP32; family P = {1, 2, ..., 128}; BF16 MFMA
ring products with FP32 accumulation and hi/lo split for p <= 4.  A step is
one maxtimes_estimate call (row/column maxima, power planes, fused p-family
GEMM with the per-entry selection and root) on inputs resident in HBM.

value = n^3 / t_step (effective max-times ops/s).  The FP64 path is timed on
the same inputs; both are checked against the exact product (computed on
the GPU by the library's exact kernel) on 1024 sampled rows.  The oracle is
timed on the host on a bounded row sample (cpu_baseline).

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# rows of C checked against the exact product (every entry of each)
ERR_ROWS = 1024
METRIC = "effective max-times ops/s (n³/t) BF16 vs FP64 path; max rel. err vs exact"
BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
FP64_PEAK_TFLOPS = 78.6     # MI355X FP64 matrix
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (256 CUs x 128 flop/clk x 2.4 GHz)
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "pfamily_gemm_bf16_8192_pmc.md")
TRACE_SUMMARY = os.path.join(ROOT, "profiles", "pfamily_gemm_bf16_8192_kernel_trace.md")
GEMM_SRC = os.path.join(ROOT, "paper_1511_05690_amd", "csrc", "mt_gemm_bf16.hip")
MAXCONV_PMC = os.path.join(ROOT, "profiles", "maxconv_fft_8192x2048_pmc.md")
MAXCONV_SRC = os.path.join(ROOT, "paper_1511_05690_amd", "csrc", "mt_maxconv.hip")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic_from_profile(summary=PMC_SUMMARY, src=GEMM_SRC):
    """HBM bytes per launch of a kernel from its committed rocprofv3 counter
    summary, if the summary was taken on the current kernel source."""
    if not os.path.exists(summary):
        return None
    text = open(summary).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_bytes = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not m_hash or not m_bytes or m_hash.group(1) != source_hash(src):
        return None
    return float(m_bytes.group(1))


def trace_from_profile(summary, src, kernel):
    """Average duration (ms) of `kernel` in a committed rocprofv3 kernel-trace
    summary, if it was taken on the current kernel source."""
    if not os.path.exists(summary):
        return None
    text = open(summary).read()
    m_hash = re.search(r"kernel_source_sha256_16:\s*([0-9a-f]+)", text)
    m_avg = re.search(r"^" + re.escape(kernel) + r"_avg_ms:\s*([0-9.eE+-]+)", text, re.M)
    if not m_hash or not m_avg or m_hash.group(1) != source_hash(src):
        return None
    return float(m_avg.group(1))


def gemm_segments(P, split_max_p=4):
    return sum(3 if p <= split_max_p else 1 for p in P)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / steps, wall


def cpu_baseline(A, B, P, tau, rows):
    """The oracle as it stands, on a bounded sample of output rows."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle

    t0 = time.perf_counter()
    oracle.pnorm_estimate_rows(A, B, P, tau, rows)
    dt = time.perf_counter() - t0
    n = B.shape[1]
    k = A.shape[1]
    blas = [p for p in threadpool_info() if p.get("user_api") == "blas"]
    threads = max([p.get("num_threads", 1) for p in blas] or [1])
    return {
        "value": len(rows) * k * n / dt,
        "unit": "max-times ops/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": (f"{len(rows)} of {A.shape[0]} output rows of the same 8192^2 workload "
                   f"(FP64 numpy: powers of all of B, {len(P)} BLAS GEMMs of {len(rows)}x{k}x{n}); "
                   f"{dt:.1f} s; elementwise numpy steps run on 1 thread, BLAS on {threads}; "
                   f"host logical CPUs {os.cpu_count()}"),
        "seconds": dt,
    }


def hbm_kernels(kern_ms, n, P, path, in_bytes=4, deferred=False):
    """Achieved HBM rate of the bandwidth-bound kernels of one step, from
    their algorithmic bytes (each input read once, each output written once)
    and the in-process launch times (ms per step).  deferred: the plane
    launches write no planes of the two smallest p (BF16 path) or of all but
    the three largest p (FP64 path); those are written later, and only if some
    entry needs them."""
    n2 = float(n) * n
    if path == "bf16":
        written = sorted(P)[2:] if deferred else P
        planes = sum(2 if p <= 4 else 1 for p in written)
        plane_bytes = 2 * (n2 * in_bytes + n2 * 2 * planes)  # both operands
    else:
        written = sorted(P)[-3:] if deferred else P
        plane_bytes = 2 * (n2 * in_bytes + n2 * 8 * len(written))
    if "mt_colmax" not in kern_ms:
        # B's column maxima ran inside the plane launches (one more read of B)
        plane_bytes += n2 * in_bytes
    algo = {
        "mt_rowmax": n2 * in_bytes,
        "mt_colmax": n2 * in_bytes,
        "mt_power_planes": plane_bytes,
        "mt_select_root": n2 * (8 + 1 + in_bytes),
    }
    out = {}
    for k, b in algo.items():
        ms = kern_ms.get(k)
        if ms:
            gbs = b / (ms / 1e3) / 1e9
            out[k] = {"ms": ms, "bytes": b, "GB/s": gbs, "frac_of_8TB/s": gbs / 8000.0}
    return out


def pfamily_128():
    return [1, 2, 4, 8, 16, 32, 64, 128]


def time_call(fn, reps, torch):
    fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / reps


def run_legs(mt, torch, np, sections=None):
    """The other rows of the hot path, each on its own workload: APSP on the
    FP64 and BF16 paths, the differentiable form, and the small FP64 product.
    Effective max-times ops: T n^3 for APSP, b m k n per product."""
    from workloads import config

    def want(name):
        return sections is None or name in sections

    legs = {}
    if want("small"):
        c1 = config(1)
        A1, B1 = torch.from_numpy(c1["A"]).cuda(), torch.from_numpy(c1["B"]).cuda()
        ms = time_call(lambda: mt.estimate(A1, B1, P=c1["P"], path="fp64"), 20, torch)
        # the product runs as one kernel (the small-product path); its span
        # on the device clock beside the whole call as Python issues it
        mt.timing_reset()
        mt.timing_enable(True)
        time_call(lambda: mt.estimate(A1, B1, P=c1["P"], path="fp64"), 20, torch)
        kms, kn = mt.timing_span("mt_small_product_f64")
        klaunch = mt.timing_read("mt_")[1]
        mt.timing_enable(False)
        mt.timing_reset()
        legs["product_256_fp64"] = {"ms": ms, "ops_per_s": 256.0 ** 3 / (ms / 1e3), "P": c1["P"],
                                    "kernel_ms": kms / kn if kn else None,
                                    "launches_per_call": klaunch / 21.0,
                                    "kernel": "mt_small_product_f64 (one launch per product)"}

    if want("apsp2048"):
        c2 = config(2)
        W2 = torch.from_numpy(c2["W"]).cuda()
        n2 = c2["W"].shape[0]
        # exact APSP on the GPU for the error columns: T squarings of the exact
        # (max, x) product (the library's VALU kernel) on X = exp(-s W)
        X = torch.exp(-c2["s"] * W2.double())
        X.fill_diagonal_(1.0)
        for _ in range(c2["T"]):
            X = mt.exact(X, X)
            X.fill_diagonal_(1.0)
        D_ex = -torch.log(X) / c2["s"]
        fin = torch.isfinite(D_ex)
        for proj in (None, "r1", "r2"):
            ms = time_call(lambda: mt.apsp(W2, s=c2["s"], P=c2["P"], path="fp64", n_squarings=c2["T"],
                                           out_dtype=torch.float64, projection=proj), 3, torch)
            D = mt.apsp(W2, s=c2["s"], P=c2["P"], path="fp64", n_squarings=c2["T"], out_dtype=torch.float64,
                        projection=proj)
            err = (D - D_ex)[fin]
            xrel = (torch.exp(-c2["s"] * D[fin]) / torch.exp(-c2["s"] * D_ex[fin]) - 1.0).abs()
            name = "apsp_er2048_fp64" + ("_" + proj if proj else "")
            legs[name] = {"ms": ms, "squarings": c2["T"], "P": c2["P"], "projection": proj or "plain",
                          "ops_per_s": c2["T"] * float(n2) ** 3 / (ms / 1e3),
                          "vs_exact": {"distance_mse": float((err ** 2).mean()), "max_abs": float(err.abs().max()),
                                       "mean": float(err.mean()), "max_rel_x": float(xrel.max()),
                                       "reachability_equal": bool(torch.equal(torch.isfinite(D), fin))}}
            # the affine correction (Sec. 4) fitted on the exact rows of 64
            # sampled sources (Bellman-Ford on the GPU), timed with them
            src = np.random.default_rng(2002).choice(n2, 64, replace=False).astype(np.int32)

            def correct():
                rows, _ = mt.apsp_exact_rows(W2, src)
                return rows, mt.apsp_affine_correct(D, src, rows, apply=False)
            ms_fit = time_call(correct, 3, torch)
            rows, ab = correct()
            Dc = D.clone()
            ab = mt.apsp_affine_correct(Dc, src, rows)
            errc = (Dc - D_ex)[fin]
            a_, b_ = [float(x) for x in ab.cpu()]
            legs[name]["affine_64_sources"] = {"ms_exact_rows_and_fit": ms_fit, "a": a_, "b": b_,
                                               "distance_mse": float((errc ** 2).mean()),
                                               "max_abs": float(errc.abs().max()), "mean": float(errc.mean())}

    if want("grad"):
        c4 = config(4)
        A4 = torch.from_numpy(c4["A"]).cuda()
        B4 = torch.from_numpy(c4["B"]).cuda()
        G4 = torch.from_numpy(c4["G"]).cuda()
        for name, P in (("grad_64x512_p16_bf16", c4["P_fixed"]), ("grad_64x512_bf16", c4["P"])):
            def fwd_bwd():
                C, ps = mt.estimate(A4, B4, P=P, path="bf16", split_max_p=4096, return_pstar=True)
                mt.estimate_backward(A4, B4, G4, C, ps, P, path="bf16")
            ms = time_call(fwd_bwd, 5, torch)
            legs[name] = {"ms_fwd_bwd": ms, "P": P, "ops_per_s": 64 * 512.0 ** 3 / (ms / 1e3)}

    if want("balance"):
        # inner-index balancing on inputs whose inner index carries a scaling:
        # A = U diag(s), B = diag(s)^-1 V, U, V uniform on (0, 1], log10 s
        # uniform on [-8, 8], 4096^3, P = {1..128}, BF16; error against the exact
        # product on 256 sampled rows, plain and balanced
        nb = 4096
        g = torch.Generator(device="cuda")
        g.manual_seed(6006)
        sc = torch.pow(10.0, torch.rand(nb, generator=g, device="cuda", dtype=torch.float64) * 16 - 8)
        Ab = ((1.0 - torch.rand(nb, nb, generator=g, device="cuda", dtype=torch.float64)) * sc[None, :]).float()
        Bb = ((1.0 - torch.rand(nb, nb, generator=g, device="cuda", dtype=torch.float64)) / sc[:, None]).float()
        rb = torch.from_numpy(np.sort(np.random.default_rng(6007).choice(nb, 256, replace=False))).cuda()
        Eb = mt.exact(Ab[rb].contiguous(), Bb).double()
        leg = {"n": nb, "P": pfamily_128(), "inner_scale_decades": 16}
        for tag, balance in (("plain", False), ("balanced", True)):
            ms = time_call(lambda: mt.estimate(Ab, Bb, P=pfamily_128(), path="bf16", balance=balance), 3, torch)
            C, ps = mt.estimate(Ab, Bb, P=pfamily_128(), path="bf16", balance=balance, return_pstar=True)
            rel = (C[rb].double() / Eb - 1.0).abs()
            psel = ps[rb].flatten().long()
            leg[tag] = {"ms": ms, "max_rel_vs_exact": float(rel.max()), "median_rel_vs_exact": float(rel.median()),
                        "pstar_hist": torch.bincount(psel, minlength=256)[:8].tolist()}
        legs["balance_inner_scaled_4096_bf16"] = leg
        del Ab, Bb, Eb, C, ps
        torch.cuda.empty_cache()

    if want("maxconv"):
        # max-convolution (Sec. 1): 8192 pairs of 2048-point probability vectors
        # (Dirichlet(1) rows), P = {1, ..., 64}, FFT convolution in FP64
        from workloads import maxconv_vectors, pfamily
        bm, nm = 8192, 2048
        xc, yc = maxconv_vectors(bm, nm, nm, seed=4004, kind="distribution")
        xd, yd = torch.from_numpy(xc).cuda(), torch.from_numpy(yc).cuda()
        del xc, yc
        Pm = pfamily(64)
        mt.timing_reset()
        mt.timing_enable(True)
        ms = time_call(lambda: mt.maxconv(xd, yd, Pm), 5, torch)
        kev_ms, kev_n = mt.timing_read("mt_maxconv")
        kms, kn = mt.timing_span("mt_maxconv")
        kflop = mt.timing_work("mt_maxconv")
        mt.timing_reset()
        ms_exact = time_call(lambda: mt.maxconv_exact(xd, yd), 1, torch)
        mt.timing_enable(False)
        z, ps = mt.maxconv(xd, yd, Pm, return_pstar=True)
        E = mt.maxconv_exact(xd, yd)
        pos = E > 0
        rel = (z[pos] / E[pos] - 1.0).abs()
        hist = torch.bincount(ps.flatten().long(), minlength=256)[:len(Pm)].tolist()
        achieved = kflop / kn / (kms / kn / 1e3) / 1e12
        legs["maxconv_8192x2048_fp64"] = {
            "ms": ms, "pairs": bm, "n": nm, "m": nm, "P": Pm,
            "ops_per_s": bm * float(nm) * nm / (ms / 1e3),
            "roofline": {"bound": "alu", "kernel": "mt_maxconv", "achieved": achieved,
                         "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                         "traffic": traffic_from_profile(MAXCONV_PMC, MAXCONV_SRC),
                         "flop_per_launch": kflop / kn, "avg_launch_ms": kms / kn,
                         "avg_launch_ms_source": "device real-time counter (maxtimes_timing_span)",
                         "avg_launch_ms_events": kev_ms / max(kev_n, 1),
                         "flop_count": "10 N log2 N per pair and p visited (two complex FFTs), N = 4096"},
            "exact_ms": ms_exact, "speedup_vs_exact": ms_exact / ms,
            "vs_exact": {"max_rel": float(rel.max()), "median_rel": float(rel.median())},
            "pstar_hist": hist,
        }
        del xd, yd, z, ps, E, pos, rel
        torch.cuda.empty_cache()

    if want("xy"):
        # top k of x + y (Sec. 2.3, the n = 8192, k = 256 case of Sec. 3): uniform
        # lists on [0, 1] and on [0, 40], the 24-power family up to 4096, the
        # plain queue and the paired one (Discussion); exact top k on the GPU by
        # torch over all n^2 sums, for the accuracy columns
        nx, kx = 8192, 256

        def lists(spread):
            rng = np.random.default_rng(5005)
            return (torch.from_numpy(rng.uniform(0, spread, nx)).cuda(),
                    torch.from_numpy(rng.uniform(0, spread, nx)).cuda())

        def accuracy(xs, ys, paired):
            v, ii, jj = mt.xy_topk(xs, ys, kx, paired=paired)
            ev, eidx = torch.topk((xs[:, None] + ys[None, :]).flatten(), kx)
            ei, ej = (eidx // nx).int(), (eidx % nx).int()
            return {"indices_found_at_rank": int(((ii == ei) & (jj == ej)).sum()),
                    "true_top_k_pairs_found": int(torch.isin(ii.long() * nx + jj.long(), eidx).sum()), "k": kx,
                    "max_abs_value_err_first_16": float((v[:16] - ev[:16]).abs().max()),
                    "max_abs_value_err": float((v - ev).abs().max())}

        xs, ys = lists(1)
        leg = {"n": nx, "k": kx, "P": list(mt.XY_FAMILY)}
        for paired, tag in ((False, ""), (True, "paired_")):
            mt.timing_reset()
            mt.timing_enable(True)
            leg[tag + "ms"] = time_call(lambda: mt.xy_topk(xs, ys, kx, paired=paired), 3, torch)
            names = ("mt_xy_sigma", "mt_xy_psi", "mt_xy_select", "mt_xy_paired" if paired else "mt_xy_queue")
            leg[tag + "kernel_ms"] = {name: mt.timing_read(name)[0] / 4 for name in names}
            mt.timing_enable(False)
        leg["naive_gpu_topk_ms"] = time_call(lambda: torch.topk((xs[:, None] + ys[None, :]).flatten(), kx), 3, torch)
        for spread in (1, 40):
            xs, ys = lists(spread)
            for paired, tag in ((False, ""), (True, "paired_")):
                leg[f"{tag}vs_exact_uniform_0_{spread}"] = accuracy(xs, ys, paired)
        legs["xy_topk_8192_k256_fp64"] = leg
        del xs, ys
        torch.cuda.empty_cache()

    if want("rgg"):
        # APSP on the 16384-vertex random geometric graph (radius 0.02, weights
        # 100 x length, s = 0.35, 14 squarings, P = {1..128}) on the BF16 path,
        # and once on the FP64 path for comparison; errors against exact rows
        # from 64 sampled sources (Bellman-Ford on the GPU, the library's
        # apsp_exact_rows)
        c5 = config(5)
        W5 = torch.from_numpy(c5["W"]).cuda()
        del c5["W"]
        n5 = W5.shape[0]
        src5 = np.sort(np.random.default_rng(5006).choice(n5, 64, replace=False)).astype(np.int32)
        ex5, rounds5 = mt.apsp_exact_rows(W5, src5)
        si = torch.from_numpy(src5.astype(np.int64)).cuda()
        # the plain estimate's far pairs sit at small p* (e^(-s d) to the power p
        # must stay above tau), so its error grows with the distance; the r = 1
        # projection (exact for tied top terms) and the affine correction fitted
        # on the same exact rows are reported beside it
        for path, proj in (("bf16", None), ("bf16", "r1"), ("fp64", None)):
            if path == "bf16":  # one untimed call first; the FP64 run (seconds) is timed once, cold
                mt.apsp(W5, s=c5["s"], P=c5["P"], path=path, n_squarings=c5["T"], out_dtype=torch.float64,
                        projection=proj)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            D5 = mt.apsp(W5, s=c5["s"], P=c5["P"], path=path, n_squarings=c5["T"], out_dtype=torch.float64,
                         projection=proj)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1)
            leg = {"ms": ms, "squarings": c5["T"], "P": c5["P"], "s": c5["s"], "projection": proj or "plain",
                   "ops_per_s": c5["T"] * float(n5) ** 3 / (ms / 1e3),
                   "vs_exact_64_sources": apsp_errors(D5[si], ex5, c5["s"], torch),
                   "exact_rows": {"sources": len(src5), "bellman_ford_rounds": rounds5}}
            if path == "bf16":
                # the squarings' GEMM on the device clock, with the MFMA work
                # its launches executed (one more call with per-launch timing)
                mt.timing_reset()
                mt.timing_enable(True)
                mt.apsp(W5, s=c5["s"], P=c5["P"], path=path, n_squarings=c5["T"], out_dtype=torch.float64,
                        projection=proj)
                torch.cuda.synchronize()
                g_ms, g_n = mt.timing_span("mt_pfamily_gemm_bf16")
                g_work = mt.timing_work("mt_pfamily_gemm_bf16")
                mt.timing_enable(False)
                mt.timing_reset()
                if g_n:
                    leg["gemm"] = {"launches": g_n, "ms_per_launch": g_ms / g_n, "flop_per_launch": g_work / g_n,
                                   "tflops": g_work / (g_ms / 1e3) / 1e12,
                                   "frac_of_bf16_peak": g_work / (g_ms / 1e3) / 1e12 / BF16_PEAK_TFLOPS}
            Dc = D5.clone()
            ab = mt.apsp_affine_correct(Dc, src5, ex5)
            leg["affine_64_sources"] = dict(apsp_errors(Dc[si], ex5, c5["s"], torch),
                                            a=float(ab[0]), b=float(ab[1]),
                                            note="fitted on the same 64 rows it is scored on")
            legs["apsp_rgg16384_" + path + ("_" + proj if proj else "")] = leg
            del D5, Dc
            torch.cuda.empty_cache()

    return legs


def apsp_errors(D, E, s, torch):
    """Errors of estimated distances D against exact ones E (same shape, FP64
    on the device): distance MSE, mean and largest absolute error over
    pairs with a finite exact distance (the paper's MSE, Table 1); the
    largest relative error in (x, max) space, |e^(-s d) / e^(-s d_exact) - 1|;
    pairs at a positive exact distance estimated at 0 (the clamp X <= 1);
    pairs with a finite exact distance estimated unreachable, and the
    reverse."""
    fin = torch.isfinite(E)
    est_fin = torch.isfinite(D)
    both = fin & est_fin
    err = (D - E)[both]
    xrel = (torch.exp(-s * (D[both] - E[both])) - 1.0).abs()
    off = E > 0
    return {"pairs": int(fin.sum()), "distance_mse": float((err ** 2).mean()),
            "mean": float(err.mean()), "max_abs": float(err.abs().max()),
            "max_rel_x": float(xrel.max()), "median_rel_x": float(xrel.median()),
            "clamped_to_zero": int((off & fin & (D == 0)).sum()),
            "finite_estimated_inf": int((fin & ~est_fin).sum()),
            "inf_estimated_finite": int((~fin & est_fin).sum())}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--only", choices=["bf16", "fp64"], default=None,
                    help="time one path only (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-rows", type=int, default=128)
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the APSP / gradient / small-product legs")
    ap.add_argument("--legs", default=None,
                    help="comma-separated leg sections to run (small, apsp2048, grad, balance, maxconv, xy, rgg); "
                         "with --only-legs, nothing else is timed (profiling runs)")
    ap.add_argument("--only-legs", action="store_true", help="run only the legs (profiling runs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only run a device-to-device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {max(args.gpus, world)}): the p-norm "
              "product is measured on one MI355X; the multi-GPU sharding is a design, not built.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calib_copy_mib:
        nbytes = args.calib_copy_mib << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calib_copy_bytes": nbytes, "launches": 3}))
        return

    import paper_1511_05690_amd as mt
    from workloads import config

    mt.load_library()
    sections = set(args.legs.split(",")) if args.legs else None
    if args.only_legs:
        print(json.dumps({"legs": run_legs(mt, torch, np, sections)}))
        return
    log("[bench] generating the 8192^2 log-normal workload")
    cfg = config(3)
    A, B, P = cfg["A"], cfg["B"], cfg["P"]
    n = A.shape[0]
    Ad = torch.from_numpy(A).cuda()
    Bd = torch.from_numpy(B).cuda()
    torch.cuda.synchronize()
    ops = float(n) ** 3

    out = {}
    res = {}
    paths = [args.only] if args.only else ["bf16", "fp64"]
    for path in paths:
        steps = args.steps if path == "bf16" else args.fp64_steps
        warm = args.warmup if path == "bf16" else 1
        ws = torch.empty(mt.workspace_size(1, n, n, n, P, path=path), dtype=torch.uint8, device="cuda")
        holder = {}

        def step():
            holder["C"] = mt.estimate(Ad, Bd, P=P, path=path, workspace=ws)

        for _ in range(warm):
            step()
        torch.cuda.synchronize()
        log(f"[bench] timing {path}: {steps} steps")
        # the step time with the per-launch timing off, then the same steps
        # again with it on for the per-kernel times and executed flops
        ms, wall = time_steps(step, steps, 0, torch)
        mt.timing_reset()
        mt.timing_enable(True)
        time_steps(step, steps, 0, torch)
        mt.timing_enable(False)
        kname = "mt_pfamily_gemm_" + ("bf16" if path == "bf16" else "f64")
        gemm_ev_ms, gemm_ev_n = mt.timing_read(kname)
        # the GEMM's duration on the device clock (first workgroup start to
        # last workgroup end), which the roofline uses; the events around the
        # launch are reported beside it
        gemm_ms, gemm_n = mt.timing_span(kname)
        gemm_work = mt.timing_work(kname)
        kern = {}
        for kn in ("mt_rowmax", "mt_colmax", "mt_power_planes", "mt_planes_if", "mt_pilot", "mt_pfamily_gemm",
                   "mt_rerun_gemm", "mt_tail", "mt_select_root", "mt_fill"):
            t, c = mt.timing_read(kn)
            if c:
                kern[kn] = round(t / steps, 4)
        if gemm_n:
            kern["mt_pfamily_gemm"] = round(gemm_ms / steps, 4)  # device clock, as above
        # deferred planes: work of the tiles that ran again (0: no entry
        # needed the planes of the two smallest p)
        rerun_work = mt.timing_work("mt_rerun_gemm")
        mt.timing_reset()
        res[path] = {"ms_per_step": ms, "wall_s": wall, "gemm_ms": gemm_ms / max(gemm_n, 1),
                     "gemm_event_ms": gemm_ev_ms / max(gemm_ev_n, 1),
                     "gemm_launches": gemm_n, "gemm_flop": gemm_work / max(gemm_n, 1),
                     "rerun_flop_per_step": rerun_work / steps,
                     "kernel_ms_per_step": kern, "C": holder["C"]}
        del ws
        log(f"[bench] {path}: {ms:.3f} ms/step, GEMM {gemm_ms / max(gemm_n, 1):.3f} ms on the device clock "
            f"({gemm_ev_ms / max(gemm_ev_n, 1):.3f} ms between the launch's events)")

    # the BF16 path with inner-index balancing (MT_FLAG_BALANCE), timed the
    # same way, for its error column
    bal = None
    if "bf16" in res:
        ws = torch.empty(mt.workspace_size(1, n, n, n, P, path="bf16", flags=mt.FLAG_BALANCE), dtype=torch.uint8,
                         device="cuda")
        holder = {}

        def step_bal():
            holder["C"] = mt.estimate(Ad, Bd, P=P, path="bf16", workspace=ws, balance=True)

        for _ in range(args.warmup):
            step_bal()
        ms_bal, _ = time_steps(step_bal, max(3, args.steps // 4), 0, torch)
        bal = {"ms_per_step": ms_bal, "value": ops / (ms_bal / 1e3), "C": holder["C"]}
        del ws
        log(f"[bench] bf16 balanced: {ms_bal:.3f} ms/step")

    # error against the exact product on sampled rows (exact kernel on the GPU)
    rows = np.sort(np.random.default_rng(3003).choice(n, ERR_ROWS, replace=False))
    ri = torch.from_numpy(rows).cuda()
    Asub = Ad[ri].contiguous()
    E = mt.exact(Asub, Bd)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    E = mt.exact(Asub, Bd)
    ev1.record()
    torch.cuda.synchronize()
    exact_ms = ev0.elapsed_time(ev1)
    E64 = E.double()
    errs = {}
    for path in res:
        rel = (res[path]["C"][ri].double() / E64 - 1.0).abs()
        errs[path] = {"max": float(rel.max()), "median": float(rel.median())}
        del res[path]["C"]
    if bal is not None:
        rel = (bal.pop("C")[ri].double() / E64 - 1.0).abs()
        errs["bf16_balanced"] = {"max": float(rel.max()), "median": float(rel.median())}

    bf = res.get("bf16") or res[paths[0]]
    main_path = "bf16" if "bf16" in res else paths[0]
    seg = gemm_segments(P) if main_path == "bf16" else len(P)
    flop_family = 2.0 * n * n * n * seg
    # MFMA flops the GEMM executed (counted by the kernel): tiles stop once
    # every entry has its p*, so this is below the whole-family count
    flop = bf["gemm_flop"]
    achieved = flop / (bf["gemm_ms"] / 1e3) / 1e12
    peak = BF16_PEAK_TFLOPS if main_path == "bf16" else FP64_PEAK_TFLOPS
    traffic = traffic_from_profile() if main_path == "bf16" else None
    # the same launch in the committed rocprofv3 kernel trace (same source)
    rp_ms = trace_from_profile(TRACE_SUMMARY, GEMM_SRC, "mt_pfamily_gemm_bf16") if main_path == "bf16" else None

    value = ops / (bf["ms_per_step"] / 1e3)
    # the planes of the smaller p wait until some entry needs them (plain
    # products the pilot steers, families of five or more p)
    deferred = bool(mt.deferred_planes()) and len(P) >= 5
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "max-times ops/s",
        "n_gpus": 1,
        "steps": args.steps if main_path == "bf16" else args.fp64_steps,
        "warmup": args.warmup if main_path == "bf16" else 1,
        "ms_per_step": bf["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16" if main_path == "bf16" else "f64",
        "data": "synthetic",
        "config": {
            "workload": "8192^2 max-times product estimate, A,B = exp(N(0,2^2)) clipped to (0,1e6] "
                        "FP32, P={1..128}, " + ("BF16 MFMA + FP32 accumulation, hi/lo split p<=4"
                                                if main_path == "bf16" else "FP64 MFMA"),
            "n": n, "p_family": P, "path": main_path,
            "tau": 1e-30 if main_path == "bf16" else 1e-290,
        },
        "roofline": {
            "bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic,
            "kernel": "mt_pfamily_gemm_" + ("bf16" if main_path == "bf16" else "f64"),
            "flop_per_launch": flop,
            "flop_per_launch_whole_family": flop_family,
            "avg_launch_ms": bf["gemm_ms"],
            "avg_launch_ms_source": "device real-time counter, first workgroup start to last workgroup end "
                                    "(maxtimes_timing_span), per launch of the timed steps",
            "avg_launch_ms_events": bf["gemm_event_ms"],
            "rocprof_avg_launch_ms": rp_ms,
            "frac_at_rocprof_avg": (flop / (rp_ms / 1e3) / 1e12 / peak) if rp_ms else None,
        },
        "kernel_ms_per_step": bf["kernel_ms_per_step"],
        "hbm_kernels": hbm_kernels(bf["kernel_ms_per_step"], n, P, main_path, deferred=deferred),
        "deferred_planes": {"on": deferred, "rerun_flop_per_step": bf.get("rerun_flop_per_step", 0.0),
                            "late_planes_ms_per_step": bf["kernel_ms_per_step"].get("mt_planes_if", 0.0)},
        "max_rel_err_vs_exact": errs,
        "exact_valu": {"rows": len(rows), "ms": exact_ms,
                       "ops_per_s": len(rows) * float(n) * n / (exact_ms / 1e3)},
    }
    if bal is not None:
        out["bf16_balanced"] = {"ms_per_step": bal["ms_per_step"], "value": bal["value"],
                                "flag": "MT_FLAG_BALANCE (inner-index balancing, A D and D^-1 B)"}
    if "fp64" in res and main_path == "bf16":
        f = res["fp64"]
        fval = ops / (f["ms_per_step"] / 1e3)
        out["fp64_path"] = {
            "value": fval, "ms_per_step": f["ms_per_step"], "steps": args.fp64_steps,
            "gemm_ms": f["gemm_ms"],
            "gemm_flop": f["gemm_flop"],
            "gemm_flop_whole_family": 2.0 * n ** 3 * len(P),
            "gemm_tflops": f["gemm_flop"] / (f["gemm_ms"] / 1e3) / 1e12,
            "gemm_frac_of_fp64_peak": f["gemm_flop"] / (f["gemm_ms"] / 1e3) / 1e12 / FP64_PEAK_TFLOPS,
            "kernel_ms_per_step": f["kernel_ms_per_step"],
            "hbm_kernels": hbm_kernels(f["kernel_ms_per_step"], n, P, "fp64", deferred=deferred),
            "rerun_flop_per_step": f.get("rerun_flop_per_step", 0.0),
        }
        out["bf16_over_fp64"] = value / fval

    if not args.no_legs and args.only is None:
        log("[bench] legs: APSP (FP64 ER 2048, BF16 RGG 16384), gradient 64x512^3, 256^2 FP64, "
            "max-convolution 8192 x 2048, x + y top 256 at n = 8192")
        del Ad, Bd, E, E64, Asub
        torch.cuda.empty_cache()
        out["legs"] = run_legs(mt, torch, np, sections)

    if not args.no_cpu_baseline:
        log(f"[bench] cpu baseline: oracle on {args.cpu_rows} rows")
        out["cpu_baseline"] = cpu_baseline(A, B, P, 1e-30, rows[:args.cpu_rows])
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out))


if __name__ == "__main__":
    main()
