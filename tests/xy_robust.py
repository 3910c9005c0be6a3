"""How deep a top-k pop sequence of x + y is insensitive to the rounding of
its ring results (test infrastructure, CPU only).

The NormQueue (Sec. 2.3, algorithm E) subtracts psi^p from the ring results
of a popped diagonal; where what is left is small, the absolute rounding of
an FFT-computed ring result decides the later pops (the accumulation of
error Sec. 3 reports).  Here the oracle's queue runs on ring results that
carry such rounding: numpy's FFT at three transform lengths.  The robust
depth is the number of leading ranks on which all three give the oracle's
direct-convolution sequence: the diagonals of both runs exactly and the
values within atol.  It is necessary, not sufficient, for a GPU sequence to
agree that deep: the GPU's FFT rounds more coarsely than numpy's (within
the bound 40 log2(N) u |x'^p| |y'^p| its ring results are tested against,
under which almost any list loses its sequence after a pop or two)."""

import math

import numpy as np

from oracle.xy_topk import queue_pops, xy_topk_estimate


def fft_ring_results(x, y, P, N):
    """sigma^(p) = x'^p * y'^p by a length-N real FFT (N >= len x + len y - 1),
    with the scale-backs max x and max y."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    mx, my = x.max(), y.max()
    xs, ys = np.exp(x - mx), np.exp(y - my)
    L = x.size + y.size - 1
    rows = [np.fft.irfft(np.fft.rfft(xs ** p, N) * np.fft.rfft(ys ** p, N), N)[:L] for p in P]
    return np.stack(rows), mx, my


def robust_depth(x, y, P, k, atol=1e-6):
    """Leading ranks (at most k) of the top k of x + y that do not depend on
    the ring results' rounding (see the module docstring)."""
    ref = xy_topk_estimate(x, y, P, k)
    n = len(x)
    N0 = max(16, 1 << math.ceil(math.log2(2 * n - 1)))
    depth = k
    for N in (N0, 2 * N0, 4 * N0):
        for yy, key in ((np.asarray(y), "diag"), (np.asarray(y)[::-1], "anti")):
            sigma, mx, my = fft_ring_results(x, yy, P, N)
            out = queue_pops(sigma, mx, my, P, k)
            ok = out["diag"] == ref[key]
            if key == "diag":
                ok &= np.abs(out["values"] - ref["values"]) <= atol
            bad = np.flatnonzero(~ok)
            if bad.size:
                depth = min(depth, int(bad[0]))
    return depth
