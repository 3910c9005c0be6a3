"""CPU oracle for the p-norm (max, x) product estimate and its APSP by repeated squaring.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package.  The product path (``paper_1511_05690_amd``) never
imports it and shares no code with it: no kernels, headers, helpers, tables
or constant generators.  The only thing both sides use is the seeded input
generator package ``workloads``, which holds none of the method's arithmetic.

Everything here is plain and slow on purpose: FP64 numpy (plus one plain C
loop for the exact product at large sizes), written from Serang,
"Fast Computation on Semirings Isomorphic to (x, max) on R+"
(arXiv 1511.05690).  Each function cites the passage it follows.

Modules
-------
pnorm   exact (max, x) product (Alg. 2), the p-norm estimate (Alg. 5 with the
        scaled ring call H' of Sec. 2.1), and its analytic gradient.
apsp    the (+, min) <-> (x, max) transform (Sec. 2.2), APSP by repeated
        squaring, Floyd-Warshall and Dijkstra, and the affine correction of
        an APSP estimate fitted on a few exact distances (Sec. 4).
maxconv the max-convolution (Sec. 1), exact and its p-norm estimate.
exact_c ctypes wrapper of ``exact_maxtimes.c`` (same definition as
        ``pnorm.exact_maxtimes``, for sizes numpy cannot finish quickly).

Parity status: every function is pinned by ``tests/test_oracle_*.py``
against closed forms, invariants, brute force or library routines; none is
"parity unpinned".
"""

from .pnorm import (  # noqa: F401
    exact_maxtimes,
    exact_maxtimes_loops,
    scale_factors,
    balance_factors,
    balanced,
    norm_power_sequence,
    select_pstar,
    pnorm_estimate,
    pnorm_estimate_rows,
    pnorm_grad,
    pnorm_forward_fixed,
    PSTAR_NONE,
)
from .apsp import (  # noqa: F401
    to_maxtimes,
    to_distances,
    apsp_by_squaring,
    apsp_estimate,
    apsp_exact_squaring,
    default_squarings,
    floyd_warshall,
    dijkstra,
    affine_fit,
    affine_apply,
)
from .maxconv import TAU_FFT, exact_maxconv, maxconv_estimate  # noqa: F401,E402
from .xy_topk import exact_topk_xy, norm_queue, xy_topk_estimate, xy_topk_paired  # noqa: F401,E402
