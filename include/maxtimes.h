/*
 * maxtimes.h -- C ABI of the MI355X (gfx950) p-norm (max, x) product library.
 *
 * The operation (Serang, "Fast Computation on Semirings Isomorphic to
 * (x, max) on R+", arXiv 1511.05690):
 *
 *   Exact product (Alg. 2, Sec. 2.2):   E_ij = max_k A_ik B_kj,  A, B >= 0.
 *   Estimate (Alg. 5 with the scaled ring call H' of Sec. 2.1):
 *       r_i = max_k A_ik,  c_j = max_k B_kj,  A' = A / r,  B' = B / c
 *       S_p = (A'^p) (B'^p)            one ordinary matrix product per p in P
 *       p*_ij = max{ p in P : S_p[i,j] >= tau }   (the highest stable p, Sec. 1)
 *       C_ij = r_i c_j S_{p*}[i,j]^(1/p*)          (the 1/p root of Sec. 1)
 *   It satisfies E <= C <= k^(1/p*) E (the error bound of Sec. 1).
 *   If no p is stable the smallest p of the family is used and p* is
 *   recorded as MT_PSTAR_NONE.  A zero row of A or column of B gives 0.
 *
 *   APSP (Sec. 2.2): X = exp(-s W) (no edge = +inf -> 0, diagonal -> 1),
 *   T squarings X <- est(X, X) each followed by X_ii <- 1 and X <- min(X, 1),
 *   then D = -log(X) / s (X = 0 -> +inf).  T defaults to ceil(log2 n)
 *   (the log n products of Sec. 1 and Sec. 2.2).
 *
 * Paths (mt_options.path):
 *   MT_PATH_FP64        powers, ring products and root in FP64 (FP64 MFMA).
 *   MT_PATH_BF16_SPLIT  powers in FP32, ring products as BF16 MFMA with FP32
 *                       accumulation; for p <= split_max_p each power is split
 *                       x = hi + lo (both BF16, round-to-nearest-even) and
 *                       S_p = hi.hi + hi.lo + lo.hi.  The stability test is
 *                       done in FP64 against tau.
 *
 * Conventions shared by every entry point:
 *   - Every array argument is a DEVICE pointer owned by the caller, row-major
 *     and contiguous, batch-major for batched operands.  A: b x m x k,
 *     B: b x k x n, C and p_star: b x m x n.  W and D: n x n.
 *   - mt_options and p_family are HOST memory read during the call only.
 *   - The library never allocates device memory: the caller passes a device
 *     workspace of at least the size returned by the matching *_workspace_size
 *     call (256-byte aligned).  Its contents on entry do not matter.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = null stream).
 *     Outputs are valid once the stream has reached the end of the call.
 *   - Argument errors are detected before anything is enqueued and returned
 *     synchronously (MT_ERR_INVALID_ARG, MT_ERR_WORKSPACE, MT_ERR_UNSUPPORTED);
 *     nothing is written.  The message is available from maxtimes_last_error().
 *   - Domain errors (negative, NaN or +inf entries of A/B; negative or NaN
 *     weights of W) are detected on the device.  They are reported as
 *     MT_ERR_DOMAIN only when MT_FLAG_VALIDATE is set, which makes the call
 *     wait for the device; otherwise outputs for such inputs are unspecified.
 *   - Launch failures return MT_ERR_DEVICE.
 *   - Calls on different streams may run concurrently only with distinct
 *     workspaces and outputs.
 */
#ifndef MAXTIMES_H
#define MAXTIMES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MT_OK = 0,
    MT_ERR_INVALID_ARG = 1,
    MT_ERR_DOMAIN = 2,
    MT_ERR_WORKSPACE = 3,
    MT_ERR_DEVICE = 4,
    MT_ERR_UNSUPPORTED = 5
} mt_status;

/* Element type of A, B, C, G, dA, dB (and of D for apsp_estimate). */
typedef enum { MT_F32 = 0, MT_F64 = 1 } mt_dtype;

typedef enum { MT_PATH_FP64 = 0, MT_PATH_BF16_SPLIT = 1 } mt_path;

/* Flags (mt_options.flags). */
#define MT_FLAG_VALIDATE     1u  /* check the input domain on the device and wait for it */
#define MT_FLAG_NORM_CORRECT 2u  /* divide C by k^(1/p*): centred error (Sec. 1) */
#define MT_FLAG_CLAMP        4u  /* clamp C to <= 1 (always on inside apsp_estimate) */
#define MT_FLAG_RAW_OUTPUT   8u  /* apsp_estimate: write X (the (x,max) matrix) instead of D */
/*
 * MT_FLAG_PROJECT_R1: estimate the max by the r = 1 projection of the norm
 * sequence (Sec. 1: the terms u_k are modelled as h copies of one value
 * alpha, so S_p = h alpha^p).  With p* selected as above and p_lo the next
 * smaller p of the family, C = r c (S_{p*} / S_{p_lo})^(1/(p* - p_lo)); for a
 * powers-of-two family p_lo = p* / 2 and this is the paper's r = 1 form.  It is
 * exact when the largest terms tie (so the APSP squarings lose the bias of
 * the tied k = i and k = j terms) and satisfies
 * E (2 (sqrt(k) - 1) / (k - 1))^(2 / p*) <= C <= E when p_lo = p* / 2.  The plain
 * root is kept where p* is the smallest p, no p is stable, or S_{p_lo} = 0.
 * maxtimes_estimate and apsp_estimate; not with MT_FLAG_NORM_CORRECT
 * (MT_ERR_INVALID_ARG); maxtimes_estimate_backward rejects it
 * (MT_ERR_UNSUPPORTED).  A tile runs one more p of the family than the
 * plain estimate needs, and the FP64 path uses 8 more workspace bytes per
 * output entry.
 */
#define MT_FLAG_PROJECT_R1  16u
/*
 * MT_FLAG_PROJECT_R2: estimate the max by the r = 2 projection (Sec. 1: the
 * terms modelled as two values, from the 2r = 4 evenly spaced norms q, 2q,
 * 3q, 4q).  p* is selected from the family as above; with p* = 4q, q and 2q
 * in the family, the library adds the norm 3q (every such 3p/4 not in the
 * family, so the family plus these may hold at most MT_MAX_P powers) and
 * takes C = r c alpha, alpha^q the largest root of g0 + g1 x + g2 x^2, g the
 * null vector of the Hankel matrix [[S_q, S_2q, S_3q], [S_2q, S_3q, S_4q]].
 * It is exact when the terms take at most two distinct values.  Where the
 * four norms are not all available and positive, the matrix has rank 1 (one
 * distinct value; numerically: |g| <= 1e-8 of the squared norm of the
 * matrix, after the norms are rescaled to S_kq / c^k with
 * c = (S_4q / S_q)^(1/3)), or the roots are complex or not positive, the r = 1
 * projection (MT_FLAG_PROJECT_R1) is used.  FP64 path only
 * (MT_ERR_UNSUPPORTED on BF16): every power's ring result is kept (no
 * early exit, 8 bytes per output entry per power of workspace) and a
 * separate pass selects and projects.  Not with MT_FLAG_NORM_CORRECT or
 * MT_FLAG_PROJECT_R1 (MT_ERR_INVALID_ARG); maxtimes_estimate_backward
 * rejects it (MT_ERR_UNSUPPORTED).
 */
#define MT_FLAG_PROJECT_R2  32u
/*
 * MT_FLAG_XY_PAIRED (xy_topk_estimate only; any other entry point answers
 * MT_ERR_INVALID_ARG): the paired NormQueue that the Discussion proposes.
 * The run on y and the run on y reversed pop in lockstep; their diagonals
 * m1 = i + j and m2 = i + n - 1 - j give the pair (i, j) of the rank before
 * the norms are updated.  The pair is accurate when it lies in the grid and
 * its scaled value v = e^(x_i - max x + y_j - max y) is at least
 * psi len^(-1/p*) on both diagonals (psi the diagonal's estimate, p* its
 * root, len its number of grid pairs: the smallest largest term that its
 * norm admits; no pair is accurate on a diagonal without a stable p).  An
 * accurate rank reports the exact x_i + y_j and (i, j) and
 * subtracts v^p from both runs' norms; any other rank reports run 0's
 * estimate with i = j = -1, and each run subtracts its own estimate (the
 * plain queue's update).  Needs k <= 4096 (MT_ERR_UNSUPPORTED above).
 */
#define MT_FLAG_XY_PAIRED   64u
/*
 * Inner-index balancing (maxtimes_estimate only).  The Discussion (Sec. 4)
 * remarks that a problem can be scaled into a bounded range.  Every term
 * A_ik B_kj, hence the product and each p-norm of the terms, is unchanged
 * when column k of A is multiplied by d_k > 0 and row k of B divided by it;
 * what changes are the scales r_i, c_j of the scaled call H' (Sec. 2.1) and
 * with them which p are stable.  With this flag the estimate is that of
 * (A D, D^-1 B), d_k = sqrt(b_k / a_k), a_k = max_i A_ik, b_k = max_j B_kj
 * (d_k = 1 where either is 0): column k of A D and row k of D^-1 B then have
 * the same largest entry, and the estimate no longer depends on how the
 * inner index of the inputs is scaled.  Where the inputs carry such a
 * scaling, r_i c_j tightens and p* rises.  p_star refers to the balanced
 * estimate; the backward accepts the flag and differentiates the estimate
 * at the given p* (balancing does not change the p-norm of the terms).
 * Costs two more reductions over A and B; workspace grows by 32 b k bytes.
 */
#define MT_FLAG_BALANCE    128u

#define MT_PSTAR_NONE 255  /* p_star value when no p of the family was stable */
#define MT_MAX_P 32        /* largest family size */
#define MT_MAX_POWER 4096  /* largest p accepted */

/* Default stability thresholds (used when tau <= 0).  A ring product of
 * nonnegative terms has no cancellation, so tau only has to rule out
 * underflow: 1e-290 in FP64, 1e-30 for the BF16/FP32 exponent range. */
#define MT_TAU_FP64_DEFAULT 1e-290
#define MT_TAU_BF16_DEFAULT 1e-30
/* FFT convolution does cancel: Sec. 2.1 puts its threshold at 1e-12. */
#define MT_TAU_FFT_DEFAULT 1e-12

typedef struct {
    const int32_t* p_family; /* host; n_p entries, strictly ascending, 1..MT_MAX_POWER */
    int32_t n_p;             /* 1..MT_MAX_P; n_p = 1 selects that p everywhere */
    int32_t path;            /* mt_path */
    double tau;              /* stability threshold; <= 0 -> the path default */
    int32_t split_max_p;     /* BF16 path: split p <= split_max_p; < 0 -> 4 */
    uint32_t flags;          /* MT_FLAG_* */
} mt_options;

/* Workspace bytes needed by maxtimes_estimate for these sizes and options. */
mt_status maxtimes_workspace_size(int64_t b, int64_t m, int64_t k, int64_t n,
                                  const mt_options* opt, size_t* bytes);

/*
 * Where maxtimes_estimate keeps its first results in the workspace (for
 * inspection after a call with the same sizes and options; byte offsets from
 * the workspace start):
 *   r_offset         b x m FP64: r_i = max_k A_ik (Sec. 2.1 scaling)
 *   c_offset         b x n FP64: c_j = max_k B_kj
 *   a_planes_offset  [b][n_planes][m_pad][k_pad]: (A / r)^p, row-major
 *   b_planes_offset  [b][n_planes][n_pad][k_pad]: (B / c)^p, transposed
 * Plane elements are BF16 bit patterns (elem_bytes = 2, BF16 path: hi, and
 * for a split p the next plane holds lo = RNE(x - hi)) or FP64 (8).  Power q
 * of the plane spec (the family, plus the added norms of
 * MT_FLAG_PROJECT_R2, ascending) is power[q], in plane first_plane[q].
 * Padding (rows >= m or n, columns >= k) holds zeros.  Host memory; same
 * argument checks as maxtimes_workspace_size.
 */
typedef struct {
    size_t r_offset, c_offset, a_planes_offset, b_planes_offset;
    int64_t m_pad, n_pad, k_pad;
    int32_t n_planes, elem_bytes, n_powers;
    int32_t power[MT_MAX_P];
    int32_t first_plane[MT_MAX_P];
    int32_t split[MT_MAX_P];
} mt_workspace_map;
mt_status maxtimes_workspace_map(int64_t b, int64_t m, int64_t k, int64_t n, const mt_options* opt,
                                 mt_workspace_map* map);

/*
 * The estimate C of the (max, x) product of A and B (Alg. 5, Sec. 2.1-2.2).
 *   A      b x m x k, dtype, entries >= 0 and finite.
 *   B      b x k x n, dtype, entries >= 0 and finite.
 *   C      b x m x n, dtype (output).
 *   p_star b x m x n uint8 (output, nullable): index into p_family of the p
 *          used per entry, MT_PSTAR_NONE if none was stable.
 * b, m, k, n >= 0: an empty C is a no-op; k = 0 gives C = 0 and p_star =
 * MT_PSTAR_NONE.  Sizes above 2^24 return MT_ERR_UNSUPPORTED, and so does
 * k above 2^23 on the BF16 path (m or n above 2^23 for its backward, n for
 * its APSP).
 * FP32 inputs are converted exactly on load for the FP64 path.
 * Range: r_i c_j may lie outside the output type (it is applied as a
 * mantissa product and one power-of-two scaling in the output precision),
 * so an entry of C overflows or underflows only where its value
 * r_i c_j S^(1/p*) itself lies outside the output type.
 */
mt_status maxtimes_estimate(const void* A, const void* B, mt_dtype dtype,
                            int64_t b, int64_t m, int64_t k, int64_t n,
                            const mt_options* opt, void* C, uint8_t* p_star,
                            void* workspace, size_t ws_bytes, void* stream);

/*
 * maxtimes_estimate without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  Same arguments, results and errors as
 * maxtimes_estimate; the workspace is a static device array of the library
 * of MT_NOALLOC_SCRATCH_BYTES bytes (one per GPU, on the device current at
 * the call, which must hold A, B, C and p_star; each GPU keeps it until the
 * process ends).  The call allocates nothing.  A product whose workspace
 * (maxtimes_workspace_size) exceeds the scratch returns MT_ERR_WORKSPACE
 * before anything is enqueued.  Every call on one GPU shares that GPU's
 * scratch: calls whose stream work overlaps on one GPU (two streams, or two
 * threads) race on it and give undefined results; calls in order on one
 * stream are safe.  The call clears with kernels what its kernels need at
 * zero; the scratch otherwise keeps the last call's contents.
 */
#define MT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
mt_status maxtimes_estimate_noalloc(const void* A, const void* B, mt_dtype dtype,
                                    int64_t b, int64_t m, int64_t k, int64_t n,
                                    const mt_options* opt, void* C, uint8_t* p_star,
                                    void* stream);

/* Workspace bytes needed by maxtimes_estimate_backward. */
mt_status maxtimes_backward_workspace_size(int64_t b, int64_t m, int64_t k, int64_t n,
                                           const mt_options* opt, size_t* bytes);

/*
 * Gradient of L = sum(G .* C) with respect to A and B for the estimate with
 * p* held fixed per entry (the paper notes the p-norm rings are continuous
 * and differentiable, Sec. 4).  With C' = C / (r_i c_j):
 *   dL/dA = sum_p A'^(p-1) .* ((Gt_p) (B'^p)^T),   Gt_p = [p* = p] G c_j C'^(1-p)
 *   dL/dB = sum_p B'^(p-1) .* ((A'^p)^T (Gt'_p)),  Gt'_p = [p* = p] G r_i C'^(1-p)
 *   A, B, C, p_star  the inputs and outputs of the forward call (same options).
 *   G                b x m x n, dtype.
 *   dA, dB           b x m x k and b x k x n, dtype (outputs, each nullable).
 * Entries whose C is 0 contribute nothing.  MT_FLAG_NORM_CORRECT is not
 * supported here (MT_ERR_UNSUPPORTED).  The BF16 path splits every power
 * and every Gt into hi + lo, because G has mixed signs.
 * Range on the BF16 path: Gt is formed in FP32 with r and c carried over a
 * per-item power of two (the exponent of the item's largest r, resp. c),
 * so G C'^(1-p) must lie in FP32 (it does for every stable entry, where
 * C'^p* >= tau, up to the range of G itself), and an r_i (c_j) more than
 * about 2^126 below the item's largest contributes 0 to dB (dA).  The FP64
 * path has the FP64 range.  With MT_FLAG_BALANCE (set as in the forward
 * call) the backward runs on the balanced pair (A D, D^-1 B) and returns
 * dA = D dA', dB = D^-1 dB': the derivative of the same estimate.
 */
mt_status maxtimes_estimate_backward(const void* A, const void* B, const void* G,
                                     const void* C, const uint8_t* p_star, mt_dtype dtype,
                                     int64_t b, int64_t m, int64_t k, int64_t n,
                                     const mt_options* opt, void* dA, void* dB,
                                     void* workspace, size_t ws_bytes, void* stream);

/* Workspace bytes needed by apsp_estimate. */
mt_status apsp_workspace_size(int64_t n, const mt_options* opt, size_t* bytes);

/*
 * Estimated all-pairs shortest distances of a directed graph (Sec. 2.2).
 *   W            n x n FP32 weights, >= 0, +inf = no edge; the diagonal is
 *                ignored (a vertex reaches itself at distance 0).
 *   s            > 0, the transform exp(-s w); s = 1 is the paper's.
 *   n_squarings  T; < 0 -> ceil(log2 n); 0 returns the transformed W
 *                itself (direct edges only).
 *   D            n x n of d_dtype (output): distances (+inf = unreachable),
 *                or with MT_FLAG_RAW_OUTPUT the (x, max) matrix X.
 *   p_star_last  n x n uint8 (nullable): p* index of the last squaring.
 * MT_FLAG_CLAMP is implied.
 */
mt_status apsp_estimate(const float* W, int64_t n, double s, int32_t n_squarings,
                        const mt_options* opt, void* D, mt_dtype d_dtype,
                        uint8_t* p_star_last, void* workspace, size_t ws_bytes,
                        void* stream);

/*
 * The exact (max, x) product E_ij = max_k A_ik B_kj (Alg. 2, Sec. 2.2), E
 * starting at 0, on the vector ALUs: products in the input precision (one
 * rounding), exact max.  A b x m x k, B b x k x n, E b x m x n, all of dtype,
 * device memory; no workspace.  For measuring the estimate's error and as
 * the exact-product throughput beside it.
 */
mt_status maxtimes_exact(const void* A, const void* B, mt_dtype dtype, int64_t b, int64_t m,
                         int64_t k, int64_t n, void* E, void* stream);

/*
 * Exact distances from a few sources: the exact pairs on which the affine
 * correction below is fitted (Sec. 4 suggests Dijkstra's algorithm for a
 * small number of vertex pairs; on the dense weight matrix the GPU runs
 * Bellman-Ford instead).
 *   W        n x n FP32 device, row-major; W[u][v] >= 0 the weight of edge
 *            u -> v, +inf for no edge (the diagonal is ignored).
 *   sources  n_src int32 device, each in 0 .. n - 1.
 *   D        n_src x n FP64 device (output): D[q][v] = the smallest sum of
 *            weights over paths from sources[q] to v (0 at the source, +inf
 *            where v is unreachable).
 *   rounds   host, nullable (output): relaxation rounds run.
 * Rounds D <- min(D, D (min,+) W) in FP64 from the one-edge distances,
 * until a round changes nothing (at most n - 1).  Synchronous: the call
 * waits on the stream every 8 rounds for the convergence flag.  Workspace
 * from apsp_exact_rows_workspace_size (8 n_src n bytes + 256).  A source
 * outside 0 .. n - 1 returns MT_ERR_INVALID_ARG.
 */
mt_status apsp_exact_rows_workspace_size(int64_t n, int32_t n_src, size_t* bytes);
mt_status apsp_exact_rows(const float* W, int64_t n, const int32_t* sources, int32_t n_src, double* D,
                          int64_t* rounds, void* workspace, size_t ws_bytes, void* stream);

/*
 * Affine correction of an APSP estimate (Sec. 4: an affine model between a
 * few exact distances and the estimated ones corrects the numerical error,
 * reducing bias and MSE).  Least squares d_exact = a d_est + b over the pairs
 * (sources[q], v), v != sources[q], with both distances finite; without such
 * pairs a = 1, b = 0, and a = 1 when every estimated distance is equal.
 *   D        n x n estimated distances, dtype (FP32 / FP64), device.
 *   sources, exact  n_src sources and their n_src x n exact FP64 distances
 *            (as apsp_exact_rows returns them); sources outside 0 .. n - 1
 *            contribute no pairs.
 *   ab       2 doubles device (output): a, b.
 *   apply    nonzero: D <- max(0, a D + b) in place on every finite
 *            off-diagonal entry (+inf and the zero diagonal stay).
 * Asynchronous on the stream; deterministic (fixed-order reductions in
 * FP64, two passes: means, then centred sums).  Workspace from
 * apsp_affine_workspace_size.
 */
mt_status apsp_affine_workspace_size(size_t* bytes);
mt_status apsp_affine_correct(void* D, mt_dtype dtype, int64_t n, const int32_t* sources, int32_t n_src,
                              const double* exact, double* ab, int32_t apply, void* workspace, size_t ws_bytes,
                              void* stream);

/*
 * Max-convolution estimate (Sec. 1; ring kernel H = FFT convolution and its
 * threshold, Sec. 2.1), batched:
 *     z[t] = max_i x[i] y[t - i],  t = 0 .. n + m - 2  (i over 0 .. n - 1 with
 *                                                       0 <= t - i < m)
 *   rx = max x, ry = max y, x' = x / rx, y' = y / ry,
 *   S_p = x'^p * y'^p                  (ordinary convolution, by FFT in FP64)
 *   p*[t] = max{ p in P : S_p[t] >= tau },   z[t] = rx ry S_{p*}[t]^(1/p*).
 * The estimate satisfies E <= z <= K^(1/p*) E up to the FFT's rounding
 * (E the exact max-convolution, K the number of terms at t).  No stable p:
 * the smallest p of the family with S clamped to >= 0, p* = MT_PSTAR_NONE.
 *   x        b x n, y  b x m, dtype (FP32 / FP64), device, nonnegative and
 *            finite (other values give unspecified results).
 *   opt      family as for maxtimes_estimate; path must be MT_PATH_FP64
 *            (else MT_ERR_UNSUPPORTED); tau <= 0 -> MT_TAU_FFT_DEFAULT;
 *            split_max_p is ignored; flags must be 0 (else
 *            MT_ERR_UNSUPPORTED).
 *   z        b x (n + m - 1), dtype, device (output).
 *   p_star   b x (n + m - 1) uint8 device (output, nullable): index of p*
 *            in the family.
 * n + m - 1 <= 4096: one workgroup per pair transforms in LDS, largest p
 * first, and stops once every index of its pair is decided; no workspace
 * (workspace may be NULL).  4096 < n + m - 1 <= 16384: the pairs go through
 * global buffers in the workspace, one p at a time for the whole batch (no
 * early exit).  Larger lengths and b >= 2^31 return MT_ERR_UNSUPPORTED.
 * n = 0, m = 0 or b = 0: empty output, nothing written.  Asynchronous on the
 * stream.  Workspace from maxconv_workspace_size (0 bytes up to 4096; about
 * 32 N + 9 (n + m - 1) bytes per pair above, N the transform length).
 */
mt_status maxconv_workspace_size(int64_t b, int64_t n, int64_t m, const mt_options* opt, size_t* bytes);
mt_status maxconv_estimate(const void* x, const void* y, mt_dtype dtype, int64_t b, int64_t n, int64_t m,
                           const mt_options* opt, void* z, uint8_t* p_star, void* workspace, size_t ws_bytes,
                           void* stream);

/*
 * The exact max-convolution z[t] = max_i x[i] y[t - i] (the definition of
 * Sec. 1, z starting at 0), one GPU thread per output, products rounded once
 * in dtype.  x b x n, y b x m, z b x (n + m - 1), device; b (n + m - 1) <= 2^38,
 * n, m <= 2^24 (else MT_ERR_UNSUPPORTED).  For measuring the estimate's error.
 */
mt_status maxconv_exact(const void* x, const void* y, mt_dtype dtype, int64_t b, int64_t n, int64_t m,
                        void* z, void* stream);

/*
 * Top k of x_i + y_j with their indices (Sec. 2.3: algorithm E, the
 * NormQueue, and the index recovery from a second run on y reversed).
 *   x' = e^(x - max x), y' = e^(y - max y)           (the (x, max) image, scaled)
 *   sigma^(p)[m] = (x'^p * y'^p)[m], m = 0 .. 2n - 2 (FFT convolution in FP64)
 *   psi[m] = sigma^(p*)[m]^(1/p*), p* the largest p with sigma^(p)[m] >= tau
 *            (0 if none: such diagonals come last)
 *   k times: m* = the diagonal with the largest psi (the lowest m on ties);
 *            report max x + max y + log(psi[m*]) and m*; subtract psi[m*]^p
 *            from sigma^(p)[m*] for every p; estimate psi[m*] again.
 *   The same on y reversed gives, rank by rank, m2 = i + (n - 1 - j); with
 *   m1 = i + j the indices are i = (m1 + m2 - n + 1) / 2, j = m1 - i (-1 when
 *   that is not an integer pair in the grid).  The values are estimates and
 *   the pops can come out of order; errors accumulate with the rank (Sec. 3).
 *   x, y     n values each, dtype (FP32 / FP64), device, finite.
 *   opt      family as for maxtimes_estimate (Sec. 3 uses 24 powers up to
 *            4096); path MT_PATH_FP64 (else MT_ERR_UNSUPPORTED); tau <= 0 ->
 *            MT_TAU_FFT_DEFAULT; flags 0 or MT_FLAG_XY_PAIRED (the paired
 *            queue of the Discussion, k <= 4096; other flags:
 *            MT_ERR_UNSUPPORTED).
 *   values   k FP64 device (output), in pop order.
 *   diag, i_idx, j_idx  k int32 device (outputs, each nullable): m1, i, j.
 * 1 <= n <= 8192 (2n - 1 <= 16384; up to n = 2048 each transform runs in
 * one workgroup's LDS, longer ones through global buffers in the workspace),
 * 0 <= k <= 2^24 (else MT_ERR_UNSUPPORTED / MT_ERR_INVALID_ARG).
 * The pops run in sequence on one wave.  For k <= 4096 it pops both runs
 * together over the K = min(k, 2n - 1) diagonals of each run with the
 * largest initial estimates (lowest m on ties: the only ones k pops can
 * reach), their sigma columns in LDS when 40 K + 16 |P| K + 4 k bytes fit in
 * 160 KiB; for larger k one wave per run scans every diagonal.  Workspace
 * from xy_topk_workspace_size (16 (|P| + 1)(2n - 1) + 16 k bytes and
 * alignment, plus 64 |P| N + 2 N bytes for the global buffers when n > 2048,
 * N the transform length, plus (24 + 16 |P|) K bytes for the candidates when
 * k <= 4096).  With
 * k = 0 only the ring results are formed: the workspace then starts with
 * sigma^(p)[m] of both runs, FP64, indexed (run |P| + q)(2n - 1) + m (run 1
 * on y reversed), for inspection.  Asynchronous on the stream.
 */
mt_status xy_topk_workspace_size(int64_t n, int32_t k, const mt_options* opt, size_t* bytes);
mt_status xy_topk_estimate(const void* x, const void* y, mt_dtype dtype, int64_t n, int32_t k,
                           const mt_options* opt, double* values, int32_t* diag, int32_t* i_idx,
                           int32_t* j_idx, void* workspace, size_t ws_bytes, void* stream);

/* Static description of a status code. */
const char* maxtimes_status_string(mt_status status);

/* Message of the last error returned on the calling thread ("" if none). */
const char* maxtimes_last_error(void);

/*
 * Per-kernel timing with HIP events recorded around every launch on the
 * launch stream (off by default).  maxtimes_timing_read waits for the
 * recorded events and returns the summed milliseconds and launch count of
 * every kernel whose name starts with `prefix` since the last reset.
 */
mt_status maxtimes_timing_enable(int on);
mt_status maxtimes_timing_reset(void);
mt_status maxtimes_timing_read(const char* prefix, double* total_ms, int64_t* launches);

/*
 * Work executed by the timed launches whose kernel name starts with `prefix`
 * since the last reset (kernels that count no work add nothing).  The p-family
 * GEMMs count MFMA flops: the forward GEMMs stop a tile as soon as every entry
 * of it has found its p* (smaller p cannot change the result), so this is at
 * most, and often less than, 2 * rows_pad * cols_pad * k_pad per segment of
 * the family.  The max-convolution counts 10 N log2 N flops (two complex FFTs
 * of N points, 5 N log2 N each by the usual count) per pair and p visited.
 * The counters are a static device array of the library (2048 launches per
 * reset, on the device current at the first timed launch that counts work;
 * nothing is allocated); reset waits for the recorded launches and clears
 * them.
 */
mt_status maxtimes_timing_work(const char* prefix, double* flops);

/*
 * Device-side duration of the timed launches whose kernel name starts with
 * `prefix`, for the kernels that count work (the p-family GEMMs and the
 * max-convolution): each workgroup reads the device's constant-rate
 * real-time counter when it starts and, after a barrier, when it ends; the
 * launch's span is the latest end minus the earliest start, converted with
 * the device's reported clock rate.  Returns the summed milliseconds and the
 * number of launches.  Unlike the events of maxtimes_timing_read, the span
 * excludes the command processor's time before the first workgroup starts
 * and after the last one ends, and cannot include work queued before the
 * launch; MT_ERR_UNSUPPORTED if the device reports no clock rate.
 */
mt_status maxtimes_timing_span(const char* prefix, double* total_ms, int64_t* launches);

/*
 * Sparse tail.  The forward GEMMs visit the family from the largest p down
 * and stop a tile once every entry has its p* (Sec. 1: p* is the largest
 * stable p, so a smaller p cannot change a decided entry).  When at most
 * `max_entries` entries of a tile are still undecided, the tile hands them
 * to a second kernel that runs the remaining p for each of them alone (one
 * dot product of a plane row of A'^p and of B'^p per p, FP32 accumulation on
 * the BF16 path, FP64 on the FP64 path) and stops.  Results equal the dense
 * path's up to the order of the FP32 / FP64 summation; on the BF16 path an
 * entry that goes up from p to 2p (both without the hi/lo split) takes S_2p
 * from the same dot product, each term squared, so its 2p terms are rounded
 * as squares of BF16 p-th powers instead of BF16 2p-th powers.  0 disables it; the
 * default is 512.  The workspace sizes grow by 32 bytes x max_entries per
 * output tile (the list and its copy sorted by row), so query them after
 * changing the threshold (a workspace sized before is reported too small).  Process-wide; not synchronised with calls
 * in flight on other threads.
 */
mt_status maxtimes_set_tail_threshold(int32_t max_entries);
int32_t maxtimes_tail_threshold(void);

/*
 * Where the forward p search starts (Sec. 1 defines p* as the largest stable
 * p; the search order only decides how much work finds it).  entry = 0
 * visits the family from the largest p down.  entry = s > 0 starts at the
 * s-th largest p (clamped to the smallest): going down from there decides
 * every entry that is not stable at the start; an entry stable at the start
 * waits unless its S rules out every larger p (S_p' <= S_p^(p'/p) for terms
 * in [0, 1]), and after the smallest p the search goes up from the (s-1)-th
 * largest p until each waiting entry meets an unstable p or such an S.
 * entry = -1, the default, lets a pilot choose per product: it forms S_p for
 * every p on a 64 x 64 grid of sampled output entries and takes the start
 * with the lowest estimated dense GEMM and sparse-tail work (products with
 * fewer than 2^22 outputs, or with the tail off, start at the largest p).
 * Results equal those of the top-down search up to entries whose S lies
 * within rounding of tau.  The r = 1 projection always searches from the
 * largest p.  Returns MT_ERR_INVALID_ARG outside -1 .. MT_MAX_P - 1.
 * Process-wide; not synchronised with calls in flight on other threads.
 */
mt_status maxtimes_set_search_start(int32_t entry);
int32_t maxtimes_search_start(void);

/*
 * Deferred planes (plain products whose search start the pilot chooses,
 * families of at least five p).  p* is the largest stable p (Sec. 1), so an
 * entry needs the planes of a smaller p only if it is unstable at every
 * larger one.  With on = 1, the default, the power planes of the two
 * smallest p (BF16 path), or of all but the three largest p (FP64 path, whose
 * tiny tau puts p* near the largest p), are not written with the others.
 * They are written before the GEMM when the pilot's sampled entries include
 * one that is unstable at every p whose planes were written; otherwise a
 * GEMM tile or a sparse-tail entry that reaches them marks its tile, and
 * after the GEMM those planes are written for the rows of A and the columns
 * of B of the marked tiles, and the marked tiles run their whole search
 * again, densely, without the sparse tail (three extra launches per
 * product, which return at once when nothing is marked).  The workspace's
 * deferred planes then hold data only where a tile needed them.
 * Results: the same selection rule on the same planes; a tile that ran
 * again sums its entries on the MFMA instead of the tail kernel, which
 * changes the order of the sums.  The workspace holds 4 bytes per output
 * tile for the marks either way.  on = 0 writes every plane up front.
 * MT_ERR_INVALID_ARG for other values.  Process-wide; not synchronised with
 * calls in flight on other threads.
 */
mt_status maxtimes_set_deferred_planes(int32_t on);
int32_t maxtimes_deferred_planes(void);

/*
 * Small products (Alg. 5 with the scaled call H' of Sec. 2.1, FP64 path):
 * maxtimes_estimate (and its _noalloc form) computes a product with
 * b * m * k * n <= max_work multiply-adds, options at most MT_FLAG_CLAMP and
 * MT_FLAG_NORM_CORRECT, b <= 65535 and m <= 2^21 in one kernel: each
 * workgroup takes the maxima of its 32 rows of A and 32 columns of B, then
 * forms S_p = A'^p B'^p for its 32 x 32 outputs in FP64 from the largest p
 * down and stops once each output has its p (the general path's seven to
 * fourteen launches cost more than such a product's arithmetic).  Same
 * results as the general path up to the order of the FP64 sums; the
 * workspace argument is checked as for the general path and not used.
 * max_work = 0 sends every product down the general path; the default is
 * 2^25.  MT_ERR_INVALID_ARG for a negative limit.  Process-wide; not
 * synchronised with calls in flight on other threads.
 */
mt_status maxtimes_set_small_product_limit(int64_t max_work);
int64_t maxtimes_small_product_limit(void);

/* Library version string. */
const char* maxtimes_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MAXTIMES_H */
