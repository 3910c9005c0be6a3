// Internal declarations shared by the HIP translation units of libmaxtimes.
// Not part of the public ABI (include/maxtimes.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "maxtimes.h"

namespace mt {

// ---------------------------------------------------------------- vector types
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

typedef __attribute__((address_space(3))) void lds_void;
typedef __attribute__((address_space(1))) const void glb_cvoid;

// ---------------------------------------------------------------- tiling
// BF16 p-family GEMM: 256 x 256 output tile per workgroup, K step 64.
constexpr int kBf16BM = 256;
constexpr int kBf16BN = 256;
constexpr int kBf16BK = 64;
// FP64 p-family GEMM: BM x BM output tile (BM = 128 or 64), K step 16.
constexpr int kF64BK = 16;
// Adjoint GEMMs: 128 x 128 (BF16) and 64 x 64 (FP64) output tiles.
constexpr int kAdjBM = 128;
constexpr int kAdjF64BM = 64;

// Workspace header: domain flag word, sparse-tail length and p* histogram.
struct WsHeader {
    int32_t domain_flag;
    uint32_t tail_count;
    int32_t start;       // plan index the forward's p search starts at
    int32_t low_missed;  // deferred planes: some tile or tail entry reached them unwritten
    int32_t low_need;    // deferred planes: the pilot saw sampled entries that need them
    int32_t pad[3];
    int32_t hist[MT_MAX_P + 1];
};

// Sparse tail: an output entry a GEMM tile handed over because only a few of
// its entries were still undecided; the tail kernel runs the remaining p of
// the plan for it alone (one dot product per p).
struct TailEntry {
    int32_t bi, i, j;  // batch item, row, column
    int16_t e_next;    // next plan entry to run
    int16_t state;     // kTailOpen, kTailR1 or kTailRise
};
// TailEntry::state
constexpr int16_t kTailOpen = 0;  // no stable p yet: run e_next, e_next + 1, ... (smaller p)
constexpr int16_t kTailR1 = 1;    // r = 1 projection: S at p* parked in the output, finish at e_next
constexpr int16_t kTailRise = 2;  // stable at e_next + 1 (S parked), a larger p may be too:
                                  // run e_next, e_next - 1, ... (larger p)

// Processing plan of the p family for one fused GEMM launch.  Entries are in
// processing order (largest p first); `pidx` maps back to the family index.
// For a split p the three segments are (hi,hi), (hi,lo), (lo,hi).
struct PlanEntry {
    int32_t pidx;       // index into the family (what p_star records)
    int32_t p;          // the power
    int32_t nseg;       // 1 or 3
    int32_t a_plane[3]; // plane index per segment (A side)
    int32_t b_plane[3]; // plane index per segment (B side)
    float inv_p;        // 1 / p
    float corr;         // k^(-1/p) with MT_FLAG_NORM_CORRECT, else 1
    float inv_dp;       // 1 / (p - p_next) for the next (smaller) p of the plan, 0 if none
    // S_q <= S_p^(q/p) for the next larger p = q (terms in [0, 1]): S below
    // rise_thr = (tau / margin)^(p/q) rules every larger p out; +inf for the
    // largest p.  rise_thr_f is its FP32 value rounded down.
    double rise_thr;
    float rise_thr_f;
};

struct FamilyPlan {
    int32_t n;  // entries
    int32_t r1; // the r = 1 projection replaces the plain root (MT_FLAG_PROJECT_R1)
    double tau;
    float tau_f;  // smallest FP32 value >= tau (exact FP32 form of S >= tau)
    PlanEntry e[MT_MAX_P];
};

// Output modes of the fused epilogue.
enum EpiMode : int32_t {
    EPI_PLAIN = 0,      // C = r c S^(1/p)   (optional clamp <= 1)
    EPI_APSP_X = 1,     // X = min(C, 1), X_ii = 1
    EPI_STORE_ALL = 2,  // FP64: S of every plan entry to its plane of a stack (r = 2 projection)
};

struct EpiArgs {
    int32_t mode;
    int32_t clamp;       // EPI_PLAIN only
    void* out;           // C (b x m x n) of out dtype
    void* out2;          // FP64 record epilogue with the r = 1 projection: S at the next smaller p
    int32_t out_f64;     // 1: out is double, 0: float
    uint8_t* pstar;      // nullable
    int32_t* hist;       // nullable: per-family-index counts (+ [MT_MAX_P] = none)
    const double* r;     // b x m (nullable: all ones)
    const double* c;     // b x n (nullable: all ones)
    TailEntry* tail;     // nullable: sparse-tail list (capacity tail_max per tile)
    uint32_t* tail_count;
    int32_t tail_max;    // a tile with 1..tail_max undecided entries hands them over
    const int32_t* start;  // nullable: plan index the p search starts at (0: largest p)
    // The tail kernel runs the list sorted by row bucket (bi * rows + i) >>
    // tail_shift and state, so that entries of one row can share its plane
    // rows: tail_sorted has the list's capacity, tail_bucket one int32 per
    // bucket (tail_buckets of them, two per row bucket, at most kTailBuckets).
    TailEntry* tail_sorted;
    int32_t* tail_bucket;
    int32_t tail_shift;
    int32_t tail_buckets;
    int64_t stack_stride;  // EPI_STORE_ALL: elements per plane of the S stack (b m n)
    // Deferred planes (the forward GEMMs): the planes of plan entries n_eval
    // and beyond are written before the GEMM only when *low_need is set.
    // Without them a tile that needs such an entry, or a tail entry that
    // reaches one, marks its tile in missed_tile and sets *low_missed; the
    // planes of the marked tiles' rows are then written and those tiles run
    // again from the start, densely (the rerun launch).  low_need null:
    // every plane is written.
    const int32_t* low_need;
    int32_t* low_missed;
    uint32_t* missed_tile;  // b x tiles_m x tiles_n: 1 where the tile must run again
    int32_t n_eval;         // plan entries whose planes are always written
};
constexpr int64_t kTailBuckets = 65536;

// Adjoint epilogue: out = sum over the p that some entry uses of
// (M / scale_rows / scale_cols)^(p-1) .* (X_p Y_p^T).
struct AdjArgs {
    const void* M;            // multiplier source, b x rows x cols (A or B)
    int32_t m_f64;            // M is double (else float)
    const double* scale_rows; // b x rows or nullptr
    const double* scale_cols; // b x cols or nullptr
    const int32_t* hist;      // per family index: number of entries using that p
    void* out;                // b x rows x cols (dA or dB)
    int32_t out_f64;
    // nullable, per batch item: the result is multiplied by 2^post_exp (the
    // BF16 adjoint planes hold c_j or r_i divided by that power of two)
    const int32_t* post_exp;
    // nullable, b x rows and b x cols: the result is multiplied by
    // out_row_mul[row] out_col_mul[col] (the chain factors of a balanced
    // forward: d_k for the columns of dA, 1 / d_k for the rows of dB)
    const double* out_row_mul;
    const double* out_col_mul;
};

// ---------------------------------------------------------------- launchers
// Every launcher returns hipSuccess or the launch error.
hipError_t launch_fill_zero_u32(void* p, int64_t words, hipStream_t st);
hipError_t launch_fill_u32(void* p, uint32_t value, int64_t words, hipStream_t st);

// Pilot of the search start: S_p of every plan entry on a grid of nr x nc
// sampled output entries (nr, nc <= kMaxPilotSide) of the planes, then the
// start with the lowest estimated cost (dense tile entries + kappa per tail
// dot product) into *start.
constexpr int kMaxPilotSide = 64;
constexpr int kMaxPilotKParts = 16;
struct PilotArgs {
    const void* X;  // planes as the GEMM reads them (BF16 or FP64)
    const void* Y;
    int64_t x_plane_elems, y_plane_elems, x_batch_elems, y_batch_elems, kp;
    int64_t rows, cols, b;
    int32_t nr, nc, kparts;
    int32_t tail_max;      // per-tile tail capacity of the launch
    int64_t tile_entries;  // output entries of one GEMM tile
    float kappa;           // one tail dot product in dense tile-entry units
    void* part;            // kparts x n x kMaxPilotSide^2 partial sums (float or double)
    void* counts;          // PilotCounts
    // plan entries whose planes exist (n: all); the sampled entries with no
    // stable p among them set *low_need (nullable; *low_missed is cleared
    // with it) and count as undecided to the last entry
    int32_t n_eval;
    int32_t* low_need;
    int32_t* low_missed;
};
// Counts over the sampled entries: es_hist[e] of e* = e (the first stable
// plan entry, the last if none); stop[s][u]: waiting at start s and decided
// at plan entry u < s on the way up.
struct PilotCounts {
    int32_t es_hist[MT_MAX_P];
    int32_t stop[MT_MAX_P][MT_MAX_P];
};
hipError_t launch_choose_start(const PilotArgs& pa, const FamilyPlan& plan, int32_t* start, int f64,
                               hipStream_t st);

// Exact rows of the APSP distance matrix from a few sources (Bellman-Ford in
// FP64; the host checks convergence every kExactRowsChunk rounds, so the
// launch synchronises the stream) and the affine correction fitted on them.
constexpr int kExactRowsChunk = 8;
size_t exact_rows_workspace(int64_t n, int32_t nsrc);
hipError_t launch_exact_rows(const float* W, int64_t n, const int32_t* src, int32_t nsrc, double* D, uint8_t* ws,
                             hipStream_t st, int64_t* rounds_out, int32_t* bad_out);
size_t affine_workspace();
hipError_t launch_affine_correct(void* D, int f64, int64_t n, const int32_t* src, int32_t nsrc, const double* ex,
                                 double* ab, uint8_t* ws, int apply, hipStream_t st);
// Counting sort of the sparse-tail list (length *count, read on the device)
// into epi.tail_sorted by row bucket; rows = rows of the output per batch item.
hipError_t launch_tail_sort(const EpiArgs& epi, int64_t rows, int64_t cap, hipStream_t st);
// Row maxima of A (rows x k; with mul, of A_rj mul[r / rows_per_batch][j])
// and column maxima of B (b x k x n; with mul, of B_bkj mul[b][k]).
hipError_t launch_rowmax(const void* A, int f64, int64_t rows, int64_t k, double* r,
                         int32_t* flag, hipStream_t st, const double* mul = nullptr,
                         int64_t rows_per_batch = 1);
hipError_t launch_colmax(const void* B, int f64, int64_t b, int64_t k, int64_t n, double* c,
                         int32_t* flag, hipStream_t st, const double* mul = nullptr);
// Inner-index balancing factors d = sqrt(b / a) (1 where a or b is 0) and 1 / d.
hipError_t launch_balance(const double* a, const double* b, int64_t count, double* d, double* dinv,
                          hipStream_t st);
hipError_t launch_apsp_transform(const float* W, int64_t n, double s, void* X, int x_f64,
                                 int32_t* flag, hipStream_t st);
hipError_t launch_apsp_to_dist(const void* X, int x_f64, int64_t n, double s, void* D,
                               int d_f64, int raw, hipStream_t st);

// Power planes.  src is b x rows x cols (row-major, element f64 ? double :
// float) when !transpose, or b x cols x rows when transpose (then planes hold
// the transpose).  Output planes: [b][plane][rows_pad][cols_pad] of bf16
// (bf16 != 0) or double.  Plane element (t, u) is src col_mul[u] /
// (scale_rows[t] * scale_cols[u]); scale_rows is b x rows, scale_cols and
// col_mul b x cols, each nullable.
// powers: ascending list; split[q] says whether power q gets a hi/lo pair
// (bf16 only).
struct PlaneSpec {
    int32_t n_p;
    int32_t p[MT_MAX_P];
    int32_t split[MT_MAX_P];
    int32_t first_plane[MT_MAX_P];  // plane index of power q (hi plane if split)
    int32_t n_planes;
    uint32_t write_mask;            // bit q: the planes of power q are written
};
// Row maxima r of a row-major FP32 operand A (b x rows x cols) and its power
// planes in one pass, the same values as launch_rowmax followed by
// launch_power_planes (untransposed, no column scales or multipliers), for
// cols_pad <= kFusedRowMaxK; with the column maxima c of B (FP32,
// b x cols x nb) taken in the same launch (c is cleared first), so the two
// passes share the GPU.  Needs at least as many plane rows (b rows_pad) as
// column-max blocks.
constexpr int64_t kFusedRowMaxK = 8192;
hipError_t launch_rowmax_planes_colmax(const float* A, const float* B, int64_t b, int64_t rows, int64_t cols,
                                       int64_t rows_pad, int64_t cols_pad, int64_t nb, double* r, double* c,
                                       int32_t* flag, const PlaneSpec& spec, int bf16, void* planes,
                                       hipStream_t st);
hipError_t launch_power_planes(const void* src, int src_f64, int transpose, int64_t b,
                               int64_t rows, int64_t cols, int64_t rows_pad, int64_t cols_pad,
                               const double* scale_rows, const double* scale_cols,
                               const PlaneSpec& spec, int bf16, void* planes, hipStream_t st,
                               const double* col_mul = nullptr);
// The planes of spec.write_mask for both operands in one launch (A untransposed
// as launch_power_planes with transpose 0, B transposed as with transpose 1;
// BF16 or FP64 planes), only when *cond is nonzero on the device (else every
// workgroup returns at once): the deferred planes, written once some entry
// needs them.  With marks (one word per output tile of side tile_bm, a
// multiple of 64 dividing mp and np), only the plane rows of the tile rows
// (A) and tile columns (B) that hold a marked tile.
hipError_t launch_planes_if(const int32_t* cond, const void* A, const void* B, int src_f64, int bf16, int64_t b,
                            int64_t m, int64_t n, int64_t k, int64_t mp, int64_t np, int64_t kp, const double* r,
                            const double* c, const double* a_mul, const double* b_mul, const PlaneSpec& spec,
                            void* a_planes, void* b_planes, hipStream_t st, const uint32_t* marks = nullptr,
                            int64_t tile_bm = 0);

// Fused p-family GEMM + selection epilogue.
hipError_t launch_pfamily_gemm_bf16(const uint16_t* Ap, const uint16_t* Bp, int64_t b, int64_t m,
                                    int64_t n, int64_t mp, int64_t np, int64_t kp, int32_t n_planes,
                                    const FamilyPlan& plan, const EpiArgs& epi, hipStream_t st);
// The rerun launch of deferred planes: the tiles marked in epi.missed_tile
// again from the start, every plane written, without the sparse tail.
hipError_t launch_rerun_gemm_bf16(const uint16_t* Ap, const uint16_t* Bp, int64_t b, int64_t m, int64_t n,
                                  int64_t mp, int64_t np, int64_t kp, int32_t n_planes, const FamilyPlan& plan,
                                  const EpiArgs& epi, hipStream_t st);
// The same for the FP64 path (bm: the forward launch's tile side).
hipError_t launch_rerun_gemm_f64(const double* Ap, const double* Bp, int64_t b, int64_t m, int64_t n, int64_t mp,
                                 int64_t np, int64_t kp, int32_t n_planes, int bm, const FamilyPlan& plan,
                                 const EpiArgs& epi, hipStream_t st);
hipError_t launch_pfamily_gemm_f64(const double* Ap, const double* Bp, int64_t b, int64_t m,
                                   int64_t n, int64_t mp, int64_t np, int64_t kp, int32_t n_planes,
                                   int bm, const FamilyPlan& plan, const EpiArgs& epi,
                                   hipStream_t st);

// FP64 path: C = r c S^(1/p*) from the GEMM's recorded S and p* index.
struct RootSpec {
    int32_t p[MT_MAX_P];
    double corr[MT_MAX_P];
    int32_t mode;   // EpiMode
    int32_t clamp;
    int32_t r1;     // r = 1 projection from S (at p*) and S2 (at the family's next smaller p)
};
// The one-kernel FP64-path estimate of small products (mt_small.hip): the
// family (ascending), its norm corrections, tau and the clamp to 1.
struct SmallSpec {
    int32_t n;
    int32_t p[MT_MAX_P];
    double corr[MT_MAX_P];
    double tau;
    int32_t clamp;
};
hipError_t launch_small_product_f64(const void* A, const void* B, int in_f64, int64_t b, int64_t m, int64_t k,
                                    int64_t n, const SmallSpec& spec, void* C, int out_f64, uint8_t* pstar,
                                    hipStream_t st);
// r = 2 projection over an S stack (plane t holds S at the t-th smallest of
// the family's p and the added 3q): per family index fi, the stack plane of
// its p (plane), of the next smaller family p (lo, -1 if none) and of q,
// 2q, 3q, 4q with 4q = its p (q4, -1 where the projection does not apply).
struct R2Spec {
    int32_t n;  // family size
    int32_t p[MT_MAX_P];
    int32_t plane[MT_MAX_P];
    int32_t lo[MT_MAX_P];
    int32_t q4[MT_MAX_P][4];
    double tau;
    int32_t mode;
    int32_t clamp;
    double k_inner;  // inner length K of the product (the rank-1 threshold)
};
hipError_t launch_select_r2_f64(const double* stack, int64_t stride, int64_t b, int64_t m, int64_t n,
                                const double* r, const double* c, const R2Spec& spec, void* out, int out_f64,
                                uint8_t* pstar_out, hipStream_t st);
hipError_t launch_select_root_f64(const double* S, const double* S2, const uint8_t* code, int64_t b,
                                  int64_t m, int64_t n, const double* r, const double* c,
                                  const RootSpec& spec, void* out, int out_f64, uint8_t* pstar_out,
                                  hipStream_t st);

// Backward: p* histogram and adjoint planes.
struct AdjPrepSpec {
    int32_t n_p;
    int32_t p[MT_MAX_P];
    int32_t planes;                    // adjoint planes per batch item (2 n_p BF16, n_p FP64)
    int64_t xa_rows_pad, xa_cols_pad;  // Gt planes (rows m, inner n)
    int64_t yb_rows_pad, yb_cols_pad;  // Gt' planes, transposed (rows n, inner m)
};
hipError_t launch_pstar_hist(const uint8_t* ps, int64_t total, int n_p, int32_t* hist, hipStream_t st);
// ex (nullable, 2 b entries, from launch_scale_exp): the planes then carry
// r_i / 2^ex[bi] and c_j / 2^ex[b + bi].
hipError_t launch_scale_exp(const double* r, const double* c, int64_t b, int64_t m, int64_t n, int32_t* ex,
                            hipStream_t st);
hipError_t launch_adjoint_prep(const void* G, const void* C, const uint8_t* pstar, int io_f64,
                               const double* r, const double* c, const int32_t* ex, int64_t b, int64_t m,
                               int64_t n, const AdjPrepSpec& spec, const int32_t* hist, int bf16, void* XA,
                               void* YB, hipStream_t st);

// Adjoint GEMMs (rows x cols output, inner k_pad; X planes per batch item,
// Y planes per batch item).
hipError_t launch_adjoint_gemm_bf16(const uint16_t* Xp, const uint16_t* Yp, int64_t b, int64_t rows,
                                    int64_t cols, int64_t rows_pad, int64_t cols_pad, int64_t kp,
                                    int32_t x_planes, int32_t y_planes, const FamilyPlan& plan,
                                    const AdjArgs& adj, hipStream_t st);
hipError_t launch_adjoint_gemm_f64(const double* Xp, const double* Yp, int64_t b, int64_t rows,
                                   int64_t cols, int64_t rows_pad, int64_t cols_pad, int64_t kp,
                                   int32_t x_planes, int32_t y_planes, const FamilyPlan& plan,
                                   const AdjArgs& adj, hipStream_t st);

// Max-convolution (Sec. 1): FFT size N = 2^logN >= n + m - 1, at most
// kMaxConvN points (the FFT runs in one workgroup's LDS).
constexpr int kMaxConvLog = 12;
constexpr int kMaxConvN = 1 << kMaxConvLog;
// The x + y ring results of longer lists go through global buffers, up to
// kLongConvN points.
constexpr int kLongConvLog = 14;
constexpr int kLongConvN = 1 << kLongConvLog;
struct MaxconvSpec {
    int32_t n;  // family size
    int32_t p[MT_MAX_P];
    double tau;
};
int maxconv_log_size(int64_t n, int64_t m);
// Buffers of the long-vector path (N > kMaxConvN); unused (null) below.
struct MaxconvWorkspace {
    double2* tw;     // twiddle octant, N / 8 + 1
    double* rxy;     // b: max x max y
    double* inv;     // 2b: 1 / max x, 1 / max y
    double* s_sel;   // b (n + m - 1): S at the selected p
    uint8_t* code;   // b (n + m - 1): its family index, MT_PSTAR_NONE, or open
    double2* buf0;   // b N
    double2* buf1;   // b N
};
hipError_t launch_maxconv(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                          const MaxconvSpec& spec, void* z, uint8_t* pstar, const MaxconvWorkspace& w,
                          hipStream_t st);
hipError_t launch_maxconv_exact(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                                void* z, hipStream_t st);
// Top k of x + y (Sec. 2.3): ring results of both runs, the second run's
// values and both runs' diagonals.
struct XyWorkspace {
    double* sigma;    // 2 x n_p x (2n - 1)
    double* psi;      // 2 x (2n - 1): the estimates before any pop
    double* values1;  // k
    int32_t* diag0;   // k
    int32_t* diag1;   // k
    // only for N > kMaxConvN: twiddle octant, maxima of x and y, two buffers of 2 n_p N
    double2* tw;
    double* mxy;
    double2* buf0;
    double2* buf1;
    // k <= kPairedMaxK: K = min(k, 2n - 1) candidates per run
    int32_t* cand_m;    // 2 x K
    double* cand_psi;   // 2 x K
    double* cand_cols;  // 2 x n_p x K: the candidates' sigma columns
};
// largest k of the queue over candidates (their estimates live in LDS); the
// paired queue needs it, the plain one falls back to every diagonal above
constexpr int kPairedMaxK = 4096;
hipError_t launch_xy_topk(const void* x, const void* y, int f64, int64_t n, int32_t k, const MaxconvSpec& spec,
                          bool paired, double* values, int32_t* diag, int32_t* ii, int32_t* jj,
                          const XyWorkspace& w, hipStream_t st);

// Exact (max, x) product on the vector ALUs.
hipError_t launch_exact_maxtimes(const void* A, const void* B, int f64, int64_t b, int64_t m,
                                 int64_t k, int64_t n, void* E, hipStream_t st);

// Per-kernel event timing (api.cpp).
void timing_before(const char* name, hipStream_t st);
void timing_after(hipStream_t st);
// Timing slot of the launch just opened by timing_before (nullptr when
// timing is off): kTimingSlotWords counters in device memory.  Word 0: the
// work the kernel executed (it adds to it).  Words 1 and 2: the earliest
// start and the latest end, over the kernel's workgroups, of the device's
// constant-rate real-time counter, so that the launch's span on the device
// is known independently of how the host-side events are stamped.
constexpr int kTimingSlotWords = 4;
unsigned long long* timing_work_slot();

__device__ __forceinline__ void timing_span_begin(unsigned long long* slot) {
    atomicMin(slot + 1, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}
__device__ __forceinline__ void timing_span_end(unsigned long long* slot) {
    atomicMax(slot + 2, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}

}  // namespace mt
