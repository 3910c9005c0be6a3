// p-family GEMMs on FP64 MFMA (gfx950): the plain-precision path.  Same
// scheme as the BF16 kernels (one main loop, two epilogues), with FP64 planes
// and v_mfma_f64_16x16x4f64.
//
// Forward (selection-record epilogue).  Ring products of every p of the
// family per output tile, largest p first (Alg. 5 and Sec. 1).  Once per
// entry the epilogue records the ring result S at the largest p with
// S_p >= tau (FP64 test) and that p's index; the FP64 root C = r c S^(1/p) is
// taken by the select-root pass (mt_elementwise.hip), which keeps the
// library's log / exp out of the unrolled epilogue.  A tile whose entries all
// have their p stops: the smaller p cannot change the result.
//
// Adjoint (accumulating epilogue).  As in the BF16 kernel: sum over the p
// some entry uses of (scaled input)^(p-1) .* (X_p Y_p^T), written once.
//
// Tiling: 256 threads = 4 waves in 2 x 2; each wave owns WT x WT MFMA tiles of
// 16 x 16.  K step 16 doubles = 128-byte LDS rows, loaded by
// global_load_lds_dwordx4 and double buffered; 16-byte chunk index
// XOR-swizzled with (row >> 1) & 7.  At most 256 registers per lane, so two
// workgroups share a CU and one hides the other's barrier waits.
#include <atomic>
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;

struct GemmGeomF64 {
    const double* X;
    const double* Y;
    int64_t x_plane_elems;
    int64_t y_plane_elems;
    int64_t x_batch_elems;
    int64_t y_batch_elems;
    int64_t kp;
    int64_t rows, cols;
    int32_t tiles_m, tiles_n;
    int32_t bm;                // output tile side
    unsigned long long* work;  // if set: MFMA flops executed, summed over workgroups
};

template <int WT_>
struct CfgF64 {
    static constexpr int WT = WT_;
    static constexpr int BM = 2 * WT * 16;
    static constexpr int A_BYTES = BM * 128;
    static constexpr int BUF_BYTES = 2 * A_BYTES;
    static constexpr int PIPE_BYTES = 2 * BUF_BYTES;
    static_assert((BM / 32) % 2 == 0, "row groups per wave must be even");
};

struct TileCtx {
    int lane, wave, wm, wn, bi;
    int64_t row0, col0;
};

// ------------------------------------------------------------ selection record
template <class C, bool R1, bool RERUN = false>
struct RecordEpi {
    static constexpr int WT = C::WT;
    static constexpr int NDEC = (WT * WT * 4 + 31) / 32;
    static constexpr int LDS_BYTES = 0;
    using Args = EpiArgs;
    EpiArgs a;
    int64_t n;
    uint32_t decided[NDEC];
    // r = 1 projection: S_{p*} recorded, S at the next smaller p still due;
    // otherwise: parked, i.e. stable at the p recorded and a larger p may be
    // stable too
    uint32_t pending[NDEC];
    int lr0, lc0;
    int64_t out_lane;
    int32_t rows_left, cols_left;
    int32_t n_eval;  // plan entries whose planes this launch may read

    static constexpr bool kCanStop = true;
    __device__ bool active(int, const FamilyPlan&) const { return true; }
    // Deferred planes: the planes of plan entries n_eval and below are not
    // written (yet), so the way down ends above them.  The rerun launch runs
    // only the tiles marked for it, with every plane written, densely to the
    // end.
    __device__ int down_end(const FamilyPlan& plan) const { return min(plan.n, n_eval); }
    static __device__ bool skip_tile(const Args& a, int64_t tile) { return RERUN && a.missed_tile[tile] == 0u; }
    __device__ void record_tile(int64_t tile, bool missed) const {
        if (RERUN || a.missed_tile == nullptr) return;
        a.missed_tile[tile] = missed ? 1u : 0u;
        if (missed) *a.low_missed = 1;
    }

    // Entries of this lane without their final record yet: `open` ones have
    // no stable p so far, `parked` ones wait for the way up (with the r = 1
    // projection, whose search starts at the largest p, all count as open).
    __device__ void counts(int& open, int& parked) const {
        constexpr int TOT = WT * WT * 4;
        open = parked = 0;
#pragma unroll
        for (int i = 0; i < NDEC; ++i) {
            const uint32_t full = (TOT - 32 * i >= 32) ? 0xFFFFFFFFu : ((1u << (TOT - 32 * i)) - 1u);
            const uint32_t und = ~decided[i] & full;
            if (R1) {
                open += __builtin_popcount(und);
            } else {
                parked += __builtin_popcount(und & pending[i]);
                open += __builtin_popcount(und & ~pending[i]);
            }
        }
    }
    __device__ int32_t start_index() const { return (!R1 && a.start) ? *a.start : 0; }
    __device__ bool can_hand_over(int total) const { return !RERUN && a.tail != nullptr && total <= a.tail_max; }
    __device__ uint32_t* tail_counter() const { return a.tail_count; }
    // Write this lane's undecided entries to the sparse-tail list from `pos`
    // on, after plan entry e of a search that started at plan entry s.
    __device__ void hand_over(uint32_t pos, int e, int s, const TileCtx& t) const {
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const int tix = i * WT + j;
                const int sh = (tix & 7) * 4;
#pragma unroll 1
                for (int r = 0; r < 4; ++r) {
                    const uint32_t mask = 1u << (sh + r);
                    if (decided[tix >> 3] & mask) continue;
                    TailEntry te;
                    te.bi = t.bi;
                    te.i = (int32_t)(t.row0 + lr0 + i * 16 + 4 * r);
                    te.j = (int32_t)(t.col0 + lc0 + j * 16);
                    if (pending[tix >> 3] & mask) {
                        te.state = R1 ? kTailR1 : kTailRise;
                        te.e_next = (int16_t)(R1 ? e + 1 : (e < s ? e - 1 : s - 1));
                    } else {
                        te.state = kTailOpen;
                        te.e_next = (int16_t)(e + 1);
                    }
                    a.tail[pos++] = te;
                }
            }
    }

    __device__ void setup(const TileCtx& t, const GemmGeomF64& g, uint8_t*, int) {
        n = g.cols;
        n_eval = MT_MAX_P;
        if (!RERUN && a.low_need != nullptr && __builtin_amdgcn_readfirstlane(*a.low_need) == 0) n_eval = a.n_eval;
#pragma unroll
        for (int i = 0; i < NDEC; ++i) decided[i] = pending[i] = 0u;
        // Entry (i, j, r) of this lane: tile row wm*WT*16 + i*16 + l/16 + 4r,
        // tile column wn*WT*16 + j*16 + l%16.
        lr0 = t.wm * WT * 16 + (t.lane >> 4);
        lc0 = t.wn * WT * 16 + (t.lane & 15);
        out_lane = ((int64_t)t.bi * g.rows + t.row0 + lr0) * n + t.col0 + lc0;
        rows_left = (int32_t)min<int64_t>(g.rows - (t.row0 + lr0), 1 << 30);
        cols_left = (int32_t)min<int64_t>(n - (t.col0 + lc0), 1 << 30);
        // Entries outside the matrix count as decided from the start.
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int tix = i * WT + j;
                    if (!(j * 16 < cols_left && i * 16 + 4 * r < rows_left))
                        decided[tix >> 3] |= 1u << ((tix & 7) * 4 + r);
                }
    }

    // stage: a free pipeline buffer; each wave stages one 16 x 16 tile
    // (lane-major) and walks its four entries per lane in a rolled loop.
    // Plan entry e of a p search that started at plan entry s: entries e >= s
    // go down from the start (smaller p), entries e < s up (larger p).
    __device__ void entry(int e, int s, const FamilyPlan& plan, f64x4 (&acc)[WT][WT], const TileCtx& t,
                          uint8_t* stage) {
        const bool last = (e == plan.n - 1);
        const bool up = e < s;  // only parked entries are left
        const bool park_here = !up && e == s && s > 0;
        const double rise_thr = plan.e[e].rise_thr;
        const double tau = plan.tau;
        const uint8_t pcode = (uint8_t)plan.e[e].pidx;
        // r = 1 projection: S_{p*} goes to `out`, S at the next smaller p to
        // `out2`; the select-root pass combines them
        const bool defer = R1 && plan.e[e].inv_dp > 0.f;
        double* out = (double*)a.out + out_lane;
        double* out2 = a.out2 ? (double*)a.out2 + out_lane : nullptr;
        uint8_t* ps = a.pstar + out_lane;
        double* stg = (double*)stage + t.wave * 256;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) stg[r * 64 + t.lane] = acc[i][j][r];
                __builtin_amdgcn_wave_barrier();
                const bool col_ok = j * 16 < cols_left;
                const int tix = i * WT + j;
                uint32_t dec = decided[tix >> 3];
                uint32_t pnd = pending[tix >> 3];
                const int sh = (tix & 7) * 4;
#pragma unroll 1
                for (int r = 0; r < 4; ++r) {
                    const uint32_t mask = 1u << (sh + r);
                    const int roff = i * 16 + 4 * r;
                    const double S = stg[r * 64 + t.lane];
                    const bool stable = S >= tau;
                    const int64_t o = (int64_t)roff * n + j * 16;
                    if constexpr (!R1) {
                        // entries outside the matrix are decided from the start
                        if (dec & mask) continue;
                        if (!up) {
                            if (pnd & mask) continue;  // parked at the start: waits for the way up
                            if (!(stable || last)) continue;
                            out[o] = S;
                            ps[o] = stable ? pcode : (uint8_t)MT_PSTAR_NONE;
                            // S_q <= S^(q/p): the next larger q may still pass
                            if (stable && park_here && S >= rise_thr)
                                pnd |= mask;
                            else
                                dec |= mask;
                        } else {
                            // not stable here: the record of the p below stands
                            if (stable) {
                                out[o] = S;
                                ps[o] = pcode;
                                if (e > 0 && S >= rise_thr) continue;
                            }
                            pnd &= ~mask;
                            dec |= mask;
                        }
                        continue;
                    }
                    if (pnd & mask) {
                        out2[o] = S;
                        pnd &= ~mask;
                        dec |= mask;
                    } else if (col_ok && roff < rows_left && !(dec & mask) && (stable || last)) {
                        out[o] = S;
                        ps[o] = stable ? pcode : (uint8_t)MT_PSTAR_NONE;
                        if (stable && defer)
                            pnd |= mask;
                        else
                            dec |= mask;
                    }
                }
                decided[tix >> 3] = dec;
                pending[tix >> 3] = pnd;
                __builtin_amdgcn_wave_barrier();
            }
    }

    __device__ void finish(const TileCtx&) {}
};

// ------------------------------------------------------------ store-all epilogue
// S of plan entry e to plane pidx of the stack out (planes of b x rows x n),
// every entry of the tile, every entry of the plan: the r = 2 projection
// needs four ring results per entry, chosen after p* is known.
template <class C>
struct StoreAllEpi {
    static constexpr int WT = C::WT;
    static constexpr int LDS_BYTES = 0;
    using Args = EpiArgs;
    static constexpr bool kCanStop = false;
    EpiArgs a;
    int64_t n, out_lane;
    int32_t rows_left, cols_left;

    __device__ bool active(int, const FamilyPlan&) const { return true; }
    __device__ int down_end(const FamilyPlan& plan) const { return plan.n; }
    static __device__ bool skip_tile(const Args&, int64_t) { return false; }
    __device__ void record_tile(int64_t, bool) const {}
    __device__ void counts(int& open, int& parked) const { open = parked = 0; }
    __device__ int32_t start_index() const { return 0; }
    __device__ bool can_hand_over(int) const { return false; }
    __device__ uint32_t* tail_counter() const { return nullptr; }
    __device__ void hand_over(uint32_t, int, int, const TileCtx&) const {}

    __device__ void setup(const TileCtx& t, const GemmGeomF64& g, uint8_t*, int) {
        n = g.cols;
        const int lr0 = t.wm * WT * 16 + (t.lane >> 4);
        const int lc0 = t.wn * WT * 16 + (t.lane & 15);
        out_lane = ((int64_t)t.bi * g.rows + t.row0 + lr0) * n + t.col0 + lc0;
        rows_left = (int32_t)min<int64_t>(g.rows - (t.row0 + lr0), 1 << 30);
        cols_left = (int32_t)min<int64_t>(n - (t.col0 + lc0), 1 << 30);
    }

    // accumulator (i, j, r) of this lane: tile row i*16 + l/16 + 4r, column
    // j*16 + l%16 (the v_mfma_f64_16x16x4f64 layout)
    __device__ void entry(int e, int, const FamilyPlan& plan, f64x4 (&acc)[WT][WT], const TileCtx&, uint8_t*) {
        double* out = (double*)a.out + (int64_t)plan.e[e].pidx * a.stack_stride + out_lane;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    if (j * 16 < cols_left && i * 16 + 4 * r < rows_left)
                        out[(int64_t)(i * 16 + 4 * r) * n + j * 16] = acc[i][j][r];
    }

    __device__ void finish(const TileCtx&) {}
};

// ------------------------------------------------------------ adjoint epilogue
template <class C, typename TM>
struct AdjointEpiF64 {
    static constexpr int WT = C::WT;
    // inverse mantissas of the row and column scales, then their exponents
    static constexpr int LDS_BYTES = 2 * C::BM * 8 + 2 * C::BM * 4;
    using Args = AdjArgs;
    static constexpr bool kCanStop = false;
    AdjArgs a;
    int64_t rows, cols;
    f64x4 tot[WT][WT];
    __device__ int down_end(const FamilyPlan& plan) const { return plan.n; }
    static __device__ bool skip_tile(const Args&, int64_t) { return false; }
    __device__ void record_tile(int64_t, bool) const {}
    double* rs;
    double* cs;
    int* res;
    int* ces;
    int lr0, lc0;
    int64_t lane_off;
    int32_t rows_left, cols_left;

    __device__ bool active(int e, const FamilyPlan& plan) const { return a.hist[plan.e[e].pidx] > 0; }
    __device__ void counts(int& open, int& parked) const { open = parked = 0; }
    __device__ int32_t start_index() const { return 0; }
    __device__ bool can_hand_over(int) const { return false; }
    __device__ uint32_t* tail_counter() const { return nullptr; }
    __device__ void hand_over(uint32_t, int, int, const TileCtx&) const {}

    __device__ void setup(const TileCtx& t, const GemmGeomF64& g, uint8_t* lds, int tid) {
        rows = g.rows;
        cols = g.cols;
        rs = (double*)lds;
        cs = rs + C::BM;
        res = (int*)(rs + 2 * C::BM);
        ces = res + C::BM;
        // scale v = m 2^e: M / v is formed as (M 2^-e) / m, finite also for
        // a subnormal scale (whose reciprocal is not)
        for (int i = tid; i < 2 * C::BM; i += kThreads) {
            double v = 1.0;
            if (i < C::BM) {
                if (a.scale_rows && t.row0 + i < rows) v = a.scale_rows[(int64_t)t.bi * rows + t.row0 + i];
            } else {
                const int64_t cc = t.col0 + (i - C::BM);
                if (a.scale_cols && cc < cols) v = a.scale_cols[(int64_t)t.bi * cols + cc];
            }
            int e = 0;
            const double m = v > 0.0 ? frexp(v, &e) : 0.0;
            rs[i] = m > 0.0 ? 1.0 / m : 0.0;
            res[i] = e;
        }
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) tot[i][j] = f64x4{};
        lr0 = t.wm * WT * 16 + (t.lane >> 4);
        lc0 = t.wn * WT * 16 + (t.lane & 15);
        lane_off = ((int64_t)t.bi * rows + t.row0 + lr0) * cols + t.col0 + lc0;
        rows_left = (int32_t)min<int64_t>(rows - (t.row0 + lr0), 1 << 30);
        cols_left = (int32_t)min<int64_t>(cols - (t.col0 + lc0), 1 << 30);
    }

    __device__ void entry(int e, int, const FamilyPlan& plan, f64x4 (&acc)[WT][WT], const TileCtx&, uint8_t*) {
        const int pm1 = plan.e[e].p - 1;
        const TM* src = (const TM*)a.M + lane_off;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                const bool col_ok = j * 16 < cols_left;
                const double cinv = cs[lc0 + j * 16];
                const int cexp = ces[lc0 + j * 16];
                double x[4], pw[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int roff = i * 16 + 4 * r;
                    x[r] = (col_ok && roff < rows_left)
                               ? __builtin_amdgcn_ldexp((double)src[(int64_t)roff * cols + j * 16],
                                                        -(res[lr0 + roff] + cexp)) *
                                     rs[lr0 + roff] * cinv
                               : 0.0;
                    pw[r] = 1.0;
                }
                for (int ex = pm1; ex; ex >>= 1) {
                    if (ex & 1) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) pw[r] *= x[r];
                    }
#pragma unroll
                    for (int r = 0; r < 4; ++r) x[r] *= x[r];
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) tot[i][j][r] += pw[r] * acc[i][j][r];
            }
    }

    __device__ void finish(const TileCtx& t) {
        const int64_t row_base = (int64_t)t.bi * rows + t.row0 + lr0;
        const int64_t col_base = (int64_t)t.bi * cols + t.col0 + lc0;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) {
                if (!(j * 16 < cols_left)) continue;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int roff = i * 16 + 4 * r;
                    if (roff < rows_left) {
                        const int64_t o = lane_off + (int64_t)roff * cols + j * 16;
                        double w = tot[i][j][r];
                        // chain factors of a balanced forward
                        if (a.out_row_mul) w *= a.out_row_mul[row_base + roff];
                        if (a.out_col_mul) w *= a.out_col_mul[col_base + j * 16];
                        if (a.out_f64)
                            ((double*)a.out)[o] = w;
                        else
                            ((float*)a.out)[o] = (float)w;
                    }
                }
            }
    }
};

// ------------------------------------------------------------ the main loop
template <class C, class Epi>
__global__ __launch_bounds__(kThreads, 2) void mt_pfamily_gemm_f64_kernel(GemmGeomF64 g,
                                                                         FamilyPlan plan,
                                                                         typename Epi::Args args) {
    constexpr int WT = C::WT;
    extern __shared__ __attribute__((aligned(1024))) uint8_t smem[];
    __shared__ int s_act[MT_MAX_P + 1];
    __shared__ int s_done[2][4];  // per wave: undecided entries (entry parity)
    __shared__ int s_open[2][4];  // per wave: of which open (entry parity)
    __shared__ uint32_t s_tail_base;

    const int tid = threadIdx.x;
    if (g.work && tid == 0) timing_span_begin(g.work);
    TileCtx t;
    t.lane = tid & 63;
    t.wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    t.wm = t.wave >> 1;
    t.wn = t.wave & 1;
    const int lane = t.lane;
    const int wave = t.wave;

    int id = blockIdx.x;
    const int nwg = gridDim.x;
    if ((nwg & 7) == 0) id = (id & 7) * (nwg >> 3) + (id >> 3);
    const int per_batch = g.tiles_m * g.tiles_n;
    t.bi = id / per_batch;
    const int tt = id - t.bi * per_batch;
    constexpr int GROUP = 8;
    const int group = tt / (GROUP * g.tiles_n);
    const int first_m = group * GROUP;
    const int gsz = min(GROUP, g.tiles_m - first_m);
    const int in_g = tt - group * GROUP * g.tiles_n;
    const int tm = first_m + in_g % gsz;
    const int tn = in_g / gsz;
    t.row0 = (int64_t)tm * C::BM;
    t.col0 = (int64_t)tn * C::BM;
    const int64_t tile_id = (int64_t)t.bi * per_batch + (int64_t)tm * g.tiles_n + tn;
    if (Epi::skip_tile(args, tile_id)) return;

    Epi epi;
    epi.a = args;
    epi.setup(t, g, smem + C::PIPE_BYTES, tid);
    if (tid == 0) epi.record_tile(tile_id, false);
    // The p search starts at plan entry e0 (0: the largest p), goes down to
    // the smallest p and then up from e0 - 1 to the largest; s_act holds the
    // active plan entries in that order.
    const int e0_req = __builtin_amdgcn_readfirstlane(epi.start_index());
    const int e0 = e0_req < 0 ? 0 : (e0_req >= plan.n ? plan.n - 1 : e0_req);
    // deferred planes not written: the way down ends above them
    const int e_end = epi.down_end(plan);
    if (tid == 0) {
        int na = 0;
        for (int e = e0; e < e_end; ++e)
            if (epi.active(e, plan)) s_act[1 + na++] = e;
        for (int e = e0 - 1; e >= 0; --e)
            if (epi.active(e, plan)) s_act[1 + na++] = e;
        s_act[0] = na;
    }

    const double* Xbase = g.X + (int64_t)t.bi * g.x_batch_elems + t.row0 * g.kp;
    const double* Ybase = g.Y + (int64_t)t.bi * g.y_batch_elems + t.col0 * g.kp;
    const int nkt = (int)(g.kp / 16);

    // Loads: lane l fills row R0 + l/8, physical 16-byte chunk l%8 holding
    // logical chunk (l%8) ^ swz(row) = (l%8) ^ ((i&1)*4 + l/16).
    const int32_t ld_even = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (lane >> 4)) * 2);
    const int32_t ld_odd = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (4 + (lane >> 4))) * 2);
    // Operand reads: row l%16 of a 16-row block, k = 4*kk + l/16, i.e.
    // logical chunk 2*kk + l/32, half (l/16)&1; swizzle (l >> 1) & 7.
    const int32_t rd_base = (lane & 15) * 128 + (((lane >> 5) ^ ((lane >> 1) & 7)) * 16) + ((lane >> 4) & 1) * 8;

    __syncthreads();
    const int nact = __builtin_amdgcn_readfirstlane(s_act[0]);

    auto issue = [&](int ai, int s, int kt, int buf) {
        const int e = __builtin_amdgcn_readfirstlane(s_act[1 + ai]);
        const double* xsrc = Xbase + (int64_t)plan.e[e].a_plane[s] * g.x_plane_elems + kt * 16;
        const double* ysrc = Ybase + (int64_t)plan.e[e].b_plane[s] * g.y_plane_elems + kt * 16;
        uint8_t* la = smem + buf * C::BUF_BYTES;
        uint8_t* lb = la + C::A_BYTES;
#pragma unroll
        for (int i = 0; i < C::BM / 32; ++i) {
            const int R0 = (wave * (C::BM / 32) + i) * 8;
            const int32_t lo = (i & 1) ? ld_odd : ld_even;
            __builtin_amdgcn_global_load_lds((glb_cvoid*)(xsrc + (int64_t)R0 * g.kp + lo),
                                             (lds_void*)(la + R0 * 128), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((glb_cvoid*)(ysrc + (int64_t)R0 * g.kp + lo),
                                             (lds_void*)(lb + R0 * 128), 16, 0, 0);
        }
    };
    auto advance = [&](int& ai, int& s, int& kt) {
        if (++kt == nkt) {
            kt = 0;
            const int e = __builtin_amdgcn_readfirstlane(s_act[1 + ai]);
            if (++s == plan.e[e].nseg) {
                s = 0;
                ++ai;
            }
        }
    };

    int la_ = 0, ls = 0, lkt = 0;
    if (nkt > 0 && nact > 0) {
        issue(la_, ls, lkt, 0);
        advance(la_, ls, lkt);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    int buf = 0;
    int64_t steps_done = 0;
    for (int ai = 0; ai < nact; ++ai) {
        const int e = __builtin_amdgcn_readfirstlane(s_act[1 + ai]);
        f64x4 acc[WT][WT];
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) acc[i][j] = f64x4{};

        const int ntiles = plan.e[e].nseg * nkt;
        for (int st = 0; st < ntiles; ++st) {
            if (la_ < nact) {
                issue(la_, ls, lkt, buf ^ 1);
                advance(la_, ls, lkt);
            }
            const uint8_t* pa = smem + buf * C::BUF_BYTES + t.wm * WT * 16 * 128;
            const uint8_t* pb = smem + buf * C::BUF_BYTES + C::A_BYTES + t.wn * WT * 16 * 128;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int32_t ro = rd_base ^ (kk << 5);
                double a[WT], b[WT];
#pragma unroll
                for (int i = 0; i < WT; ++i) a[i] = *(const double*)(pa + i * 16 * 128 + ro);
#pragma unroll
                for (int j = 0; j < WT; ++j) b[j] = *(const double*)(pb + j * 16 * 128 + ro);
#pragma unroll
                for (int i = 0; i < WT; ++i)
#pragma unroll
                    for (int j = 0; j < WT; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
            }

            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            buf ^= 1;
        }
        steps_done += ntiles;
        // the buffer the last step read is free until the next step's loads,
        // which wait for the barrier below
        epi.entry(e, e0, plan, acc, t, smem + (buf ^ 1) * C::BUF_BYTES);
        int lane_pre = 0;
        if (Epi::kCanStop) {
            int n_open, n_parked;
            epi.counts(n_open, n_parked);
            const int cnt = n_open + n_parked;
            int incl = cnt, incl_open = n_open;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const int y = __shfl_up(incl, d);
                const int yo = __shfl_up(incl_open, d);
                if (lane >= d) {
                    incl += y;
                    incl_open += yo;
                }
            }
            lane_pre = incl - cnt;
            const int wtot = __shfl(incl, 63);
            const int wopen = __shfl(incl_open, 63);
            if (lane == 0) {
                s_done[ai & 1][wave] = wtot;
                s_open[ai & 1][wave] = wopen;
            }
        }
        __syncthreads();
        if (Epi::kCanStop) {
            int total = 0, open = 0, wave_pre = 0;
#pragma unroll
            for (int w = 0; w < 4; ++w) {
                const int x = s_done[ai & 1][w];
                total += x;
                open += s_open[ai & 1][w];
                wave_pre += w < wave ? x : 0;
            }
            total = __builtin_amdgcn_readfirstlane(total);
            open = __builtin_amdgcn_readfirstlane(open);
            // every entry has its p; the next entry's loads have landed
            // (vmcnt(0) above) and are left unused
            if (total == 0) break;
            // a few left: the sparse tail finishes them
            if (ai + 1 < nact && epi.can_hand_over(total)) {
                if (tid == 0) s_tail_base = atomicAdd(epi.tail_counter(), (uint32_t)total);
                __syncthreads();
                epi.hand_over(s_tail_base + (uint32_t)(wave_pre + lane_pre), e, e0, t);
                break;
            }
            // deferred planes: entries still open after the way down (which
            // ends above the deferred p) and not handed to the tail need
            // those p; the tile runs again once their planes are written
            // (what it records meanwhile is overwritten then)
            if (e_end < plan.n && e == e_end - 1 && open > 0 && tid == 0) epi.record_tile(tile_id, true);
            // going down with nothing open left: only the entries parked at
            // the start wait, for larger p; skip to the way up (plan entry
            // e0 - 1) and reload its first K step in place of the prefetched one
            const int n_down = e_end - e0;
            if (open == 0 && e >= e0 && e0 > 0 && ai + 1 < n_down) {
                ai = n_down - 1;  // ++ai below -> first entry of the way up
                la_ = n_down;
                ls = 0;
                lkt = 0;
                if (nkt > 0) {
                    issue(la_, ls, lkt, buf);
                    advance(la_, ls, lkt);
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
            }
        }
    }
    epi.finish(t);
    if (g.work) {
        // timed launch: the work, and the end once every wave is done
        __syncthreads();
        if (tid == 0) {
            atomicAdd(g.work, (unsigned long long)steps_done * (2ull * C::BM * C::BM * 16));
            timing_span_end(g.work);
        }
    }
}

// ------------------------------------------------------------ the sparse tail
// One wave per handed-over entry: S_p as an FP64 dot product of the entry's
// X and Y plane rows for the plan entries from e_next on, recorded exactly
// as the record epilogue does (S, p* index; with the r = 1 projection S at
// the next smaller p in out2) for the select-root pass.
// S_p of one entry: lane l sums the 2-element chunks l, l + 64, ... in
// order, U chunks loaded before any is used (16 loads in flight per wave).
__device__ double tail_dot_f64(const double* xr, const double* yr, const PlanEntry& pe, const GemmGeomF64& g,
                               int lane) {
    const double* xp = xr + (int64_t)pe.a_plane[0] * g.x_plane_elems;
    const double* yp = yr + (int64_t)pe.b_plane[0] * g.y_plane_elems;
    double acc = 0.0;
    int64_t k0 = lane * 2;
    constexpr int U = 8;
    for (; k0 + (U - 1) * 128 < g.kp; k0 += U * 128) {
        double2 vx[U], vy[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            vx[u] = *(const double2*)(xp + k0 + u * 128);
            vy[u] = *(const double2*)(yp + k0 + u * 128);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc = fma(vx[u].x, vy[u].x, acc);
            acc = fma(vx[u].y, vy[u].y, acc);
        }
    }
    for (; k0 < g.kp; k0 += 128) {
        const double2 vx = *(const double2*)(xp + k0), vy = *(const double2*)(yp + k0);
        acc = fma(vx.x, vy.x, acc);
        acc = fma(vx.y, vy.y, acc);
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) acc += __shfl_xor(acc, d);
    return acc;
}

template <bool R1>
__global__ __launch_bounds__(256) void mt_tail_f64_kernel(GemmGeomF64 g, FamilyPlan plan, EpiArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t count = __builtin_amdgcn_readfirstlane(*a.tail_count);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    // each wave takes a contiguous run of the row-sorted list
    const int64_t run = ((int64_t)count + waves - 1) / waves;
    const int64_t w0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * run;
    const int64_t w1 = min<int64_t>(w0 + run, (int64_t)count);
    double* out = (double*)a.out;
    double* out2 = (double*)a.out2;
    // deferred planes not written: an entry that reaches them marks its tile
    // for the rerun launch instead
    int n_eval = MT_MAX_P;
    if (a.low_need != nullptr && __builtin_amdgcn_readfirstlane(*a.low_need) == 0) n_eval = a.n_eval;
    for (int64_t w = w0; w < w1; ++w) {
        const TailEntry te = a.tail_sorted[w];
        const int64_t o = ((int64_t)te.bi * g.rows + te.i) * g.cols + te.j;
        const double* xr = g.X + (int64_t)te.bi * g.x_batch_elems + (int64_t)te.i * g.kp;
        const double* yr = g.Y + (int64_t)te.bi * g.y_batch_elems + (int64_t)te.j * g.kp;
        if (!R1 && te.state == kTailRise) {
            // stable at e_next + 1 (recorded): go up while a larger p may be
            // stable too; an unstable p leaves the record below standing
            for (int e = te.e_next; e >= 0; --e) {
                const PlanEntry& pe = plan.e[e];
                const double acc = tail_dot_f64(xr, yr, pe, g, lane);
                if (!(acc >= plan.tau)) break;
                if (lane == 0) {
                    out[o] = acc;
                    a.pstar[o] = (uint8_t)pe.pidx;
                }
                if (!(acc >= pe.rise_thr)) break;
            }
            continue;
        }
        bool pend = R1 && te.state == kTailR1;
        for (int e = te.e_next; e < plan.n; ++e) {
            if (e >= n_eval) {
                if (lane == 0) {
                    a.missed_tile[((int64_t)te.bi * g.tiles_m + te.i / g.bm) * g.tiles_n + te.j / g.bm] = 1u;
                    *a.low_missed = 1;
                }
                break;
            }
            const PlanEntry& pe = plan.e[e];
            const double acc = tail_dot_f64(xr, yr, pe, g, lane);
            if (R1 && pend) {
                if (lane == 0) out2[o] = acc;
                break;
            }
            const bool stable = acc >= plan.tau;
            if (!(stable || e == plan.n - 1)) continue;
            if (lane == 0) {
                out[o] = acc;
                a.pstar[o] = stable ? (uint8_t)pe.pidx : (uint8_t)MT_PSTAR_NONE;
            }
            if (R1 && stable && pe.inv_dp > 0.f) {
                pend = true;
                continue;
            }
            break;
        }
    }
}

template <class C, class Epi>
hipError_t launch_gemm(const GemmGeomF64& g, int64_t b, const FamilyPlan& plan,
                       const typename Epi::Args& args, const char* name, hipStream_t st) {
    const int lds = C::PIPE_BYTES + Epi::LDS_BYTES;
    auto kern = mt_pfamily_gemm_f64_kernel<C, Epi>;
    // the dynamic-LDS limit is a per-device attribute of the kernel
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_set.load() & bit)) {
        e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    const int64_t nwg = b * (int64_t)g.tiles_m * g.tiles_n;
    timing_before(name, st);
    GemmGeomF64 gw = g;
    gw.work = timing_work_slot();
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(kThreads), lds, st, gw, plan, args);
    timing_after(st);
    return hipGetLastError();
}

GemmGeomF64 make_geom(const double* X, const double* Y, int64_t rows, int64_t cols, int64_t rows_pad,
                      int64_t cols_pad, int64_t kp, int32_t x_planes, int32_t y_planes, int bm) {
    GemmGeomF64 g;
    g.X = X;
    g.Y = Y;
    g.x_plane_elems = rows_pad * kp;
    g.y_plane_elems = cols_pad * kp;
    g.x_batch_elems = g.x_plane_elems * x_planes;
    g.y_batch_elems = g.y_plane_elems * y_planes;
    g.kp = kp;
    g.rows = rows;
    g.cols = cols;
    g.tiles_m = (int32_t)(rows_pad / bm);
    g.tiles_n = (int32_t)(cols_pad / bm);
    g.bm = bm;
    g.work = nullptr;
    return g;
}

}  // namespace

hipError_t launch_pfamily_gemm_f64(const double* Ap, const double* Bp, int64_t b, int64_t m,
                                   int64_t n, int64_t mp, int64_t np, int64_t kp, int32_t n_planes,
                                   int bm, const FamilyPlan& plan, const EpiArgs& epi,
                                   hipStream_t st) {
    const GemmGeomF64 g = make_geom(Ap, Bp, m, n, mp, np, kp, n_planes, n_planes, bm);
    const char* name = "mt_pfamily_gemm_f64";
    hipError_t e = hipErrorInvalidValue;
    if (epi.mode == EPI_STORE_ALL) {
        if (bm == 128) return launch_gemm<CfgF64<4>, StoreAllEpi<CfgF64<4>>>(g, b, plan, epi, name, st);
        if (bm == 64) return launch_gemm<CfgF64<2>, StoreAllEpi<CfgF64<2>>>(g, b, plan, epi, name, st);
        return e;
    }
    if (bm == 128)
        e = plan.r1 ? launch_gemm<CfgF64<4>, RecordEpi<CfgF64<4>, true>>(g, b, plan, epi, name, st)
                    : launch_gemm<CfgF64<4>, RecordEpi<CfgF64<4>, false>>(g, b, plan, epi, name, st);
    else if (bm == 64)
        e = plan.r1 ? launch_gemm<CfgF64<2>, RecordEpi<CfgF64<2>, true>>(g, b, plan, epi, name, st)
                    : launch_gemm<CfgF64<2>, RecordEpi<CfgF64<2>, false>>(g, b, plan, epi, name, st);
    if (e != hipSuccess || !epi.tail) return e;
    // the sparse tail for the entries the tiles handed over
    const int64_t cap = (int64_t)epi.tail_max * b * g.tiles_m * g.tiles_n;
    e = launch_tail_sort(epi, g.rows, cap, st);
    if (e != hipSuccess) return e;
    int64_t blocks = (cap + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    timing_before("mt_tail_f64", st);
    if (plan.r1)
        hipLaunchKernelGGL(mt_tail_f64_kernel<true>, dim3((unsigned)blocks), dim3(256), 0, st, g, plan, epi);
    else
        hipLaunchKernelGGL(mt_tail_f64_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, g, plan, epi);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_rerun_gemm_f64(const double* Ap, const double* Bp, int64_t b, int64_t m, int64_t n, int64_t mp,
                                 int64_t np, int64_t kp, int32_t n_planes, int bm, const FamilyPlan& plan,
                                 const EpiArgs& epi, hipStream_t st) {
    if (epi.missed_tile == nullptr || plan.r1 || epi.mode != EPI_PLAIN) return hipErrorInvalidValue;
    const GemmGeomF64 g = make_geom(Ap, Bp, m, n, mp, np, kp, n_planes, n_planes, bm);
    // a launch of its own name: the forward GEMM's timing and work stay apart
    // (a tile that is not marked adds no work and ends no span)
    const char* name = "mt_rerun_gemm_f64";
    if (bm == 128) return launch_gemm<CfgF64<4>, RecordEpi<CfgF64<4>, false, true>>(g, b, plan, epi, name, st);
    if (bm == 64) return launch_gemm<CfgF64<2>, RecordEpi<CfgF64<2>, false, true>>(g, b, plan, epi, name, st);
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint_gemm_f64(const double* Xp, const double* Yp, int64_t b, int64_t rows,
                                   int64_t cols, int64_t rows_pad, int64_t cols_pad, int64_t kp,
                                   int32_t x_planes, int32_t y_planes, const FamilyPlan& plan,
                                   const AdjArgs& adj, hipStream_t st) {
    using CA = CfgF64<2>;
    static_assert(CA::BM == kAdjF64BM, "adjoint tile");
    const GemmGeomF64 g = make_geom(Xp, Yp, rows, cols, rows_pad, cols_pad, kp, x_planes, y_planes, CA::BM);
    const char* name = "mt_adjoint_gemm_f64";
    if (adj.m_f64) return launch_gemm<CA, AdjointEpiF64<CA, double>>(g, b, plan, adj, name, st);
    return launch_gemm<CA, AdjointEpiF64<CA, float>>(g, b, plan, adj, name, st);
}

}  // namespace mt
