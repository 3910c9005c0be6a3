// p-family GEMMs on BF16 MFMA (gfx950): one main loop, two epilogues.
//
// Forward (selection epilogue).  For one output tile the kernel runs the ring
// product S_p = A'^p B'^p of every p of the family (Alg. 5, first loop;
// Sec. 2.1 distributivity), one after the other, largest p first, and after
// each p keeps, per entry, the first p whose ring result passes the stability
// test S_p >= tau (Sec. 1, the highest stable p).  Because the entries are
// visited from the largest p down, the first pass is the largest stable p,
// and C = r c S^(1/p) is written exactly once per entry.  Entries that never
// pass take the smallest p (index MT_PSTAR_NONE).  Once every entry of the
// tile has its p, the smaller p cannot change the result and the tile stops:
// the products of those p are not computed at all.
//
// Adjoint (accumulating epilogue).  For the gradient with p* held fixed the
// kernel runs, for every p that some entry uses, the product X_p Y_p of an
// adjoint plane and a power plane, multiplies it elementwise by the scaled
// input to the power p - 1 and sums over p in registers; the tile is written
// once at the end.
//
// Operands are BF16 planes, K contiguous: X planes rows x k_pad and Y planes
// cols x k_pad (Y holds the transpose of the right factor).  A split p is
// three products (hi.hi + hi.lo + lo.hi) accumulated into one FP32 sum.
//
// Tiling: 512 threads = 8 waves (two per SIMD, so one wave's barrier and LDS
// waits overlap the other's MFMAs) in 2 x 4; each wave owns WT_M x WT_N MFMA
// tiles of 32 x 32 (v_mfma_f32_32x32x16_bf16).  The operand tiles of a step
// are copied global -> LDS by the direct-to-LDS loads
// (global_load_lds_dwordx4), double buffered, so the next step's loads fly
// while the current step's MFMAs run.  Every step moves the same bytes:
//   plain p: X and Y tiles, K step 64, 128-byte LDS rows, 16-byte chunk
//            index XOR-swizzled with (row >> 1) & 7;
//   split p: X hi, X lo, Y hi, Y lo tiles, K step 32, 64-byte LDS rows,
//            chunk index XOR-swizzled with (row >> 2) & 3; the three
//            products share each loaded tile, so a split p loads 4/6 of the
//            bytes of three separate products.
// Either swizzle puts the MFMA operand reads (16 rows x one chunk per LDS
// read phase) on distinct banks.
#include <atomic>
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

__device__ __forceinline__ int swz(int row) { return (row >> 1) & 7; }



// A row or column scale as mantissa x 2^exp, mantissa in [0.5, 1) (0 for a
// zero scale).  The epilogues multiply the FP32 mantissas with the root and
// apply the summed exponent with one ldexp in the output's precision, so
// r_i c_j S^(1/p) over- or underflows only where the result itself does,
// whatever the range of r and c (FP64 inputs may hold scales far outside
// FP32; FP32 inputs may have r_i c_j beyond FP32 with a finite result).
struct ScaleSplit {
    float m;
    int e;
};
__device__ __forceinline__ ScaleSplit split_scale(double v) {
    if (!(v > 0.0)) return ScaleSplit{0.f, 0};
    int e = 0;
    const double m = frexp(v, &e);
    return ScaleSplit{(float)m, e};
}
// v * 2^e in the output type, rounded once.
template <typename TO>
__device__ __forceinline__ TO scale_out(float v, int e) {
    if constexpr (sizeof(TO) == 8)
        return __builtin_amdgcn_ldexp((double)v, e);
    else
        return __builtin_amdgcn_ldexpf(v, e);
}

// S^(1/p) in FP32 with the hardware log2 / exp2 (about 1 ulp each); S = 0
// gives 0 (log2 0 = -inf, 2^-inf = 0), denormal S is rescaled first.
__device__ __forceinline__ float root_f32(float S, float inv_p) {
    const bool tiny = S < 1.17549435e-38f;
    const float l = __builtin_amdgcn_logf(tiny ? S * 18446744073709551616.f : S) - (tiny ? 64.f : 0.f);
    return __builtin_amdgcn_exp2f(l * inv_p);
}

struct GemmGeom {
    const uint16_t* X;
    const uint16_t* Y;
    int64_t x_plane_elems;  // rows_pad * k_pad
    int64_t y_plane_elems;  // cols_pad * k_pad
    int64_t x_batch_elems;  // planes per batch item * x_plane_elems
    int64_t y_batch_elems;
    int64_t kp;             // padded inner length
    int64_t rows, cols;     // output rows x cols per batch item
    int32_t tiles_m, tiles_n;
    unsigned long long* work;  // if set: MFMA flops executed, summed over workgroups
};

// WAVES_M x WAVES_N waves, each owning WT_M x WT_N MFMA tiles of 32 x 32.
template <int WAVES_M, int WAVES_N, int WT_M_, int WT_N_, int MINW_ = 1>
struct Cfg {
    static constexpr int MINW = MINW_;  // waves per SIMD the kernel must allow
    static constexpr int NW = WAVES_M * WAVES_N;
    static constexpr int THREADS = 64 * NW;
    static constexpr int WT_M = WT_M_, WT_N = WT_N_;
    static constexpr int BM = WAVES_M * WT_M_ * 32;
    static constexpr int BN = WAVES_N * WT_N_ * 32;
    static constexpr int WN = WAVES_N;
    static constexpr int A_BYTES = BM * 128;
    static constexpr int B_BYTES = BN * 128;
    static constexpr int BUF_BYTES = A_BYTES + B_BYTES;
    static constexpr int PIPE_BYTES = 2 * BUF_BYTES;
    static constexpr int GA = BM / 8 / NW;  // load instructions per wave per plain step (X)
    static constexpr int GB = BN / 8 / NW;  // (Y)
    static constexpr int SA = BM / 16 / NW;  // per wave per split step, each of X hi / X lo
    static constexpr int SB = BN / 16 / NW;  // (Y hi / Y lo)
    static_assert(GA % 2 == 0 && GB % 2 == 0, "row groups per wave must be even");
    static_assert(SA >= 1 && SB >= 1, "split steps need 16 rows per wave");
};

struct TileCtx {
    int lane, wave, wm, wn, bi;
    int64_t row0, col0;
};

// ------------------------------------------------------------ selection epilogue
template <class C, int MODE, typename TO, bool R1, bool RERUN = false>
struct SelectEpi {
    static constexpr int WT_M = C::WT_M, WT_N = C::WT_N;
    static constexpr int NDEC = (WT_M * WT_N * 16 + 31) / 32;
    static constexpr int STG = 16 * 64;  // floats of one wave's staging tile (rolled walk)
    // row and column scales: FP32 mantissas, then int exponents
    static constexpr int LDS_BYTES = (C::BM + C::BN) * 8;
    static_assert(C::NW * STG * 4 <= C::BUF_BYTES, "staging must fit in one pipeline buffer");

    using Args = EpiArgs;
    EpiArgs a;
    int64_t m, n;
    uint32_t decided[NDEC];
    // r = 1 projection: entries whose p* was found at the previous p and
    // whose S_{p*} is parked in `out` until S at this (next smaller) p is known
    uint32_t pending[NDEC];
    // row scales of the tile (BM), then its column scales (BN), each as
    // (FP32 mantissa bits, exponent): one 8-byte LDS read per scale
    int2* rsc;
    int2* csc;
    int lr0, lc0;
    int64_t out_lane;
    int32_t rows_left, cols_left, diag_off;
    int32_t n_eval;  // plan entries whose planes this launch may read

    // Row offset, from this lane's first row lr0, of accumulator element q
    // of sub-tile row i (the 32 x 32 MFMA layout: element q of lane l is row
    // (q / 4) * 8 + (l / 32) * 4 + q % 4, column l % 32 of the sub-tile).
    static __device__ __forceinline__ int roff_of(int i, int q) { return i * 32 + (q >> 2) * 8 + (q & 3); }

    static constexpr bool kAllActive = true;
    static constexpr bool kCanStop = true;
    __device__ bool active(int, const FamilyPlan&) const { return true; }
    // Deferred planes: the planes of plan entries n_eval and beyond are not
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

    // Entries of this lane without a final output yet: `open` ones have no
    // stable p so far; `parked` ones are stable at the p the search started
    // at (or at a larger one on the way up) and a still larger p may be
    // stable too (their S waits in `out`).  With the r = 1 projection the
    // search always starts at the largest p and its parked entries (S_{p*}
    // waiting for S_{p_lo}) count as open.
    __device__ void counts(int& open, int& parked) const {
        constexpr int TOT = WT_M * WT_N * 16;
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
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
                const int tix = i * WT_N + j;
                const int sh = (tix & 1) * 16;
                const uint32_t dec = decided[tix >> 1] >> sh;
                const uint32_t pnd = pending[tix >> 1] >> sh;
#pragma unroll 1
                for (int q = 0; q < 16; ++q) {
                    if ((dec >> q) & 1u) continue;
                    TailEntry te;
                    te.bi = t.bi;
                    te.i = (int32_t)(t.row0 + lr0 + roff_of(i, q));
                    te.j = (int32_t)(t.col0 + lc0 + j * 32);
                    if ((pnd >> q) & 1u) {
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

    __device__ void setup(const TileCtx& t, const GemmGeom& g, uint8_t* lds, int tid) {
        m = g.rows;
        n = g.cols;
        n_eval = MT_MAX_P;
        if (!RERUN && a.low_need != nullptr && __builtin_amdgcn_readfirstlane(*a.low_need) == 0) n_eval = a.n_eval;
        rsc = (int2*)lds;
        csc = rsc + C::BM;
        // Row / column scales of this tile (1 where absent or padding).
        for (int i = tid; i < C::BM + C::BN; i += C::THREADS) {
            double v = 1.0;
            if (i < C::BM) {
                if (a.r && t.row0 + i < m) v = a.r[(int64_t)t.bi * m + t.row0 + i];
            } else {
                const int64_t cc = t.col0 + (i - C::BM);
                if (a.c && cc < n) v = a.c[(int64_t)t.bi * n + cc];
            }
            const ScaleSplit sp = split_scale(v);
            rsc[i] = make_int2(__float_as_int(sp.m), sp.e);
        }
        // Lane l handles the accumulator elements it holds: column l % 32 of
        // each 32 x 32 sub-tile and rows roff_of(i, q) from lr0 (lanes 0-31
        // and 32-63 store two row runs 4 apart).
        lr0 = t.wm * WT_M * 32 + (t.lane >> 5) * 4;
        lc0 = t.wn * WT_N * 32 + (t.lane & 31);
        out_lane = ((int64_t)t.bi * m + t.row0 + lr0) * n + t.col0 + lc0;
        rows_left = (int32_t)min<int64_t>(m - (t.row0 + lr0), 1 << 30);
        cols_left = (int32_t)min<int64_t>(n - (t.col0 + lc0), 1 << 30);
        diag_off = (int32_t)((t.col0 + lc0) - (t.row0 + lr0));
        // Entries outside the matrix count as decided from the start, so a
        // tile whose every entry is decided can be skipped as a whole.
#pragma unroll
        for (int i = 0; i < NDEC; ++i) decided[i] = pending[i] = 0u;
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
                const int tix = i * WT_N + j;
                uint32_t bits = 0u;
#pragma unroll
                for (int q = 0; q < 16; ++q)
                    if (!(j * 32 < cols_left && roff_of(i, q) < rows_left)) bits |= 1u << q;
                decided[tix >> 1] |= bits << ((tix & 1) * 16);
            }
    }

    // Walk the (i, j) sub-tiles of this wave: f(roff, j, S, mask, dec, pnd)
    // sees each entry of this lane straight from its accumulator register
    // (row offset roff from lr0, bit `mask` of the sub-tile's decided /
    // pending words).  A sub-tile whose entries all have a bit of `skip` set
    // is passed over.  Unrolled: the hot path (every entry of a top-down
    // search).
    template <class F>
    __device__ void each_unrolled(f32x16 (&acc)[WT_M][WT_N], float*, int, bool skip_pending, F&& f) {
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
                const int tix = i * WT_N + j;
                uint32_t dec = decided[tix >> 1];
                uint32_t pnd = pending[tix >> 1];
                const int sh = (tix & 1) * 16;
                const uint32_t skip = skip_pending ? (dec | pnd) : dec;
                if (__all(((skip >> sh) & 0xFFFFu) == 0xFFFFu)) continue;
                // the sub-tile's 16 values in a local array that the
                // partly unrolled walk indexes by register (a fully unrolled
                // walk is too large and puts the accumulators in scratch)
                float vals[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) vals[q] = acc[i][j][q];
#pragma unroll 2
                for (int q = 0; q < 16; ++q) f(roff_of(i, q), j, vals[q], 1u << (sh + q), dec, pnd);
                decided[tix >> 1] = dec;
                pending[tix >> 1] = pnd;
            }
    }
    // The same with the sub-tile loop rolled (the per-entry code appears
    // once; the sub-tile is copied to LDS, stg, so that the rolled loop can
    // index it): for the entries of a search that does not start at the
    // largest p, which run once or a few times per tile.
    template <class F>
    __device__ void each_rolled(f32x16 (&acc)[WT_M][WT_N], float* stg, int lane, F&& f) {
#pragma unroll 1
        for (int tix = 0; tix < WT_M * WT_N; ++tix) {
            const int i = tix / WT_N, j = tix % WT_N;
            uint32_t dec = 0, pnd = 0;
#pragma unroll
            for (int w = 0; w < NDEC; ++w)
                if (w == (tix >> 1)) {
                    dec = decided[w];
                    pnd = pending[w];
                }
            const int sh = (tix & 1) * 16;
            if (__all(((dec >> sh) & 0xFFFFu) == 0xFFFFu)) continue;
#pragma unroll
            for (int ii = 0; ii < WT_M; ++ii)
#pragma unroll
                for (int jj = 0; jj < WT_N; ++jj)
                    if (ii * WT_N + jj == tix) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) stg[r * 64 + lane] = acc[ii][jj][r];
                    }
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int q = 0; q < 16; ++q) f(roff_of(i, q), j, stg[q * 64 + lane], 1u << (sh + q), dec, pnd);
#pragma unroll
            for (int w = 0; w < NDEC; ++w)
                if (w == (tix >> 1)) {
                    decided[w] = dec;
                    pending[w] = pnd;
                }
            __builtin_amdgcn_wave_barrier();
        }
    }

    // The walk of the search at its start and going down (every entry of
    // a search passes here: the hot path).  Per sub-tile the decisions are
    // bit masks: `stab` the entries stable at this p, `act` those acted on
    // here (stable, or any at the smallest p, and neither decided nor
    // parked).  At the start (`start`, a search that did not begin at the
    // largest p) an acted-on entry that is stable with S >= rise_thr may be
    // stable at a larger p too: it parks S in `out` (`park`) instead of being
    // decided.  The output of element q is formed when some lane acts on its
    // entry q and stored under the mask, so the lanes do not branch one by
    // one.
    __device__ void down_walk(f32x16 (&acc)[WT_M][WT_N], bool last, float tau_f, float inv_p, bool p_is_1,
                              float corr, uint8_t pcode, TO* out, uint8_t* ps, bool start, float rise_thr) {
        float cm[WT_N];
        int ce[WT_N];
#pragma unroll
        for (int j = 0; j < WT_N; ++j) {
            const int2 cv = csc[lc0 + j * 32];
            cm[j] = __int_as_float(cv.x);
            ce[j] = cv.y;
        }
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
                const int tix = i * WT_N + j;
                const int sh = (tix & 1) * 16;
                const uint32_t busy = ((decided[tix >> 1] | pending[tix >> 1]) >> sh) & 0xFFFFu;
                if (__all(busy == 0xFFFFu)) continue;
                // the sub-tile's values in a local array that the partly
                // unrolled loop below indexes by register
                float vals[16];
                uint32_t stab = 0, rise = 0;
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    vals[q] = acc[i][j][q];
                    stab |= (vals[q] >= tau_f ? 1u : 0u) << q;
                    rise |= (vals[q] >= rise_thr ? 1u : 0u) << q;
                }
                const uint32_t act = (last ? 0xFFFFu : stab) & ~busy;
                if (!__any(act != 0)) continue;
                const uint32_t park = start ? (act & stab & rise) : 0u;
                decided[tix >> 1] |= (act & ~park) << sh;
                pending[tix >> 1] |= park << sh;
#pragma unroll 2
                for (int q = 0; q < 16; ++q) {
                    const bool take = (act >> q) & 1u;
                    if (!__any(take)) continue;
                    const int roff = roff_of(i, q);
                    const int2 rv = rsc[lr0 + roff];
                    const float S = vals[q];
                    const float v = __int_as_float(rv.x) * cm[j] * (p_is_1 ? S : root_f32(S, inv_p)) * corr;
                    TO w = scale_out<TO>(v, rv.y + ce[j]);
                    if (MODE == EPI_APSP_X || a.clamp) w = w < TO(1) ? w : TO(1);
                    if (MODE == EPI_APSP_X && roff - j * 32 == diag_off) w = TO(1);
                    if ((park >> q) & 1u) w = (TO)S;  // parked: S waits in `out`
                    if (take) {
                        const int64_t o = (int64_t)roff * n + j * 32;
                        out[o] = w;
                        if (ps) ps[o] = ((stab >> q) & 1u) ? pcode : (uint8_t)MT_PSTAR_NONE;
                    }
                }
            }
    }

    // Final output of entry (roff, j) from its ring result S at a p with
    // root factor inv_p (p_is_1: no root) and norm correction corr.
    __device__ void put(TO* out, int roff, int j, int64_t o, float S, bool p_is_1, float inv_p, float corr) {
        const int2 rv = rsc[lr0 + roff], cv = csc[lc0 + j * 32];
        const float v = __int_as_float(rv.x) * __int_as_float(cv.x) * (p_is_1 ? S : root_f32(S, inv_p)) * corr;
        TO w = scale_out<TO>(v, rv.y + cv.y);
        if (MODE == EPI_APSP_X || a.clamp) w = w < TO(1) ? w : TO(1);
        if (MODE == EPI_APSP_X && roff - j * 32 == diag_off) w = TO(1);
        out[o] = w;
    }

    // stage: a free pipeline buffer (C::NW staging tiles of STG floats).
    // Plan entry e of a p search that started at plan entry s: entries e >= s
    // go down from the start (smaller p), entries e < s up (larger p).
    __device__ void entry(int e, int s, const FamilyPlan& plan, f32x16 (&acc)[WT_M][WT_N],
                          const TileCtx& t, uint8_t* stage) {
        float* stg = (float*)stage + t.wave * STG;
        const bool last = (e == plan.n - 1);
        const float inv_p = plan.e[e].inv_p;
        const bool p_is_1 = plan.e[e].p == 1;
        const float corr = plan.e[e].corr;
        // S >= tau in FP64 is S >= tau_f in FP32 (tau_f: tau rounded up to FP32)
        const float tau_f = plan.tau_f;
        const uint8_t pcode = (uint8_t)plan.e[e].pidx;
        TO* out = (TO*)a.out + out_lane;
        uint8_t* ps = a.pstar ? a.pstar + out_lane : nullptr;
        const int lane = t.lane;
        if constexpr (R1) {
            // r = 1 projection: an entry stable here, with a smaller p still
            // to come, parks S_{p*} in `out` and is finished at that p with
            // (S_{p*} / S_{p_lo})^(1/(p* - p_lo)) (Sec. 1, one projected value)
            const bool defer = plan.e[e].inv_dp > 0.f;
            const float prev_inv_dp = e > 0 ? plan.e[e - 1].inv_dp : 0.f;
            const float prev_inv_p = e > 0 ? plan.e[e - 1].inv_p : 1.f;
            each_unrolled(acc, stg, lane, false,
                          [&](int roff, int j, float S, uint32_t mask, uint32_t& dec, uint32_t& pnd) {
                              const int64_t o = (int64_t)roff * n + j * 32;
                              const bool stable = S >= tau_f;
                              if (pnd & mask) {
                                  // S here is the ring result at p_lo of an entry parked at p*
                                  const float Sh = (float)out[o];
                                  pnd &= ~mask;
                                  dec |= mask;
                                  if (S > 0.f)
                                      put(out, roff, j, o, Sh / S, false, prev_inv_dp, 1.f);
                                  else
                                      put(out, roff, j, o, Sh, false, prev_inv_p, 1.f);
                              } else if (!(dec & mask) && (stable || last)) {
                                  if (ps) ps[o] = stable ? pcode : (uint8_t)MT_PSTAR_NONE;
                                  if (stable && defer) {
                                      out[o] = (TO)S;
                                      pnd |= mask;
                                  } else {
                                      dec |= mask;
                                      put(out, roff, j, o, S, p_is_1, inv_p, corr);
                                  }
                              }
                          });
        } else if (e > s || s == 0) {
            // going down: decide entries stable here (or at the smallest p);
            // entries parked at the start wait
            down_walk(acc, last, tau_f, inv_p, p_is_1, corr, pcode, out, ps, false, 0.f);
        } else if (e == s) {
            // the start: an entry stable here whose S does not rule out the
            // next larger p (S_q <= S^(q/p)) parks S in `out`
            down_walk(acc, last, tau_f, inv_p, p_is_1, corr, pcode, out, ps, true, plan.e[e].rise_thr_f);
        } else {
            // going up: only parked entries are left, their S from plan
            // entry e + 1 waits in `out`
            const float rise_thr = plan.e[e].rise_thr_f;
            const PlanEntry& pb = plan.e[e + 1];
            const float below_inv_p = pb.inv_p;
            const bool below_p_is_1 = pb.p == 1;
            const float below_corr = pb.corr;
            each_rolled(acc, stg, lane, [&](int roff, int j, float S, uint32_t mask, uint32_t& dec, uint32_t& pnd) {
                if (dec & mask) return;
                const bool stable = S >= tau_f;
                const int64_t o = (int64_t)roff * n + j * 32;
                if (stable) {
                    if (ps) ps[o] = pcode;
                    if (e > 0 && S >= rise_thr) {
                        out[o] = (TO)S;  // stable here too, and maybe above
                        return;
                    }
                }
                pnd &= ~mask;
                dec |= mask;
                if (stable)
                    put(out, roff, j, o, S, p_is_1, inv_p, corr);
                else  // p* is the p below
                    put(out, roff, j, o, (float)out[o], below_p_is_1, below_inv_p, below_corr);
            });
        }
    }

    __device__ void finish(const TileCtx&) {}
};

// ------------------------------------------------------------ adjoint epilogue
// out[bi, row, col] = sum over active p of M'(row, col)^(p-1) * acc_p, where
// M' = M / scale_rows[row] / scale_cols[col] is the scaled input (A' for the
// gradient of A, B' for the gradient of B).
template <class C, typename TM>
struct AdjointEpi {
    static constexpr int WT_M = C::WT_M, WT_N = C::WT_N;
    // inverse mantissas of the row and column scales, then their exponents
    static constexpr int LDS_BYTES = (C::BM + C::BN) * 8;

    using Args = AdjArgs;
    AdjArgs a;
    int64_t rows, cols;
    f32x16 tot[WT_M][WT_N];
    float* rs;
    float* cs;
    int* res;
    int* ces;
    int lr0, lc0;
    int64_t lane_off;
    int32_t rows_left, cols_left;

    static constexpr bool kAllActive = false;
    static constexpr bool kCanStop = false;
    __device__ bool active(int e, const FamilyPlan& plan) const { return a.hist[plan.e[e].pidx] > 0; }
    __device__ int down_end(const FamilyPlan& plan) const { return plan.n; }
    static __device__ bool skip_tile(const Args&, int64_t) { return false; }
    __device__ void record_tile(int64_t, bool) const {}
    __device__ void counts(int& open, int& parked) const { open = parked = 0; }
    __device__ int32_t start_index() const { return 0; }
    __device__ bool can_hand_over(int) const { return false; }
    __device__ uint32_t* tail_counter() const { return nullptr; }
    __device__ void hand_over(uint32_t, int, int, const TileCtx&) const {}

    __device__ void setup(const TileCtx& t, const GemmGeom& g, uint8_t* lds, int tid) {
        rows = g.rows;
        cols = g.cols;
        rs = (float*)lds;
        cs = rs + C::BM;
        res = (int*)(rs + C::BM + C::BN);
        ces = res + C::BM;
        // scale v = m 2^e: M / v is formed as (M 2^-e) / m, so neither a
        // scale outside FP32 nor an FP64 entry beyond it overflows (the
        // scaled value is in [0, 1])
        for (int i = tid; i < C::BM + C::BN; i += C::THREADS) {
            double v = 1.0;
            if (i < C::BM) {
                if (a.scale_rows && t.row0 + i < rows) v = a.scale_rows[(int64_t)t.bi * rows + t.row0 + i];
            } else {
                const int64_t cc = t.col0 + (i - C::BM);
                if (a.scale_cols && cc < cols) v = a.scale_cols[(int64_t)t.bi * cols + cc];
            }
            const ScaleSplit sp = split_scale(v);
            rs[i] = sp.m > 0.f ? 1.f / sp.m : 0.f;
            res[i] = sp.e;
        }
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) tot[i][j] = f32x16{};
        // MFMA output layout: entry (i, j, r) of lane l is tile row
        // wm*WT_M*32 + i*32 + (r/4)*8 + (l/32)*4 + r%4, column wn*WT_N*32 + j*32 + l%32.
        lr0 = t.wm * WT_M * 32 + (t.lane >> 5) * 4;
        lc0 = t.wn * WT_N * 32 + (t.lane & 31);
        lane_off = ((int64_t)t.bi * rows + t.row0 + lr0) * cols + t.col0 + lc0;
        rows_left = (int32_t)min<int64_t>(rows - (t.row0 + lr0), 1 << 30);
        cols_left = (int32_t)min<int64_t>(cols - (t.col0 + lc0), 1 << 30);
    }

    __device__ void entry(int e, int, const FamilyPlan& plan, f32x16 (&acc)[WT_M][WT_N], const TileCtx&,
                          uint8_t*) {
        const int pm1 = plan.e[e].p - 1;
        const TM* src = (const TM*)a.M + lane_off;
        // one sub-tile at a time (a rolled loop keeps one sub-tile's inputs
        // and powers live, not all of them)
#pragma unroll 1
        for (int tix = 0; tix < WT_M * WT_N; ++tix) {
            const int i = tix / WT_N, j = tix % WT_N;
            f32x16 av{};
#pragma unroll
            for (int ii = 0; ii < WT_M; ++ii)
#pragma unroll
                for (int jj = 0; jj < WT_N; ++jj)
                    if (ii * WT_N + jj == tix) av = acc[ii][jj];
            const bool col_ok = j * 32 < cols_left;
            const float cinv = cs[lc0 + j * 32];
            const int cexp = ces[lc0 + j * 32];
            float x[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int roff = i * 32 + (r >> 2) * 8 + (r & 3);
                float v = 0.f;
                if (col_ok && roff < rows_left) {
                    const int ex = -(res[lr0 + roff] + cexp);
                    const TM mv = src[(int64_t)roff * cols + j * 32];
                    if constexpr (sizeof(TM) == 8)
                        v = (float)__builtin_amdgcn_ldexp(mv, ex);
                    else
                        v = __builtin_amdgcn_ldexpf(mv, ex);
                    v = v * rs[lr0 + roff] * cinv;
                }
                x[r] = v;
            }
            // x^(p-1) by binary powering (p uniform); 0^0 = 1
            float pw[16];
#pragma unroll
            for (int r = 0; r < 16; ++r) pw[r] = 1.f;
            for (int ex = pm1; ex; ex >>= 1) {
                if (ex & 1) {
#pragma unroll
                    for (int r = 0; r < 16; ++r) pw[r] *= x[r];
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) x[r] *= x[r];
            }
#pragma unroll
            for (int ii = 0; ii < WT_M; ++ii)
#pragma unroll
                for (int jj = 0; jj < WT_N; ++jj)
                    if (ii * WT_N + jj == tix) {
#pragma unroll
                        for (int r = 0; r < 16; ++r) tot[ii][jj][r] += pw[r] * av[r];
                    }
        }
    }

    __device__ void finish(const TileCtx& t) {
        // the adjoint planes carry the scales divided by 2^post (per batch item)
        const int post = a.post_exp ? a.post_exp[t.bi] : 0;
        const bool mul = a.out_row_mul || a.out_col_mul;
        const int64_t row_base = (int64_t)t.bi * rows + t.row0 + lr0;
        const int64_t col_base = (int64_t)t.bi * cols + t.col0 + lc0;
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
                if (!(j * 32 < cols_left)) continue;
                const double cm = a.out_col_mul ? a.out_col_mul[col_base + j * 32] : 1.0;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int roff = i * 32 + (r >> 2) * 8 + (r & 3);
                    if (roff < rows_left) {
                        const int64_t o = lane_off + (int64_t)roff * cols + j * 32;
                        if (mul) {
                            // chain factors of a balanced forward, in FP64
                            const double rm = a.out_row_mul ? a.out_row_mul[row_base + roff] : 1.0;
                            const double w = __builtin_amdgcn_ldexp((double)tot[i][j][r] * rm * cm, post);
                            if (a.out_f64)
                                ((double*)a.out)[o] = w;
                            else
                                ((float*)a.out)[o] = (float)w;
                        } else if (a.out_f64) {
                            ((double*)a.out)[o] = scale_out<double>(tot[i][j][r], post);
                        } else {
                            ((float*)a.out)[o] = scale_out<float>(tot[i][j][r], post);
                        }
                    }
                }
            }
    }
};

// ------------------------------------------------------------ the main loop
template <class C, class Epi>
__global__ __launch_bounds__(C::THREADS, C::MINW) void mt_pfamily_gemm_bf16_kernel(GemmGeom g,
                                                                            FamilyPlan plan,
                                                                            typename Epi::Args args) {
    constexpr int WT_M = C::WT_M, WT_N = C::WT_N;
    extern __shared__ __attribute__((aligned(1024))) uint8_t smem[];
    __shared__ int s_act[MT_MAX_P + 1];
    __shared__ int s_done[2][C::NW];  // per wave: undecided entries (entry parity)
    __shared__ int s_open[2][C::NW];  // per wave: of which open (entry parity)
    __shared__ uint32_t s_tail_base;

    const int tid = threadIdx.x;
    if (g.work && tid == 0) timing_span_begin(g.work);
    TileCtx t;
    t.lane = tid & 63;
    t.wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    t.wm = t.wave / C::WN;
    t.wn = t.wave % C::WN;
    const int lane = t.lane;
    const int wave = t.wave;

    // Workgroup -> tile.  Consecutive workgroup ids are spread over the 8
    // XCDs; regroup so each XCD owns a contiguous run of tiles, then walk the
    // run in bands of 4 tile rows so concurrently resident tiles share X rows
    // and Y rows in that XCD's L2 (bands of 4 measured 1.2 % faster than 8
    // at 8192^2).
    int id = blockIdx.x;
    const int nwg = gridDim.x;
    if ((nwg & 7) == 0) id = (id & 7) * (nwg >> 3) + (id >> 3);
    const int per_batch = g.tiles_m * g.tiles_n;
    t.bi = id / per_batch;
    const int tt = id - t.bi * per_batch;
    constexpr int GROUP = 4;
    const int group = tt / (GROUP * g.tiles_n);
    const int first_m = group * GROUP;
    const int gsz = min(GROUP, g.tiles_m - first_m);
    const int in_g = tt - group * GROUP * g.tiles_n;
    const int tm = first_m + in_g % gsz;
    const int tn = in_g / gsz;
    t.row0 = (int64_t)tm * C::BM;
    t.col0 = (int64_t)tn * C::BN;
    const int64_t tile_id = (int64_t)t.bi * per_batch + (int64_t)tm * g.tiles_n + tn;
    if (Epi::skip_tile(args, tile_id)) return;

    Epi epi;
    epi.a = args;
    epi.setup(t, g, smem + C::PIPE_BYTES, tid);
    if (!Epi::kAllActive && tid == 0) {
        int na = 0;
        for (int e = 0; e < plan.n; ++e)
            if (epi.active(e, plan)) s_act[1 + na++] = e;
        s_act[0] = na;
    }

    const uint16_t* Xbase = g.X + (int64_t)t.bi * g.x_batch_elems + t.row0 * g.kp;
    const uint16_t* Ybase = g.Y + (int64_t)t.bi * g.y_batch_elems + t.col0 * g.kp;

    // Global source offsets of the direct-to-LDS loads.  Plain step: load
    // instruction i of this wave fills LDS rows R0 .. R0+7, R0 = (wave * G +
    // i) * 8 with G (even) row groups per wave; lane l fills row R0 + l/8,
    // physical chunk l%8, which holds logical chunk (l%8) ^ swz(row).  For
    // even G the swizzle is (i&1)*4 + l/16, so two lane offsets cover every
    // instruction.  Split step: instruction i fills 64-byte rows R0 .. R0+15,
    // R0 a multiple of 16; lane l fills row R0 + l/4, physical chunk l%4,
    // holding logical chunk (l%4) ^ ((row >> 2) & 3) = (l%4) ^ ((l >> 4) & 3).
    // As byte offsets from the plane row block of the step (X and Y load the
    // same row pattern: GA == GB, SA == SB), 32-bit so that each load is a
    // uniform base plus one VGPR (kp < 2^22 keeps them in range).
    static_assert(C::GA == C::GB && C::SA == C::SB, "X and Y share the load offsets");
    const uint32_t kpb = (uint32_t)g.kp * 2u;
    const uint32_t ld_even = (lane >> 3) * kpb + (((lane & 7) ^ (lane >> 4)) * 16);
    const uint32_t ld_odd = (lane >> 3) * kpb + (((lane & 7) ^ (4 + (lane >> 4))) * 16);
    const uint32_t ld_split = (lane >> 2) * kpb + (((lane & 3) ^ ((lane >> 4) & 3)) * 16);
    uint32_t voff_p[C::GA], voff_s[C::SA];
#pragma unroll
    for (int i = 0; i < C::GA; ++i) voff_p[i] = (uint32_t)((wave * C::GA + i) * 8) * kpb + ((i & 1) ? ld_odd : ld_even);
#pragma unroll
    for (int i = 0; i < C::SA; ++i) voff_s[i] = (uint32_t)((wave * C::SA + i) * 16) * kpb + ld_split;
    // LDS operand reads: row (lane & 31) of a 32-row block, logical chunk
    // 2*kk + lane/32; plain swizzle (lane >> 1) & 7, split swizzle
    // (lane >> 2) & 3 (block bases are multiples of 32 rows).
    const int32_t rd_base = (lane & 31) * 128 + (((lane >> 5) ^ ((lane >> 1) & 7)) * 16);
    const int32_t rd_split = (lane & 31) * 64 + (((lane >> 5) ^ ((lane >> 2) & 3)) * 16);

    __syncthreads();
    // (deferred planes: the way down ends above them, plan entry e_end)
    const int e_end = epi.down_end(plan);
    const int nact = Epi::kAllActive ? e_end : __builtin_amdgcn_readfirstlane(s_act[0]);
    // The p search starts at plan entry s (0: the largest p), goes down to
    // the smallest p and then up from s - 1 to the largest (forward only).
    int s0 = Epi::kAllActive ? __builtin_amdgcn_readfirstlane(epi.start_index()) : 0;
    const int s = s0 < 0 ? 0 : (s0 >= nact ? nact - 1 : s0);

    // plan entry of processing index ai
    auto entry_of = [&](int ai) -> int {
        if (!Epi::kAllActive) return __builtin_amdgcn_readfirstlane(s_act[1 + ai]);
        return ai < nact - s ? s + ai : nact - 1 - ai;
    };
    const int nkt64 = (int)(g.kp / 64);  // plain steps per entry
    const int nkt32 = 2 * nkt64;          // split steps per entry
    // The next K step to load: processing index la_, step lkt of its entry,
    // and that entry's plane rows (A hi, A lo, B hi, B lo; the lo rows are
    // unused for a plain p), set once per entry.
    int la_ = 0, lkt = 0, lnk = 0;
    bool lsplit = false;
    const uint16_t *lxh = Xbase, *lxl = Xbase, *lyh = Ybase, *lyl = Ybase;
    auto set_cursor = [&]() {
        if (la_ >= nact) return;
        const PlanEntry& pe = plan.e[entry_of(la_)];
        lsplit = pe.nseg == 3;
        lnk = lsplit ? nkt32 : nkt64;
        lxh = Xbase + (int64_t)pe.a_plane[0] * g.x_plane_elems;
        lxl = Xbase + (int64_t)pe.a_plane[2] * g.x_plane_elems;
        lyh = Ybase + (int64_t)pe.b_plane[0] * g.y_plane_elems;
        lyl = Ybase + (int64_t)pe.b_plane[1] * g.y_plane_elems;
    };
    auto issue = [&](int buf) {
        uint8_t* la = smem + buf * C::BUF_BYTES;
        if (lsplit) {
            const char* xh = (const char*)lxh + lkt * 64;
            const char* xl = (const char*)lxl + lkt * 64;
            const char* yh = (const char*)lyh + lkt * 64;
            const char* yl = (const char*)lyl + lkt * 64;
            uint8_t* lxl_ = la + C::BM * 64;
            uint8_t* lyh_ = la + C::A_BYTES;
            uint8_t* lyl_ = lyh_ + C::BN * 64;
#pragma unroll
            for (int i = 0; i < C::SA; ++i) {
                const int R0 = (wave * C::SA + i) * 16;
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(xh + voff_s[i]), (lds_void*)(la + R0 * 64), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(xl + voff_s[i]), (lds_void*)(lxl_ + R0 * 64), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(yh + voff_s[i]), (lds_void*)(lyh_ + R0 * 64), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(yl + voff_s[i]), (lds_void*)(lyl_ + R0 * 64), 16, 0, 0);
            }
        } else {
            const char* xsrc = (const char*)lxh + lkt * 128;
            const char* ysrc = (const char*)lyh + lkt * 128;
            uint8_t* lb = la + C::A_BYTES;
#pragma unroll
            for (int i = 0; i < C::GA; ++i) {
                const int R0 = (wave * C::GA + i) * 8;
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(xsrc + voff_p[i]), (lds_void*)(la + R0 * 128), 16, 0, 0);
                __builtin_amdgcn_global_load_lds((glb_cvoid*)(ysrc + voff_p[i]), (lds_void*)(lb + R0 * 128), 16, 0, 0);
            }
        }
    };
    auto advance = [&]() {
        if (++lkt == lnk) {
            lkt = 0;
            ++la_;
            set_cursor();
        }
    };

    // Software pipeline: the loads of the next K step (possibly of the next
    // family entry) are issued before the MFMAs of the current one.
    set_cursor();
    if (nkt64 > 0 && nact > 0) {
        issue(0);
        advance();
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    int buf = 0;
    int64_t kunits = 0;  // executed MFMA work in units of BM x BN x 1 products
    if (tid == 0) epi.record_tile(tile_id, false);
    for (int ai = 0; ai < nact; ++ai) {
        const int e = entry_of(ai);
        f32x16 acc[WT_M][WT_N];
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) acc[i][j] = f32x16{};

        if (plan.e[e].nseg == 3) {
            // split p: hi.hi + hi.lo + lo.hi per K step of 32
            for (int st = 0; st < nkt32; ++st) {
                if (la_ < nact) {
                    issue(buf ^ 1);
                    advance();
                }
                const uint8_t* pxh = smem + buf * C::BUF_BYTES + t.wm * WT_M * 32 * 64;
                const uint8_t* pxl = pxh + C::BM * 64;
                const uint8_t* pyh = smem + buf * C::BUF_BYTES + C::A_BYTES + t.wn * WT_N * 32 * 64;
                const uint8_t* pyl = pyh + C::BN * 64;
                __builtin_amdgcn_s_setprio(1);
#pragma unroll
                for (int kk = 0; kk < 2; ++kk) {
                    const int32_t ro = rd_split ^ (kk << 5);
                    bf16x8 ah[WT_M], al[WT_M], bh[WT_N], bl[WT_N];
#pragma unroll
                    for (int i = 0; i < WT_M; ++i) ah[i] = *(const bf16x8*)(pxh + i * 32 * 64 + ro);
#pragma unroll
                    for (int j = 0; j < WT_N; ++j) bh[j] = *(const bf16x8*)(pyh + j * 32 * 64 + ro);
#pragma unroll
                    for (int j = 0; j < WT_N; ++j) bl[j] = *(const bf16x8*)(pyl + j * 32 * 64 + ro);
#pragma unroll
                    for (int i = 0; i < WT_M; ++i) al[i] = *(const bf16x8*)(pxl + i * 32 * 64 + ro);
#pragma unroll
                    for (int i = 0; i < WT_M; ++i)
#pragma unroll
                        for (int j = 0; j < WT_N; ++j) {
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
                        }
#pragma unroll
                    for (int i = 0; i < WT_M; ++i)
#pragma unroll
                        for (int j = 0; j < WT_N; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
                }
                __builtin_amdgcn_iglp_opt(1);
                __builtin_amdgcn_s_setprio(0);
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                buf ^= 1;
            }
            kunits += (int64_t)nkt32 * 96;
        } else {
            for (int st = 0; st < nkt64; ++st) {
                if (la_ < nact) {
                    issue(buf ^ 1);
                    advance();
                }
                const uint8_t* pa = smem + buf * C::BUF_BYTES + t.wm * WT_M * 32 * 128;
                const uint8_t* pb = smem + buf * C::BUF_BYTES + C::A_BYTES + t.wn * WT_N * 32 * 128;
                // MFMA issue runs at raised wave priority; the fragments of
                // sub-step kk + 1 are read from LDS while kk's MFMAs run.
                __builtin_amdgcn_s_setprio(1);
                bf16x8 fa[2][WT_M], fb[2][WT_N];
#pragma unroll
                for (int i = 0; i < WT_M; ++i) fa[0][i] = *(const bf16x8*)(pa + i * 32 * 128 + rd_base);
#pragma unroll
                for (int j = 0; j < WT_N; ++j) fb[0][j] = *(const bf16x8*)(pb + j * 32 * 128 + rd_base);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    const int cur = kk & 1;
                    if (kk + 1 < 4) {
                        const int32_t ro = rd_base ^ ((kk + 1) << 5);
#pragma unroll
                        for (int i = 0; i < WT_M; ++i) fa[cur ^ 1][i] = *(const bf16x8*)(pa + i * 32 * 128 + ro);
#pragma unroll
                        for (int j = 0; j < WT_N; ++j) fb[cur ^ 1][j] = *(const bf16x8*)(pb + j * 32 * 128 + ro);
                    }
#pragma unroll
                    for (int i = 0; i < WT_M; ++i)
#pragma unroll
                        for (int j = 0; j < WT_N; ++j)
                            acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa[cur][i], fb[cur][j], acc[i][j], 0, 0, 0);
                }
                // let the scheduler interleave the LDS operand reads with
                // the MFMAs (LLVM's single-wave small-GEMM strategy; -6 %
                // time on the 8192^2 forward)
                __builtin_amdgcn_iglp_opt(1);
                __builtin_amdgcn_s_setprio(0);
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                __syncthreads();
                buf ^= 1;
            }
            kunits += (int64_t)nkt64 * 64;
        }
        // the buffer the last step read is free until the next step's loads,
        // which wait for the barrier below
        epi.entry(e, s, plan, acc, t, smem + (buf ^ 1) * C::BUF_BYTES);
        int lane_pre = 0;
        if (Epi::kCanStop) {
            // undecided entries per lane -> exclusive prefix in the wave
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
            for (int w = 0; w < C::NW; ++w) {
                const int x = s_done[ai & 1][w];
                total += x;
                open += s_open[ai & 1][w];
                wave_pre += w < wave ? x : 0;
            }
            total = __builtin_amdgcn_readfirstlane(total);
            open = __builtin_amdgcn_readfirstlane(open);
            // Every entry of the tile has its p: the remaining p cannot
            // change the output.  The loads already issued for the next entry
            // have landed (vmcnt(0) above) and are simply unused.
            if (total == 0) break;
            // Only a few are left: hand them to the sparse tail, which runs
            // the remaining p for them alone, and stop the tile.
            if (ai + 1 < nact && epi.can_hand_over(total)) {
                if (tid == 0) s_tail_base = atomicAdd(epi.tail_counter(), (uint32_t)total);
                __syncthreads();
                epi.hand_over(s_tail_base + (uint32_t)(wave_pre + lane_pre), e, s, t);
                break;
            }
            // deferred planes: entries still open after the way down (which
            // ends above the deferred p) and not handed to the tail need
            // those p; the tile runs again once their planes are written
            // (what it stores meanwhile is overwritten then)
            if (e_end < plan.n && e == e_end - 1 && open > 0 && tid == 0) epi.record_tile(tile_id, true);
            // Going down with nothing open left: only the entries parked at
            // the start wait, for larger p.  Skip to the way up (plan entry
            // s - 1): reload its first K step in place of the prefetched one.
            if (open == 0 && e >= s && s > 0 && ai + 1 < nact - s) {
                ai = nact - s - 1;  // ++ai below -> first entry of the way up
                la_ = nact - s;
                lkt = 0;
                set_cursor();
                if (nkt64 > 0) {
                    issue(buf);
                    advance();
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
            atomicAdd(g.work, (unsigned long long)kunits * (2ull * C::BM * C::BN));
            timing_span_end(g.work);
        }
    }
}

// ------------------------------------------------------------ the sparse tail
// One wave per handed-over entry (TailEntry): for the plan entries from
// e_next on it forms S_p = sum_k A'_ik^p B'_kj^p as a dot product of the
// entry's X and Y plane rows (split p: hi.hi + hi.lo + lo.hi, FP32
// accumulation, the same BF16 operands the GEMM reads) and applies the same
// selection as the GEMM epilogue.  The list length is read on the device;
// the grid is a fixed set of waves that stride over it.
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// S_p of up to G entries of one row at once (act: which take part): each
// chunk of the row's X plane is loaded once for all of them.  Lane l sums the
// 8-element chunks l, l + 64, ... in order, as tail_dot_bf16 does.
// SQ (an unsplit p only): S2 gets the sum of the squared terms, S_2p formed
// from the planes of p, for an entry that rises from p to 2p.
template <int G, bool SQ = false>
__device__ void tail_dot_group_bf16(const uint16_t* xr, const uint16_t* const (&yr)[G], const bool (&act)[G],
                                    const PlanEntry& pe, const GemmGeom& g, int lane, float (&S)[G],
                                    float (&S2)[G]) {
    float acc[G], acc2[G];
#pragma unroll
    for (int q = 0; q < G; ++q) acc[q] = acc2[q] = 0.f;
    if (pe.nseg == 3) {
        const uint16_t* xh = xr + (int64_t)pe.a_plane[0] * g.x_plane_elems;
        const uint16_t* xl = xr + (int64_t)pe.a_plane[2] * g.x_plane_elems;
        const int64_t oyh = (int64_t)pe.b_plane[0] * g.y_plane_elems;
        const int64_t oyl = (int64_t)pe.b_plane[1] * g.y_plane_elems;
        for (int64_t k0 = lane * 8; k0 < g.kp; k0 += 512) {
            const u32x4 vxh = *(const u32x4*)(xh + k0), vxl = *(const u32x4*)(xl + k0);
            u32x4 vyh[G], vyl[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (act[q]) {
                    vyh[q] = *(const u32x4*)(yr[q] + oyh + k0);
                    vyl[q] = *(const u32x4*)(yr[q] + oyl + k0);
                }
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (act[q]) {
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        acc[q] += bf16_lo(vxh[h]) * bf16_lo(vyh[q][h]);
                        acc[q] += bf16_lo(vxh[h]) * bf16_lo(vyl[q][h]);
                        acc[q] += bf16_lo(vxl[h]) * bf16_lo(vyh[q][h]);
                        acc[q] += bf16_hi(vxh[h]) * bf16_hi(vyh[q][h]);
                        acc[q] += bf16_hi(vxh[h]) * bf16_hi(vyl[q][h]);
                        acc[q] += bf16_hi(vxl[h]) * bf16_hi(vyh[q][h]);
                    }
                }
        }
    } else {
        const uint16_t* xp = xr + (int64_t)pe.a_plane[0] * g.x_plane_elems;
        const int64_t oy = (int64_t)pe.b_plane[0] * g.y_plane_elems;
        for (int64_t k0 = lane * 8; k0 < g.kp; k0 += 512) {
            const u32x4 vx = *(const u32x4*)(xp + k0);
            u32x4 vy[G];
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (act[q]) vy[q] = *(const u32x4*)(yr[q] + oy + k0);
#pragma unroll
            for (int q = 0; q < G; ++q)
                if (act[q]) {
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        const float x0 = bf16_lo(vx[h]), y0 = bf16_lo(vy[q][h]);
                        const float x1 = bf16_hi(vx[h]), y1 = bf16_hi(vy[q][h]);
                        acc[q] = __builtin_fmaf(x0, y0, acc[q]);
                        acc[q] = __builtin_fmaf(x1, y1, acc[q]);
                        if (SQ) {
                            // the term of the doubled power: the square of
                            // this term (a BF16 x BF16 product is exact in FP32)
                            const float t0 = x0 * y0, t1 = x1 * y1;
                            acc2[q] = __builtin_fmaf(t0, t0, acc2[q]);
                            acc2[q] = __builtin_fmaf(t1, t1, acc2[q]);
                        }
                    }
                }
        }
    }
#pragma unroll
    for (int q = 0; q < G; ++q) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) acc[q] += __shfl_xor(acc[q], d);
        S[q] = acc[q];
        if (SQ) {
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) acc2[q] += __shfl_xor(acc2[q], d);
            S2[q] = acc2[q];
        }
    }
}

// Entries of one row with the same state are taken in groups of up to
// kTailGroup, which share the row's X plane loads.
constexpr int kTailGroup = 4;

template <int MODE, typename TO, bool R1>
__global__ __launch_bounds__(256) void mt_tail_bf16_kernel(GemmGeom g, FamilyPlan plan, EpiArgs a) {
    constexpr int G = kTailGroup;
    const int lane = threadIdx.x & 63;
    const uint32_t count = __builtin_amdgcn_readfirstlane(*a.tail_count);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    // each wave takes a contiguous run of the list, which is sorted by row
    // (and state within a row)
    const int64_t run = ((int64_t)count + waves - 1) / waves;
    const int64_t w0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)) * run;
    const int64_t w1 = min<int64_t>(w0 + run, (int64_t)count);
    TO* out = (TO*)a.out;
    const float tau_f = plan.tau_f;
    // deferred planes not written: an entry that reaches them marks its tile
    // for the rerun launch instead
    int n_eval = MT_MAX_P;
    if (a.low_need != nullptr && __builtin_amdgcn_readfirstlane(*a.low_need) == 0) n_eval = a.n_eval;
    for (int64_t w = w0; w < w1;) {
        TailEntry te[G];
        te[0] = a.tail_sorted[w];
        int gn = 1;
        while (gn < G && w + gn < w1) {
            const TailEntry t = a.tail_sorted[w + gn];
            if (t.bi != te[0].bi || t.i != te[0].i || t.state != te[0].state) break;
            te[gn++] = t;
        }
        w += gn;
        const int16_t state = te[0].state;
        const uint16_t* xr = g.X + (int64_t)te[0].bi * g.x_batch_elems + (int64_t)te[0].i * g.kp;
        const ScaleSplit r_i = split_scale(a.r ? a.r[(int64_t)te[0].bi * g.rows + te[0].i] : 1.0);
        const uint16_t* yr[G];
        int64_t o[G];
        float Sh[G], S[G];
        int e_first[G];
        bool live[G], act[G];
#pragma unroll
        for (int q = 0; q < G; ++q) {
            live[q] = q < gn;
            const TailEntry& t = te[q < gn ? q : 0];
            yr[q] = g.Y + (int64_t)t.bi * g.y_batch_elems + (int64_t)t.j * g.kp;
            o[q] = ((int64_t)t.bi * g.rows + t.i) * g.cols + t.j;
            e_first[q] = t.e_next;
            Sh[q] = (live[q] && state != kTailOpen) ? (float)out[o[q]] : 0.f;
        }
        // final value of entry q: the scales, clamp and APSP diagonal
        auto put = [&](int q, float v) {
            const ScaleSplit c_j = split_scale(a.c ? a.c[(int64_t)te[q].bi * g.cols + te[q].j] : 1.0);
            TO w = scale_out<TO>(v * r_i.m * c_j.m, r_i.e + c_j.e);
            if (MODE == EPI_APSP_X || a.clamp) w = w < TO(1) ? w : TO(1);
            if (MODE == EPI_APSP_X && te[q].i == te[q].j) w = TO(1);
            if (lane == 0) out[o[q]] = w;
            live[q] = false;
        };
        if (!R1 && state == kTailRise) {
            // stable at e_next + 1 (S parked): go up while a larger p may be
            // stable too.  Where the next larger p doubles this one (both
            // unsplit), its S comes from the same plane rows, each term
            // squared: one pass decides both, and the planes of the larger p
            // are not read.  nxt: the plan entry each entry runs next.
            int e = e_first[0];
            int nxt[G];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                nxt[q] = e_first[q];
                if (live[q] && e_first[q] > e) e = e_first[q];
            }
            for (; e >= 0; --e) {
                bool any_live = false, any_act = false;
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    act[q] = live[q] && e == nxt[q];
                    any_live |= live[q];
                    any_act |= act[q];
                }
                if (!any_live) break;
                if (!any_act) continue;
                const PlanEntry& pe = plan.e[e];
                const bool paired = e > 0 && pe.nseg == 1 && plan.e[e - 1].nseg == 1 && plan.e[e - 1].p == 2 * pe.p;
                float S2[G];
                if (paired)
                    tail_dot_group_bf16<G, true>(xr, yr, act, pe, g, lane, S, S2);
                else
                    tail_dot_group_bf16<G, false>(xr, yr, act, pe, g, lane, S, S2);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (!act[q]) continue;
                    const bool stable = S[q] >= tau_f;
                    if (stable && lane == 0 && a.pstar) a.pstar[o[q]] = (uint8_t)pe.pidx;
                    if (stable && e > 0 && S[q] >= pe.rise_thr_f) {
                        if (!paired) {
                            Sh[q] = S[q];
                            nxt[q] = e - 1;
                            continue;
                        }
                        // the doubled p, plan entry e - 1, from the squared terms
                        const PlanEntry& pu = plan.e[e - 1];
                        const bool stable_u = S2[q] >= tau_f;
                        if (stable_u && lane == 0 && a.pstar) a.pstar[o[q]] = (uint8_t)pu.pidx;
                        if (stable_u && e - 1 > 0 && S2[q] >= pu.rise_thr_f) {
                            Sh[q] = S2[q];
                            nxt[q] = e - 2;
                            continue;
                        }
                        if (stable_u)
                            put(q, root_f32(S2[q], pu.inv_p) * pu.corr);
                        else
                            put(q, (pe.p == 1 ? S[q] : root_f32(S[q], pe.inv_p)) * pe.corr);
                        continue;
                    }
                    if (stable) {
                        put(q, (pe.p == 1 ? S[q] : root_f32(S[q], pe.inv_p)) * pe.corr);
                    } else {
                        const PlanEntry& pb = plan.e[e + 1];
                        put(q, (pb.p == 1 ? Sh[q] : root_f32(Sh[q], pb.inv_p)) * pb.corr);
                    }
                }
            }
        } else {
            // going down from e_next (r = 1: an entry parked at p* finishes
            // at the next smaller p)
            bool pend[G];
            int e = e_first[0];
#pragma unroll
            for (int q = 0; q < G; ++q) {
                pend[q] = R1 && state == kTailR1;
                if (live[q] && e_first[q] < e) e = e_first[q];
            }
            for (; e < plan.n; ++e) {
                bool any_live = false, any_act = false;
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    act[q] = live[q] && e >= e_first[q];
                    any_live |= live[q];
                    any_act |= act[q];
                }
                if (!any_live) break;
                if (e >= n_eval) {
#pragma unroll
                    for (int q = 0; q < G; ++q)
                        if (live[q] && lane == 0) {
                            const int64_t tile = ((int64_t)te[q].bi * g.tiles_m + te[q].i / kBf16BM) * g.tiles_n +
                                                 te[q].j / kBf16BN;
                            a.missed_tile[tile] = 1u;
                            *a.low_missed = 1;
                        }
                    break;
                }
                if (!any_act) continue;
                const PlanEntry& pe = plan.e[e];
                float S2[G];
                tail_dot_group_bf16<G, false>(xr, yr, act, pe, g, lane, S, S2);
#pragma unroll
                for (int q = 0; q < G; ++q) {
                    if (!act[q]) continue;
                    if (R1 && pend[q]) {
                        put(q, S[q] > 0.f ? root_f32(Sh[q] / S[q], plan.e[e - 1].inv_dp)
                                          : root_f32(Sh[q], plan.e[e - 1].inv_p));
                        continue;
                    }
                    const bool stable = S[q] >= tau_f;
                    if (!(stable || e == plan.n - 1)) continue;
                    if (lane == 0 && a.pstar) a.pstar[o[q]] = stable ? (uint8_t)pe.pidx : (uint8_t)MT_PSTAR_NONE;
                    if (R1 && stable && pe.inv_dp > 0.f) {
                        Sh[q] = S[q];
                        pend[q] = true;
                        continue;
                    }
                    put(q, (pe.p == 1 ? S[q] : root_f32(S[q], pe.inv_p)) * pe.corr);
                }
            }
        }
    }
}

template <int MODE, typename TO, bool R1>
hipError_t launch_tail(const GemmGeom& g, const FamilyPlan& plan, const EpiArgs& epi, int64_t cap,
                       hipStream_t st) {
    hipError_t e = launch_tail_sort(epi, g.rows, cap, st);
    if (e != hipSuccess) return e;
    int64_t blocks = (cap + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    timing_before("mt_tail_bf16", st);
    hipLaunchKernelGGL((mt_tail_bf16_kernel<MODE, TO, R1>), dim3((unsigned)blocks), dim3(256), 0, st, g, plan, epi);
    timing_after(st);
    return hipGetLastError();
}

template <class C, class Epi>
hipError_t launch_gemm(const GemmGeom& g, int64_t b, const FamilyPlan& plan,
                       const typename Epi::Args& args, const char* name, hipStream_t st) {
    const int lds = C::PIPE_BYTES + Epi::LDS_BYTES;
    auto kern = mt_pfamily_gemm_bf16_kernel<C, Epi>;
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
    GemmGeom gw = g;
    gw.work = timing_work_slot();
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(C::THREADS), lds, st, gw, plan, args);
    timing_after(st);
    return hipGetLastError();
}

// Forward: 8 waves (2 per SIMD) in 2 x 4, each 128 x 64 -> 256 x 256 tiles.
using FwdCfg = Cfg<2, 4, 4, 2>;
// Adjoint: 8 waves in 2 x 4, each 64 x 32 -> 128 x 128 tiles, held to 128
// registers (4 waves per SIMD) so that two workgroups share a CU and one's
// loads and barriers overlap the other's MFMAs (the batched 512^3 products
// have short K loops); the accumulator plus running sum fit that budget with
// the epilogue walking one sub-tile at a time.
using AdjCfg = Cfg<2, 4, 2, 1, 4>;
static_assert(FwdCfg::BM == kBf16BM && FwdCfg::BN == kBf16BN, "forward tile");
static_assert(AdjCfg::BM == kAdjBM && AdjCfg::BN == kAdjBM, "adjoint tile");

GemmGeom make_geom(const uint16_t* X, const uint16_t* Y, int64_t rows, int64_t cols,
                   int64_t rows_pad, int64_t cols_pad, int64_t kp, int32_t x_planes,
                   int32_t y_planes, int bm, int bn) {
    GemmGeom g;
    g.rows = rows;
    g.cols = cols;
    g.X = X;
    g.Y = Y;
    g.x_plane_elems = rows_pad * kp;
    g.y_plane_elems = cols_pad * kp;
    g.x_batch_elems = g.x_plane_elems * x_planes;
    g.y_batch_elems = g.y_plane_elems * y_planes;
    g.kp = kp;
    g.tiles_m = (int32_t)(rows_pad / bm);
    g.tiles_n = (int32_t)(cols_pad / bn);
    g.work = nullptr;
    return g;
}

}  // namespace

hipError_t launch_pfamily_gemm_bf16(const uint16_t* Ap, const uint16_t* Bp, int64_t b, int64_t m,
                                    int64_t n, int64_t mp, int64_t np, int64_t kp,
                                    int32_t n_planes, const FamilyPlan& plan, const EpiArgs& epi,
                                    hipStream_t st) {
    const GemmGeom g = make_geom(Ap, Bp, m, n, mp, np, kp, n_planes, n_planes, kBf16BM, kBf16BN);
    const char* name = "mt_pfamily_gemm_bf16";
    using CF = FwdCfg;
    // the GEMM, then (when a tail list is given) the sparse tail for the
    // entries the tiles handed over
    const int64_t cap = (int64_t)epi.tail_max * b * g.tiles_m * g.tiles_n;
#define MT_SEL(MODE, TO, R1)                                                                     \
    {                                                                                            \
        hipError_t e = launch_gemm<CF, SelectEpi<CF, MODE, TO, R1>>(g, b, plan, epi, name, st);  \
        if (e == hipSuccess && epi.tail) e = launch_tail<MODE, TO, R1>(g, plan, epi, cap, st);   \
        return e;                                                                                \
    }
#define MT_SEL2(MODE, TO) \
    if (plan.r1) MT_SEL(MODE, TO, true) else MT_SEL(MODE, TO, false)
    if (epi.mode == EPI_APSP_X) {
        if (epi.out_f64) MT_SEL2(EPI_APSP_X, double) else MT_SEL2(EPI_APSP_X, float)
    }
    if (epi.low_need != nullptr) {
        // deferred planes (plain products, no r = 1 projection)
        if (plan.r1 || epi.mode != EPI_PLAIN || !epi.tail) return hipErrorInvalidValue;
        if (epi.out_f64) MT_SEL(EPI_PLAIN, double, false) else MT_SEL(EPI_PLAIN, float, false)
    }
    if (epi.out_f64) MT_SEL2(EPI_PLAIN, double) else MT_SEL2(EPI_PLAIN, float)
#undef MT_SEL2
#undef MT_SEL
}

hipError_t launch_rerun_gemm_bf16(const uint16_t* Ap, const uint16_t* Bp, int64_t b, int64_t m, int64_t n,
                                  int64_t mp, int64_t np, int64_t kp, int32_t n_planes, const FamilyPlan& plan,
                                  const EpiArgs& epi, hipStream_t st) {
    if (epi.missed_tile == nullptr || plan.r1 || epi.mode != EPI_PLAIN) return hipErrorInvalidValue;
    const GemmGeom g = make_geom(Ap, Bp, m, n, mp, np, kp, n_planes, n_planes, kBf16BM, kBf16BN);
    // a launch of its own name: the forward GEMM's timing and work stay apart
    // (a tile that is not marked adds no work and ends no span)
    if (epi.out_f64)
        return launch_gemm<FwdCfg, SelectEpi<FwdCfg, EPI_PLAIN, double, false, true>>(g, b, plan, epi,
                                                                                      "mt_rerun_gemm_bf16", st);
    return launch_gemm<FwdCfg, SelectEpi<FwdCfg, EPI_PLAIN, float, false, true>>(g, b, plan, epi,
                                                                                "mt_rerun_gemm_bf16", st);
}

hipError_t launch_adjoint_gemm_bf16(const uint16_t* Xp, const uint16_t* Yp, int64_t b, int64_t rows,
                                    int64_t cols, int64_t rows_pad, int64_t cols_pad, int64_t kp,
                                    int32_t x_planes, int32_t y_planes, const FamilyPlan& plan,
                                    const AdjArgs& adj, hipStream_t st) {
    const GemmGeom g =
        make_geom(Xp, Yp, rows, cols, rows_pad, cols_pad, kp, x_planes, y_planes, kAdjBM, kAdjBM);
    const char* name = "mt_adjoint_gemm_bf16";
    using CA = AdjCfg;
    if (adj.m_f64) return launch_gemm<CA, AdjointEpi<CA, double>>(g, b, plan, adj, name, st);
    return launch_gemm<CA, AdjointEpi<CA, float>>(g, b, plan, adj, name, st);
}

}  // namespace mt
