// Fused p-family GEMM on BF16 MFMA (gfx950) with the selection epilogue.
//
// For one output tile the kernel runs the ring product S_p = A'^p B'^p of
// every p of the family (Alg. 5, first loop; Sec. 2.1 distributivity), one
// after the other, largest p first, and after each p keeps, per entry, the
// first p whose ring result passes the stability test S_p >= tau (Sec. 1,
// the highest stable p).  Because the entries are visited from the largest p
// down, the first pass is the largest stable p, and C = r c S^(1/p) is
// written exactly once per entry.  Entries that never pass take the smallest
// p (index MT_PSTAR_NONE).
//
// Operands are the BF16 power planes written by the plane kernel: A planes
// m_pad x k_pad and B^T planes n_pad x k_pad, K contiguous.  A split p is
// three segments (hi.hi + hi.lo + lo.hi) accumulated into one FP32 sum.
//
// Tiling: 256 threads = 4 waves in 2 x 2; each wave owns WT_M x WT_N MFMA
// tiles of 32 x 32 (v_mfma_f32_32x32x16_bf16).  K step 64: the A and B tiles
// of a step are copied global -> LDS by the direct-to-LDS loads
// (global_load_lds_dwordx4), double buffered, so the next step's loads fly
// while the current step's MFMAs run.  The LDS rows are 128 bytes; the
// 16-byte chunk index is XOR-swizzled with (row >> 1) & 7 so that the MFMA
// operand reads (16 rows x one chunk per 256 bytes) hit distinct banks.
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int swz(int row) { return (row >> 1) & 7; }

// S^(1/p) in FP32 with the hardware log2 / exp2 (about 1 ulp each); S = 0
// gives 0 (log2 0 = -inf, 2^-inf = 0), denormal S is rescaled first.
__device__ __forceinline__ float root_f32(float S, float inv_p) {
    const bool tiny = S < 1.17549435e-38f;
    const float l = __builtin_amdgcn_logf(tiny ? S * 18446744073709551616.f : S) - (tiny ? 64.f : 0.f);
    return __builtin_amdgcn_exp2f(l * inv_p);
}

struct GemmGeom {
    const uint16_t* A;
    const uint16_t* B;
    int64_t a_plane_elems;  // m_pad * k_pad
    int64_t b_plane_elems;  // n_pad * k_pad
    int64_t m, n, kp;
    int32_t n_planes;
    int32_t tiles_m, tiles_n;
};

template <int WT_M, int WT_N>
struct Cfg {
    static constexpr int BM = 2 * WT_M * 32;
    static constexpr int BN = 2 * WT_N * 32;
    static constexpr int A_BYTES = BM * 128;
    static constexpr int B_BYTES = BN * 128;
    static constexpr int BUF_BYTES = A_BYTES + B_BYTES;
    static constexpr int NDEC = (WT_M * WT_N * 16 + 31) / 32;
    static constexpr int STG = 32 * 33;  // floats of one wave's staging tile
    static constexpr int LDS_BYTES = 2 * BUF_BYTES + (BM + BN) * 4 + 4 * STG * 4;
};

template <int WT_M, int WT_N, int MODE, typename TO>
__global__ __launch_bounds__(kThreads, 1) void mt_pfamily_gemm_bf16_kernel(GemmGeom g,
                                                                          FamilyPlan plan,
                                                                          EpiArgs epi) {
    using C = Cfg<WT_M, WT_N>;
    static_assert((C::BM / 32) % 2 == 0 && (C::BN / 32) % 2 == 0, "row groups per wave must be even");
    extern __shared__ __attribute__((aligned(1024))) uint8_t smem[];
    float* rs = (float*)(smem + 2 * C::BUF_BYTES);  // BM row scales
    float* cs = rs + C::BM;                         // BN column scales
    float* stg_all = cs + C::BN;                    // 4 x (32 x 33) epilogue staging

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;

    // Workgroup -> tile.  Consecutive workgroup ids are spread over the 8
    // XCDs; regroup so each XCD owns a contiguous run of tiles, then walk the
    // run in bands of 8 tile rows so concurrently resident tiles share A rows
    // and B columns in that XCD's L2.
    int id = blockIdx.x;
    const int nwg = gridDim.x;
    if ((nwg & 7) == 0) id = (id & 7) * (nwg >> 3) + (id >> 3);
    const int per_batch = g.tiles_m * g.tiles_n;
    const int bi = id / per_batch;
    const int t = id - bi * per_batch;
    constexpr int GROUP = 8;
    const int group = t / (GROUP * g.tiles_n);
    const int first_m = group * GROUP;
    const int gsz = min(GROUP, g.tiles_m - first_m);
    const int in_g = t - group * GROUP * g.tiles_n;
    const int tm = first_m + in_g % gsz;
    const int tn = in_g / gsz;
    const int64_t row0 = (int64_t)tm * C::BM;
    const int64_t col0 = (int64_t)tn * C::BN;

    // Row / column scales of this tile into LDS (1 where absent or padding).
    for (int i = tid; i < C::BM + C::BN; i += kThreads) {
        double v = 1.0;
        if (i < C::BM) {
            if (epi.r && row0 + i < g.m) v = epi.r[(int64_t)bi * g.m + row0 + i];
        } else {
            const int64_t cc = col0 + (i - C::BM);
            if (epi.c && cc < g.n) v = epi.c[(int64_t)bi * g.n + cc];
        }
        rs[i] = (float)v;
    }

    const uint16_t* Abase = g.A + (int64_t)bi * g.n_planes * g.a_plane_elems + row0 * g.kp;
    const uint16_t* Bbase = g.B + (int64_t)bi * g.n_planes * g.b_plane_elems + col0 * g.kp;
    const int nkt = (int)(g.kp / 64);

    // Global source offsets of the direct-to-LDS loads.  Load instruction i
    // of this wave fills LDS rows R0 .. R0+7, R0 = (wave * G + i) * 8 with G
    // row groups per wave; lane l fills row R0 + l/8, physical chunk l%8,
    // which holds logical chunk (l%8) ^ swz(row).  For even G the swizzle is
    // (i&1)*4 + l/16, so two lane offsets cover every instruction.
    const int32_t ld_even = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (lane >> 4)) * 8);
    const int32_t ld_odd = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (4 + (lane >> 4))) * 8);
    // LDS operand reads: row (lane & 31) of a 32-row block, logical chunk
    // 2*kk + lane/32, swizzle (lane >> 1) & 7 (block bases are multiples of 32).
    const int32_t rd_base = (lane & 31) * 128 + (((lane >> 5) ^ ((lane >> 1) & 7)) * 16);

    auto issue = [&](int e, int s, int kt, int buf) {
        const uint16_t* asrc = Abase + (int64_t)plan.e[e].a_plane[s] * g.a_plane_elems + kt * 64;
        const uint16_t* bsrc = Bbase + (int64_t)plan.e[e].b_plane[s] * g.b_plane_elems + kt * 64;
        uint8_t* la = smem + buf * C::BUF_BYTES;
        uint8_t* lb = la + C::A_BYTES;
#pragma unroll
        for (int i = 0; i < C::BM / 32; ++i) {
            const int R0 = (wave * (C::BM / 32) + i) * 8;
            __builtin_amdgcn_global_load_lds(
                (glb_cvoid*)(asrc + (int64_t)R0 * g.kp + ((i & 1) ? ld_odd : ld_even)),
                (lds_void*)(la + R0 * 128), 16, 0, 0);
        }
#pragma unroll
        for (int i = 0; i < C::BN / 32; ++i) {
            const int R0 = (wave * (C::BN / 32) + i) * 8;
            __builtin_amdgcn_global_load_lds(
                (glb_cvoid*)(bsrc + (int64_t)R0 * g.kp + ((i & 1) ? ld_odd : ld_even)),
                (lds_void*)(lb + R0 * 128), 16, 0, 0);
        }
    };
    auto advance = [&](int& e, int& s, int& kt) {
        if (++kt == nkt) {
            kt = 0;
            if (++s == plan.e[e].nseg) {
                s = 0;
                ++e;
            }
        }
    };

    uint32_t decided[C::NDEC];
#pragma unroll
    for (int i = 0; i < C::NDEC; ++i) decided[i] = 0u;

    // Epilogue addressing.  Tile (i, j) of this wave is staged through LDS as
    // a 32 x 32 block; lane l then handles rows 2q + l/32 (q = 0..15) of
    // column l%32, so lanes 0-31 and 32-63 store two consecutive row runs.
    float* stg = stg_all + wave * C::STG;
    const int lr0 = wm * WT_M * 32 + (lane >> 5);
    const int lc0 = wn * WT_N * 32 + (lane & 31);
    const int64_t out_lane = ((int64_t)bi * g.m + row0 + lr0) * g.n + col0 + lc0;
    // entry valid iff its row offset < rows_left and column offset < cols_left
    const int32_t rows_left = (int32_t)min<int64_t>(g.m - (row0 + lr0), 1 << 30);
    const int32_t cols_left = (int32_t)min<int64_t>(g.n - (col0 + lc0), 1 << 30);
    const int32_t diag_off = (int32_t)((col0 + lc0) - (row0 + lr0));  // APSP diagonal

    // Software pipeline: the loads of the next K step (possibly of the next
    // segment or family entry) are issued before the MFMAs of the current one.
    int le = 0, ls = 0, lkt = 0;
    if (nkt > 0) {
        issue(le, ls, lkt, 0);
        advance(le, ls, lkt);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    int buf = 0;
    for (int e = 0; e < plan.n; ++e) {
        f32x16 acc[WT_M][WT_N];
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) acc[i][j] = f32x16{};

        const int ntiles = plan.e[e].nseg * nkt;
        for (int t = 0; t < ntiles; ++t) {
            if (le < plan.n) {
                issue(le, ls, lkt, buf ^ 1);
                advance(le, ls, lkt);
            }
            const uint8_t* la = smem + buf * C::BUF_BYTES + wm * WT_M * 32 * 128;
            const uint8_t* lb = smem + buf * C::BUF_BYTES + C::A_BYTES + wn * WT_N * 32 * 128;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int32_t ro = rd_base ^ (kk << 5);
                bf16x8 a[WT_M], b[WT_N];
#pragma unroll
                for (int i = 0; i < WT_M; ++i) a[i] = *(const bf16x8*)(la + i * 32 * 128 + ro);
#pragma unroll
                for (int j = 0; j < WT_N; ++j) b[j] = *(const bf16x8*)(lb + j * 32 * 128 + ro);
#pragma unroll
                for (int i = 0; i < WT_M; ++i)
#pragma unroll
                    for (int j = 0; j < WT_N; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
            }
            asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
            __syncthreads();
            buf ^= 1;
        }

        // ---- selection epilogue for family entry ce
        const bool last = (e == plan.n - 1);
        const float inv_p = plan.e[e].inv_p;
        const bool p_is_1 = plan.e[e].p == 1;
        const float corr = plan.e[e].corr;
        // S >= tau in FP64 is S >= tau_f in FP32 (tau_f: tau rounded up to FP32)
        const float tau_f = plan.tau_f;
        const uint8_t pcode = (uint8_t)plan.e[e].pidx;
        TO* out = (TO*)epi.out + out_lane;
        uint8_t* ps = epi.pstar ? epi.pstar + out_lane : nullptr;
#pragma unroll
        for (int i = 0; i < WT_M; ++i)
#pragma unroll
            for (int j = 0; j < WT_N; ++j) {
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    stg[((r >> 2) * 8 + (lane >> 5) * 4 + (r & 3)) * 33 + (lane & 31)] = acc[i][j][r];
                __builtin_amdgcn_wave_barrier();
                const float cj = cs[lc0 + j * 32];
                const bool col_ok = j * 32 < cols_left;
                const int tix = i * WT_N + j;
                uint32_t dec = decided[tix >> 1];
                const int sh = (tix & 1) * 16;
#pragma unroll 2
                for (int q = 0; q < 16; ++q) {
                    const int roff = i * 32 + 2 * q;
                    const float S = stg[(2 * q + (lane >> 5)) * 33 + (lane & 31)];
                    const bool stable = S >= tau_f;
                    const uint32_t mask = 1u << (sh + q);
                    if (col_ok && roff < rows_left && !(dec & mask) && (stable || last)) {
                        dec |= mask;
                        float v = rs[lr0 + roff] * cj * (p_is_1 ? S : root_f32(S, inv_p)) * corr;
                        if (MODE == EPI_APSP_X || epi.clamp) v = fminf(v, 1.f);
                        if (MODE == EPI_APSP_X && roff - j * 32 == diag_off) v = 1.f;
                        const int64_t o = (int64_t)roff * g.n + j * 32;
                        out[o] = (TO)v;
                        if (ps) ps[o] = stable ? pcode : (uint8_t)MT_PSTAR_NONE;
                    }
                }
                decided[tix >> 1] = dec;
                __builtin_amdgcn_wave_barrier();
            }
    }
}

template <int WT_M, int WT_N, int MODE, typename TO>
hipError_t launch_cfg(const GemmGeom& g, int64_t b, const FamilyPlan& plan, const EpiArgs& epi,
                      hipStream_t st) {
    using C = Cfg<WT_M, WT_N>;
    const int lds = C::LDS_BYTES;
    auto kern = mt_pfamily_gemm_bf16_kernel<WT_M, WT_N, MODE, TO>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t nwg = b * (int64_t)g.tiles_m * g.tiles_n;
    timing_before("mt_pfamily_gemm_bf16", st);
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(kThreads), lds, st, g, plan, epi);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pfamily_gemm_bf16(const uint16_t* Ap, const uint16_t* Bp, int64_t b, int64_t m,
                                    int64_t n, int64_t mp, int64_t np, int64_t kp,
                                    int32_t n_planes, const FamilyPlan& plan, const EpiArgs& epi,
                                    hipStream_t st) {
    GemmGeom g;
    g.A = Ap;
    g.B = Bp;
    g.a_plane_elems = mp * kp;
    g.b_plane_elems = np * kp;
    g.m = m;
    g.n = n;
    g.kp = kp;
    g.n_planes = n_planes;
    g.tiles_m = (int32_t)(mp / kBf16BM);
    g.tiles_n = (int32_t)(np / kBf16BN);
    if (epi.mode == EPI_APSP_X) {
        if (epi.out_f64) return launch_cfg<4, 4, EPI_APSP_X, double>(g, b, plan, epi, st);
        return launch_cfg<4, 4, EPI_APSP_X, float>(g, b, plan, epi, st);
    }
    if (epi.out_f64) return launch_cfg<4, 4, EPI_PLAIN, double>(g, b, plan, epi, st);
    return launch_cfg<4, 4, EPI_PLAIN, float>(g, b, plan, epi, st);
}

}  // namespace mt
