// Fused p-family GEMM on FP64 MFMA (gfx950) with the selection step: the
// plain-precision path of the p-norm estimate.  Same scheme as the BF16
// kernel (ring product of every p of the family per output tile, largest p
// first; Alg. 5 and Sec. 1), with FP64 power planes, v_mfma_f64_16x16x4f64 and
// an FP64 stability test.  The epilogue records, once per entry, the ring
// result S at the largest p with S_p >= tau and that p's index; the FP64 root
// C = r c S^(1/p) is taken by the select-root pass (mt_elementwise.hip).
//
// Tiling: 256 threads = 4 waves in 2 x 2; each wave owns WT x WT MFMA tiles of
// 16 x 16.  K step 16 doubles = 128-byte LDS rows, loaded by
// global_load_lds_dwordx4 and double buffered; 16-byte chunk index
// XOR-swizzled with (row >> 1) & 7.
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;

struct GemmGeomF64 {
    const double* A;
    const double* B;
    int64_t a_plane_elems;
    int64_t b_plane_elems;
    int64_t m, n, kp;
    int32_t n_planes;
    int32_t tiles_m, tiles_n;
};

template <int WT>
struct CfgF64 {
    static constexpr int BM = 2 * WT * 16;
    static constexpr int A_BYTES = BM * 128;
    static constexpr int BUF_BYTES = 2 * A_BYTES;
    static constexpr int NDEC = (WT * WT * 4 + 31) / 32;
    static constexpr int LDS_BYTES = 2 * BUF_BYTES;
};

template <int WT>
__global__ __launch_bounds__(kThreads, 1) void mt_pfamily_gemm_f64_kernel(GemmGeomF64 g,
                                                                         FamilyPlan plan,
                                                                         EpiArgs epi) {
    using C = CfgF64<WT>;
    static_assert((C::BM / 32) % 2 == 0, "row groups per wave must be even");
    extern __shared__ __attribute__((aligned(1024))) uint8_t smem[];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;

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
    const int64_t col0 = (int64_t)tn * C::BM;

    const double* Abase = g.A + (int64_t)bi * g.n_planes * g.a_plane_elems + row0 * g.kp;
    const double* Bbase = g.B + (int64_t)bi * g.n_planes * g.b_plane_elems + col0 * g.kp;
    const int nkt = (int)(g.kp / 16);

    // Loads: lane l fills row R0 + l/8, physical 16-byte chunk l%8 holding
    // logical chunk (l%8) ^ swz(row) = (l%8) ^ ((i&1)*4 + l/16).
    const int32_t ld_even = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (lane >> 4)) * 2);
    const int32_t ld_odd = (lane >> 3) * (int32_t)g.kp + (((lane & 7) ^ (4 + (lane >> 4))) * 2);
    // Operand reads: row l%16 of a 16-row block, k = 4*kk + l/16, i.e.
    // logical chunk 2*kk + l/32, half (l/16)&1; swizzle (l >> 1) & 7.
    const int32_t rd_base = (lane & 15) * 128 + (((lane >> 5) ^ ((lane >> 1) & 7)) * 16) + ((lane >> 4) & 1) * 8;

    auto issue = [&](int e, int s, int kt, int buf) {
        const double* asrc = Abase + (int64_t)plan.e[e].a_plane[s] * g.a_plane_elems + kt * 16;
        const double* bsrc = Bbase + (int64_t)plan.e[e].b_plane[s] * g.b_plane_elems + kt * 16;
        uint8_t* la = smem + buf * C::BUF_BYTES;
        uint8_t* lb = la + C::A_BYTES;
#pragma unroll
        for (int i = 0; i < C::BM / 32; ++i) {
            const int R0 = (wave * (C::BM / 32) + i) * 8;
            const int32_t lo = (i & 1) ? ld_odd : ld_even;
            __builtin_amdgcn_global_load_lds((glb_cvoid*)(asrc + (int64_t)R0 * g.kp + lo),
                                             (lds_void*)(la + R0 * 128), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((glb_cvoid*)(bsrc + (int64_t)R0 * g.kp + lo),
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

    // Entry (i, j, r) of this lane: tile row wm*WT*16 + i*16 + l/16 + 4r,
    // tile column wn*WT*16 + j*16 + l%16.
    const int lr0 = wm * WT * 16 + (lane >> 4);
    const int lc0 = wn * WT * 16 + (lane & 15);
    const int64_t out_lane = ((int64_t)bi * g.m + row0 + lr0) * g.n + col0 + lc0;
    const int32_t rows_left = (int32_t)min<int64_t>(g.m - (row0 + lr0), 1 << 30);
    const int32_t cols_left = (int32_t)min<int64_t>(g.n - (col0 + lc0), 1 << 30);

    int le = 0, ls = 0, lkt = 0;
    if (nkt > 0) {
        issue(le, ls, lkt, 0);
        advance(le, ls, lkt);
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();

    int buf = 0;
    for (int e = 0; e < plan.n; ++e) {
        f64x4 acc[WT][WT];
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) acc[i][j] = f64x4{};

        const int ntiles = plan.e[e].nseg * nkt;
        for (int t2 = 0; t2 < ntiles; ++t2) {
            if (le < plan.n) {
                issue(le, ls, lkt, buf ^ 1);
                advance(le, ls, lkt);
            }
            const uint8_t* la = smem + buf * C::BUF_BYTES + wm * WT * 16 * 128;
            const uint8_t* lb = smem + buf * C::BUF_BYTES + C::A_BYTES + wn * WT * 16 * 128;
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
                const int32_t ro = rd_base ^ (kk << 5);
                double a[WT], b[WT];
#pragma unroll
                for (int i = 0; i < WT; ++i) a[i] = *(const double*)(la + i * 16 * 128 + ro);
#pragma unroll
                for (int j = 0; j < WT; ++j) b[j] = *(const double*)(lb + j * 16 * 128 + ro);
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

        // ---- selection for family entry e: record S at the selected p and
        // the p index; the root r c S^(1/p) is applied by the select-root pass.
        const bool last = (e == plan.n - 1);
        const double tau = plan.tau;
        const uint8_t pcode = (uint8_t)plan.e[e].pidx;
        double* out = (double*)epi.out + out_lane;
        uint8_t* ps = epi.pstar + out_lane;
        // Stage each 16 x 16 tile (lane-major) in the buffer just consumed
        // (free until the next issue, which waits for the barrier below) and
        // walk its four entries per lane in a rolled loop.
        double* stg = (double*)(smem + (buf ^ 1) * C::BUF_BYTES) + wave * 256;
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j) {
#pragma unroll
                for (int r = 0; r < 4; ++r) stg[r * 64 + lane] = acc[i][j][r];
                __builtin_amdgcn_wave_barrier();
                const bool col_ok = j * 16 < cols_left;
                const int tix = i * WT + j;
                uint32_t dec = decided[tix >> 3];
                const int sh = (tix & 7) * 4;
#pragma unroll 1
                for (int r = 0; r < 4; ++r) {
                    const uint32_t mask = 1u << (sh + r);
                    const int roff = i * 16 + 4 * r;
                    const double S = stg[r * 64 + lane];
                    const bool stable = S >= tau;
                    if (col_ok && roff < rows_left && !(dec & mask) && (stable || last)) {
                        dec |= mask;
                        const int64_t o = (int64_t)roff * g.n + j * 16;
                        out[o] = S;
                        ps[o] = stable ? pcode : (uint8_t)MT_PSTAR_NONE;
                    }
                }
                decided[tix >> 3] = dec;
                __builtin_amdgcn_wave_barrier();
            }
        __syncthreads();
    }
}

template <int WT>
hipError_t launch_cfg(const GemmGeomF64& g, int64_t b, const FamilyPlan& plan, const EpiArgs& epi,
                      hipStream_t st) {
    using C = CfgF64<WT>;
    auto kern = mt_pfamily_gemm_f64_kernel<WT>;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e =
            hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, C::LDS_BYTES);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    const int64_t nwg = b * (int64_t)g.tiles_m * g.tiles_n;
    timing_before("mt_pfamily_gemm_f64", st);
    hipLaunchKernelGGL(kern, dim3((unsigned)nwg), dim3(kThreads), C::LDS_BYTES, st, g, plan, epi);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pfamily_gemm_f64(const double* Ap, const double* Bp, int64_t b, int64_t m,
                                   int64_t n, int64_t mp, int64_t np, int64_t kp, int32_t n_planes,
                                   int bm, const FamilyPlan& plan, const EpiArgs& epi,
                                   hipStream_t st) {
    GemmGeomF64 g;
    g.A = Ap;
    g.B = Bp;
    g.a_plane_elems = mp * kp;
    g.b_plane_elems = np * kp;
    g.m = m;
    g.n = n;
    g.kp = kp;
    g.n_planes = n_planes;
    g.tiles_m = (int32_t)(mp / bm);
    g.tiles_n = (int32_t)(np / bm);
    if (bm == 128) return launch_cfg<4>(g, b, plan, epi, st);
    if (bm == 64) return launch_cfg<2>(g, b, plan, epi, st);
    return hipErrorInvalidValue;
}

}  // namespace mt
