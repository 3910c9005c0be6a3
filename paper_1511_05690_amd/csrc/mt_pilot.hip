// Choice of the plan entry the forward p search starts at.
//
// p* is the largest stable p (Sec. 1); where the search starts only decides
// how much work finds it.  A tile that starts at plan entry s runs the dense
// GEMM for s, s + 1, ... until the entries still undecided fit the sparse
// tail, and hands them over; entries stable at s whose S does not rule out a
// larger p wait and go up from s - 1.  Starting below the largest p skips
// dense entries that only a few entries of each tile need, at the price of
// more tail work for those few.
//
// A pilot forms S_p for every plan entry on a grid of sampled output entries
// (the same planes the GEMM reads, FP32 / FP64 accumulation in another order:
// it only steers the work, the results do not depend on it), and a chooser
// estimates, for every start, the dense entries and tail dot products of a
// tile from the sampled p*, and writes the cheapest start to the workspace
// header, where the GEMM reads it.

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kPilotRows = 8;    // sample rows per pilot block
constexpr int kPilotKC = 64;     // K chunk staged through LDS
constexpr int kPilotThreads = 256;

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int64_t sample_index(int q, int nq, int64_t extent) {
    return ((2 * (int64_t)q + 1) * extent) / (2 * (int64_t)nq);
}

// Block (row group, plan entry e, K part): S_e of kPilotRows sample rows x pa.nc
// sample columns over its K range, written to part[kpart][e][r][c].
template <bool F64>
__global__ __launch_bounds__(kPilotThreads) void pilot_kernel(PilotArgs pa, FamilyPlan plan) {
    static_assert(F64, "the BF16 planes take the MFMA pilot");
    using T = typename std::conditional<F64, double, float>::type;
    using E = typename std::conditional<F64, double, uint16_t>::type;
    constexpr int NS = F64 ? 1 : 2;  // hi (and lo for a split p)
    // rows padded to KC + 16 bytes: 16-byte aligned for vector reads, and
    // the 32 columns a half-wave reads fall in different banks
    constexpr int LDR = kPilotKC + 16 / sizeof(T);
    __shared__ __attribute__((aligned(16))) T xs[NS][kPilotRows][LDR];
    __shared__ __attribute__((aligned(16))) T ys[NS][kMaxPilotSide][LDR];
    __shared__ int64_t roff[kPilotRows + kMaxPilotSide];  // row starts (element offsets, plane 0)
    const int tid = threadIdx.x;
    const int rg = blockIdx.x, e = blockIdx.y, kpart = blockIdx.z;
    const PlanEntry& pe = plan.e[e];
    const bool split = !F64 && pe.nseg == 3;
    const int64_t kchunk = ((pa.kp / pa.kparts + kPilotKC - 1) / kPilotKC) * kPilotKC;
    const int64_t k_lo = kpart * kchunk;
    const int64_t k_hi = min<int64_t>(k_lo + kchunk, pa.kp);
    const int nr = pa.nr, nc = pa.nc;
    // the rows of this block and the columns they meet come from batch item
    // rg % b; -1 marks a row or column outside the sample
    const int64_t bi = rg % pa.b;
    if (tid < kPilotRows + kMaxPilotSide) {
        int64_t o = -1;
        if (tid < kPilotRows) {
            const int r = rg * kPilotRows + tid;
            if (r < nr) o = bi * pa.x_batch_elems + sample_index(r, nr, pa.rows) * pa.kp;
        } else {
            const int c = tid - kPilotRows;
            if (c < nc) o = bi * pa.y_batch_elems + sample_index(c, nc, pa.cols) * pa.kp;
        }
        roff[tid] = o;
    }
    __syncthreads();
    const E* X = (const E*)pa.X;
    const E* Y = (const E*)pa.Y;
    const int64_t xh = (int64_t)pe.a_plane[0] * pa.x_plane_elems, xl = (int64_t)pe.a_plane[2] * pa.x_plane_elems;
    const int64_t yh = (int64_t)pe.b_plane[0] * pa.y_plane_elems, yl = (int64_t)pe.b_plane[1] * pa.y_plane_elems;
    // outputs of this thread: row tid / 32, columns tid % 32 and tid % 32 + 32
    const int orow = tid >> 5, oc0 = tid & 31, oc1 = oc0 + 32;
    T acc0 = 0, acc1 = 0;
    // staging: 16-byte loads of V elements; slot q of the chunk is row q / VR,
    // elements (q % VR) * V .. + V - 1 (VR = KC / V slots per row)
    constexpr int V = 16 / sizeof(E);
    constexpr int VR = kPilotKC / V;
    constexpr int SLOTS = (kPilotRows + kMaxPilotSide) * VR;
    constexpr int PER = (SLOTS + kPilotThreads - 1) / kPilotThreads;
    typedef uint32_t u32x4v __attribute__((ext_vector_type(4)));
    u32x4v vh[PER], vl[PER];
    // 16-byte loads of the chunk at k0 into vh / vl (zeros outside the sample
    // or the K range; k and k_hi are multiples of V, so a load is wholly
    // inside or outside)
    auto load = [&](int64_t k0) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = tid + j * kPilotThreads;
            vh[j] = u32x4v{0u, 0u, 0u, 0u};
            vl[j] = u32x4v{0u, 0u, 0u, 0u};
            if (q < SLOTS) {
                const int rr = q / VR;
                const int64_t k = k0 + (q % VR) * V;
                const int64_t o = roff[rr];
                if (o >= 0 && k < k_hi) {
                    const bool isx = rr < kPilotRows;
                    const E* base = isx ? X : Y;
                    vh[j] = *(const u32x4v*)(base + o + (isx ? xh : yh) + k);
                    if (split) vl[j] = *(const u32x4v*)(base + o + (isx ? xl : yl) + k);
                }
            }
        }
    };
    if (k_lo < k_hi) load(k_lo);
    for (int64_t k0 = k_lo; k0 < k_hi; k0 += kPilotKC) {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int q = tid + j * kPilotThreads;
            if (q >= SLOTS) continue;
            const int rr = q / VR, kk = (q % VR) * V;
            T* dh = rr < kPilotRows ? &xs[0][rr][kk] : &ys[0][rr - kPilotRows][kk];
            T* dl = rr < kPilotRows ? &xs[NS - 1][rr][kk] : &ys[NS - 1][rr - kPilotRows][kk];
            if constexpr (F64) {
                const double* d = (const double*)&vh[j];
                dh[0] = d[0];
                dh[1] = d[1];
            } else {
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    dh[2 * h] = __uint_as_float(vh[j][h] << 16);
                    dh[2 * h + 1] = __uint_as_float(vh[j][h] & 0xFFFF0000u);
                    dl[2 * h] = __uint_as_float(vl[j][h] << 16);
                    dl[2 * h + 1] = __uint_as_float(vl[j][h] & 0xFFFF0000u);
                }
            }
        }
        __syncthreads();
        // the next chunk's loads run while this one is summed
        if (k0 + kPilotKC < k_hi) load(k0 + kPilotKC);
        // 16-byte LDS reads: RV consecutive k per read
        constexpr int RV = 16 / sizeof(T);
        typedef T tvec __attribute__((ext_vector_type(RV)));
#pragma unroll 4
        for (int kk = 0; kk < kPilotKC; kk += RV) {
            const tvec xv = *(const tvec*)&xs[0][orow][kk];
            const tvec y0 = *(const tvec*)&ys[0][oc0][kk];
            const tvec y1 = *(const tvec*)&ys[0][oc1][kk];
#pragma unroll
            for (int h = 0; h < RV; ++h) {
                acc0 += xv[h] * y0[h];
                acc1 += xv[h] * y1[h];
            }
            if (split) {
                const tvec xl_ = *(const tvec*)&xs[NS - 1][orow][kk];
                const tvec l0 = *(const tvec*)&ys[NS - 1][oc0][kk];
                const tvec l1 = *(const tvec*)&ys[NS - 1][oc1][kk];
#pragma unroll
                for (int h = 0; h < RV; ++h) {
                    acc0 += xv[h] * l0[h] + xl_[h] * y0[h];
                    acc1 += xv[h] * l1[h] + xl_[h] * y1[h];
                }
            }
        }
        __syncthreads();
    }
    const int r = rg * kPilotRows + orow;
    if (r < nr) {
        T* part = (T*)pa.part + ((int64_t)kpart * plan.n + e) * kMaxPilotSide * kMaxPilotSide;
        if (oc0 < nc) part[r * kMaxPilotSide + oc0] = acc0;
        if (oc1 < nc) part[r * kMaxPilotSide + oc1] = acc1;
    }
}

// BF16 planes on MFMA: one wave per (tile t of the 2 x 2 grid of 32 x 32
// sample tiles, plan entry e, K part) sums its part of S_e for the tile with
// v_mfma_f32_32x32x16_bf16 (a split p as hi.hi + hi.lo + lo.hi, like the
// GEMM) into part[kpart][e][r][c].  Lane l loads row l % 32 of the tile, 8
// elements at k + 8 (l / 32), straight from the plane (the operand layout of
// the MFMA).
__global__ __launch_bounds__(64) void pilot_mfma_bf16_kernel(PilotArgs pa, FamilyPlan plan) {
    const int lane = threadIdx.x;
    const int t = blockIdx.x, e = blockIdx.y, kpart = blockIdx.z;
    const int mt = t >> 1, nt = t & 1;
    const PlanEntry& pe = plan.e[e];
    const bool split = pe.nseg == 3;
    const int64_t bi = t % pa.b;  // one batch item per sample tile
    const int r = mt * 32 + (lane & 31), c = nt * 32 + (lane & 31);
    const uint16_t* X = (const uint16_t*)pa.X;
    const uint16_t* Y = (const uint16_t*)pa.Y;
    const bool rok = r < pa.nr, cok = c < pa.nc;
    const int64_t xo = rok ? bi * pa.x_batch_elems + sample_index(r, pa.nr, pa.rows) * pa.kp : 0;
    const int64_t yo = cok ? bi * pa.y_batch_elems + sample_index(c, pa.nc, pa.cols) * pa.kp : 0;
    const uint16_t* xh = X + xo + (int64_t)pe.a_plane[0] * pa.x_plane_elems;
    const uint16_t* xl = X + xo + (int64_t)pe.a_plane[2] * pa.x_plane_elems;
    const uint16_t* yh = Y + yo + (int64_t)pe.b_plane[0] * pa.y_plane_elems;
    const uint16_t* yl = Y + yo + (int64_t)pe.b_plane[1] * pa.y_plane_elems;
    const int64_t kchunk = ((pa.kp + pa.kparts * 16 - 1) / (pa.kparts * 16)) * 16;
    const int64_t k_lo = kpart * kchunk, k_hi = min<int64_t>(k_lo + kchunk, pa.kp);
    const int ko = (lane >> 5) * 8;
    f32x16 acc = f32x16{};
    const bf16x8 zero = bf16x8{};
    constexpr int U = 4;
    int64_t k = k_lo;
    auto ld = [&](const uint16_t* p, bool ok, int64_t kk) { return ok ? *(const bf16x8*)(p + kk + ko) : zero; };
    for (; k + (U - 1) * 16 < k_hi; k += U * 16) {
        bf16x8 ah[U], bh[U], al[U], bl[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            ah[u] = ld(xh, rok, k + u * 16);
            bh[u] = ld(yh, cok, k + u * 16);
            if (split) {
                al[u] = ld(xl, rok, k + u * 16);
                bl[u] = ld(yl, cok, k + u * 16);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[u], bh[u], acc, 0, 0, 0);
            if (split) {
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[u], bl[u], acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[u], bh[u], acc, 0, 0, 0);
            }
        }
    }
    for (; k < k_hi; k += 16) {
        const bf16x8 a0 = ld(xh, rok, k), b0 = ld(yh, cok, k);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b0, acc, 0, 0, 0);
        if (split) {
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, ld(yl, cok, k), acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ld(xl, rok, k), b0, acc, 0, 0, 0);
        }
    }
    // accumulator element i of lane l: row (i / 4) * 8 + (l / 32) * 4 + i % 4,
    // column l % 32 of the tile
    float* part = (float*)pa.part + ((int64_t)kpart * plan.n + e) * kMaxPilotSide * kMaxPilotSide;
    const int ocol = nt * 32 + (lane & 31);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int orow = mt * 32 + (i >> 2) * 8 + (lane >> 5) * 4 + (i & 3);
        if (orow < pa.nr && ocol < pa.nc) part[orow * kMaxPilotSide + ocol] = acc[i];
    }
}

// One thread per sampled entry: its S_e (the K parts summed in order), its
// e* (first stable plan entry; the smallest p if none) and, for every start
// s where it would wait, the plan entry u where it is decided on the way up.
// Histograms of e* and of (s, u) per wave (ballots), then per block (LDS)
// and over the grid (global atomics): integer counts, so the choice does not
// depend on the order of the atomics.
template <bool F64>
__global__ __launch_bounds__(kPilotThreads) void pilot_count_kernel(PilotArgs pa, FamilyPlan plan) {
    using T = typename std::conditional<F64, double, float>::type;
    __shared__ PilotCounts sc;
    const int tid = threadIdx.x, lane = tid & 63;
    const int n = plan.n;
    for (int i = tid; i < (int)(sizeof(PilotCounts) / 4); i += kPilotThreads) ((int32_t*)&sc)[i] = 0;
    __syncthreads();
    const T tau = F64 ? (T)plan.tau : (T)plan.tau_f;
    const int q = blockIdx.x * kPilotThreads + tid;
    const bool in = q < pa.nr * pa.nc;
    const int r = in ? q / pa.nc : 0, c = in ? q % pa.nc : 0;
    T S[MT_MAX_P];
    int es = n - 1;
#pragma unroll
    for (int e = MT_MAX_P - 1; e >= 0; --e) {
        T v = 0;
        if (e < pa.n_eval && in) {
            T pv[kMaxPilotKParts];
#pragma unroll
            for (int kp = 0; kp < kMaxPilotKParts; ++kp)
                pv[kp] = kp < pa.kparts ? ((const T*)pa.part)[((int64_t)kp * n + e) * kMaxPilotSide * kMaxPilotSide +
                                                             r * kMaxPilotSide + c]
                                        : (T)0;
#pragma unroll
            for (int kp = 0; kp < kMaxPilotKParts; ++kp) v += pv[kp];
            if (v >= tau) es = e;
        }
        S[e] = v;
    }
    for (int e = 0; e < n; ++e) {
        const int cnt = __popcll(__ballot(in && es == e));
        if (lane == 0 && cnt) atomicAdd(&sc.es_hist[e], cnt);
    }
#pragma unroll
    for (int s = 1; s < MT_MAX_P; ++s) {
        if (s >= n) break;
        const T thr = F64 ? (T)plan.e[s].rise_thr : (T)plan.e[s].rise_thr_f;
        const bool parked = in && S[s] >= tau && S[s] >= thr;
        int u = s - 1;  // decided at plan entry u going up
        bool up = parked;
#pragma unroll
        for (int uu = MT_MAX_P - 2; uu > 0; --uu) {
            if (uu >= s) continue;
            const T tu = F64 ? (T)plan.e[uu].rise_thr : (T)plan.e[uu].rise_thr_f;
            if (up && S[uu] >= tau && S[uu] >= tu) u = uu - 1;
            else up = false;
        }
        for (int v = 0; v < s; ++v) {
            const int cnt = __popcll(__ballot(parked && u == v));
            if (lane == 0 && cnt) atomicAdd(&sc.stop[s][v], cnt);
        }
    }
    __syncthreads();
    PilotCounts* gc = (PilotCounts*)pa.counts;
    for (int i = tid; i < (int)(sizeof(PilotCounts) / 4); i += kPilotThreads) {
        const int32_t v = ((int32_t*)&sc)[i];
        if (v) atomicAdd(&((int32_t*)gc)[i], v);
    }
}

// The cost model on the counts, one lane per start s.  Costs are in dense
// tile-entry units (one plain p of the family over one tile; a split p
// counts 3) plus kappa per tail dot product (a split p's dot reads four
// plane rows and counts 2).
template <bool F64>
__global__ __launch_bounds__(64) void pilot_choose_kernel(PilotArgs pa, FamilyPlan plan, int32_t* start) {
    __shared__ float cost[MT_MAX_P];
    __shared__ PilotCounts sc;
    __shared__ float Wc[MT_MAX_P], Wd[MT_MAX_P];
    for (int i = threadIdx.x; i < (int)(sizeof(PilotCounts) / 4); i += 64)
        ((int32_t*)&sc)[i] = ((const int32_t*)pa.counts)[i];
    const int n = plan.n;
    if (threadIdx.x == 0) {
        float w = 0.f;
        for (int e = 0; e < n; ++e) {
            const bool sp = !F64 && plan.e[e].nseg == 3;
            w += sp ? 2.f : 1.f;
            Wc[e] = w;
            Wd[e] = sp ? 3.f : 1.f;
        }
    }
    __syncthreads();
    const int s = threadIdx.x;
    // W(e): dot weight of plan entries 0 .. e; wdense(e): dense cost of entry e
    auto W = [&](int e) { return Wc[e]; };
    auto wdense = [&](int e) { return Wd[e]; };
    if (s < n) {
        const int nsamp = pa.nr * pa.nc;
        const float scale = (float)pa.tile_entries / (float)(nsamp > 0 ? nsamp : 1);
        // a tile hands over when its expected undecided count is at most
        // half the tail capacity (counts vary between tiles)
        const float cap = 0.5f * (float)pa.tail_max;
        float pk = 0.f, updots = 0.f;
        for (int u = 0; u < s; ++u) {
            pk += (float)sc.stop[s][u];
            updots += (float)sc.stop[s][u] * (W(s - 1) - (u > 0 ? W(u - 1) : 0.f));
        }
        pk *= scale;
        float dense = 0.f, dots = 0.f;
        for (int d = s; d < n; ++d) {
            dense += wdense(d);
            // open after d: e* > d (those are not waiting: they are unstable at s)
            float open = 0.f, odots = 0.f;
            if (d < n - 1)
                for (int e = d + 1; e < n; ++e) {
                    open += (float)sc.es_hist[e];
                    odots += (float)sc.es_hist[e] * (W(e) - W(d));
                }
            open *= scale;
            if (open + pk <= cap && open + pk > 0.f) {
                dots = (odots + updots) * scale;
                break;
            }
            if (open < 0.5f) {
                if (pk >= 0.5f) {
                    // only waiting entries left: dense entries on the way up
                    for (int u = s - 1; u >= 0; --u) {
                        dense += wdense(u);
                        float left = 0.f;
                        for (int v = 0; v < u; ++v) left += (float)sc.stop[s][v];
                        left *= scale;
                        if (left <= cap) {
                            // their remaining dots: about half the weight above u
                            dots = left * (u > 0 ? W(u - 1) : 0.f) * 0.5f;
                            break;
                        }
                    }
                }
                break;
            }
        }
        cost[s] = dense + pa.kappa * dots;
    }
    __syncthreads();
    if (s == 0) {
        int best = 0;
        float best_cost = cost[0];
        // a start on deferred planes is not an option
        for (int x = 1; x < pa.n_eval; ++x)
            if (cost[x] < best_cost * 0.98f) {  // a start further down must save at least 2 %
                best_cost = cost[x];
                best = x;
            }
        *start = best;
        if (pa.low_need != nullptr) {
            // sampled entries with no stable p among the evaluated plan
            // entries (e* counted at the last entry) need the deferred planes
            int need = 0;
            for (int e = pa.n_eval; e < n; ++e) need |= sc.es_hist[e];
            *pa.low_need = need != 0 ? 1 : 0;
            *pa.low_missed = 0;
        }
    }
}

}  // namespace

hipError_t launch_choose_start(const PilotArgs& pa, const FamilyPlan& plan, int32_t* start, int f64,
                               hipStream_t st) {
    if (plan.n < 2 || pa.nr <= 0 || pa.nc <= 0) {
        // no pilot: the search starts at the largest p, every plane is due
        if (pa.low_need != nullptr) {
            hipError_t e = launch_fill_u32(pa.low_need, 1u, 1, st);
            if (e == hipSuccess) e = launch_fill_zero_u32(pa.low_missed, 1, st);
            if (e != hipSuccess) return e;
        }
        return launch_fill_u32(start, 0u, 1, st);
    }
    hipError_t e = launch_fill_zero_u32(pa.counts, sizeof(PilotCounts) / 4, st);
    if (e != hipSuccess) return e;
    if (pa.n_eval < 1 || pa.n_eval > plan.n) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((pa.nr + kPilotRows - 1) / kPilotRows), (unsigned)pa.n_eval, (unsigned)pa.kparts);
    const dim3 cgrid((unsigned)((pa.nr * pa.nc + kPilotThreads - 1) / kPilotThreads));
    timing_before("mt_pilot", st);
    if (f64) {
        hipLaunchKernelGGL(pilot_kernel<true>, grid, dim3(kPilotThreads), 0, st, pa, plan);
        hipLaunchKernelGGL(pilot_count_kernel<true>, cgrid, dim3(kPilotThreads), 0, st, pa, plan);
        hipLaunchKernelGGL(pilot_choose_kernel<true>, dim3(1), dim3(64), 0, st, pa, plan, start);
    } else {
        hipLaunchKernelGGL(pilot_mfma_bf16_kernel, dim3(4, (unsigned)pa.n_eval, (unsigned)pa.kparts), dim3(64), 0, st, pa, plan);
        hipLaunchKernelGGL(pilot_count_kernel<false>, cgrid, dim3(kPilotThreads), 0, st, pa, plan);
        hipLaunchKernelGGL(pilot_choose_kernel<false>, dim3(1), dim3(64), 0, st, pa, plan, start);
    }
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
