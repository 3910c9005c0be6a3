// One-kernel product estimate on the FP64 path for small products: the row
// and column scales of the scaled ring call H' (Sec. 2.1), the powers, the
// ring products S_p = A'^p B'^p (Alg. 3 / Alg. 5) and the selection of the
// largest stable p with its 1/p root (Sec. 1, Alg. 5) in one launch.
//
// A workgroup owns a 32 x 32 output tile of one batch item.  It holds up to
// 256 inner indices of its 32 rows of A and 32 columns of B in LDS at a time
// (the whole inner dimension for k <= 256, loaded once), takes the row and
// column maxima from them, then visits the family from the largest p down:
// for each p it stages (a / r)^p and (b / c)^p of 32 inner indices at a
// time and accumulates S_p in FP64 on the vector ALUs (each thread 2 x 2
// entries).  An entry takes the first p with S_p >= tau (at the smallest p:
// whatever S is, with no stable p marked); the tile stops once every entry
// has its p.  For the small products it serves (b m k n up to a few times
// 256^3) this replaces the general path's seven to fourteen launches
// (maxima, planes, MFMA GEMM, sparse tail, root) whose fixed costs exceed the
// arithmetic.  The numbers are those of the general FP64 path up to the
// order of the FP64 sums.
#include <atomic>
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kSmTile = 32;      // output tile edge
constexpr int kSmK = 32;         // inner indices of one staged power chunk
constexpr int kSmKR = 256;       // inner indices held raw in LDS at a time
constexpr int kSmThreads = 256;  // 16 x 16 threads, 2 x 2 entries each
// LDS in doubles: raw A [32][KR + 1], raw B [KR][32], powers A [32][K + 1],
// powers B [K][32], then r, 1/r, c, 1/c
constexpr int kSmRawA = kSmTile * (kSmKR + 1);
constexpr int kSmRawB = kSmKR * kSmTile;
constexpr int kSmPowA = kSmTile * (kSmK + 1);
constexpr int kSmPowB = kSmK * kSmTile;
constexpr size_t kSmLdsBytes = sizeof(double) * (kSmRawA + kSmRawB + kSmPowA + kSmPowB + 4 * kSmTile);

// the scaled input a / s of H': one reciprocal per line when s is normal
// (inv > 0), a division when s is subnormal, 0 for a zero line
__device__ inline double sm_scaled(double a, double s, double inv) {
    if (__builtin_expect(inv > 0.0, 1)) return a * inv;
    return s > 0.0 ? a / s : 0.0;
}

template <typename TS, typename TO>
__global__ __launch_bounds__(kSmThreads) void mt_small_product_f64_kernel(const TS* __restrict__ A,
                                                                         const TS* __restrict__ B, int64_t m,
                                                                         int64_t k, int64_t n, SmallSpec spec,
                                                                         TO* __restrict__ C,
                                                                         uint8_t* __restrict__ pstar,
                                                                         unsigned long long* work) {
    extern __shared__ double sm[];
    double* ar = sm;              // [i * (KR + 1) + kk]
    double* br = ar + kSmRawA;    // [kk * 32 + j]
    double* ap = br + kSmRawB;    // [i * (K + 1) + kk]
    double* bp = ap + kSmPowA;    // [kk * 32 + j]
    double* rs = bp + kSmPowB;
    double* rinv = rs + kSmTile;
    double* cs = rinv + kSmTile;
    double* cinv = cs + kSmTile;

    const int tid = threadIdx.x;
    if (work && tid == 0) timing_span_begin(work);
    const int64_t bi = blockIdx.z;
    const int64_t row0 = (int64_t)blockIdx.y * kSmTile;
    const int64_t col0 = (int64_t)blockIdx.x * kSmTile;
    const TS* a = A + bi * m * k;
    const TS* b = B + bi * k * n;

    // raw inner indices kr0 .. kr0 + KR - 1 of the tile's rows of A (read
    // along k) and columns of B (read along the columns) into LDS; 0 outside.
    // Every load is issued (indices outside are clamped to the last row,
    // column or inner index and the value dropped), so that they are all in
    // flight at once instead of one conditional load after another.
    auto load_raw = [&](int64_t kr0, bool scale) {
        constexpr int L = kSmTile * kSmKR / kSmThreads;
        double v[L];
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int e = tid + s * kSmThreads;
            const int i = e / kSmKR, kk = e % kSmKR;
            const int64_t row = min(row0 + i, m - 1), q = min(kr0 + kk, k - 1);
            v[s] = (double)a[row * k + q];
        }
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int e = tid + s * kSmThreads;
            const int i = e / kSmKR, kk = e % kSmKR;
            double x = (row0 + i < m && kr0 + kk < k) ? v[s] : 0.0;
            if (scale) x = sm_scaled(x, rs[i], rinv[i]);
            ar[i * (kSmKR + 1) + kk] = x;
        }
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int e = tid + s * kSmThreads;
            const int kk = e / kSmTile, j = e % kSmTile;
            const int64_t col = min(col0 + j, n - 1), q = min(kr0 + kk, k - 1);
            v[s] = (double)b[q * n + col];
        }
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int e = tid + s * kSmThreads;
            const int kk = e / kSmTile, j = e % kSmTile;
            double y = (col0 + j < n && kr0 + kk < k) ? v[s] : 0.0;
            if (scale) y = sm_scaled(y, cs[j], cinv[j]);
            br[kk * kSmTile + j] = y;
        }
    };

    // r_i = max_k A_ik and c_j = max_k B_kj of the tile: thread t keeps the
    // maximum of row t / 8 over inner indices = t (mod 8) and of column t % 32
    // over inner indices = t / 32 (mod 8); the 8 parts are combined at the end
    double rpart = 0.0, cpart = 0.0;
    for (int64_t kr0 = 0; kr0 < k; kr0 += kSmKR) {
        if (kr0 > 0) __syncthreads();
        load_raw(kr0, false);
        __syncthreads();
        const int ri = tid / 8, rp = tid % 8;
        const int cj = tid % kSmTile, cp = tid / kSmTile;
        double rv[kSmKR / 8], cv[kSmKR / 8];
#pragma unroll
        for (int s = 0; s < kSmKR / 8; ++s) {
            rv[s] = ar[ri * (kSmKR + 1) + rp + 8 * s];
            cv[s] = br[(cp + 8 * s) * kSmTile + cj];
        }
#pragma unroll
        for (int s = 0; s < kSmKR / 8; ++s) {
            rpart = fmax(rpart, rv[s]);
            cpart = fmax(cpart, cv[s]);
        }
    }
    // rows: the 8 parts are 8 consecutive lanes
    for (int off = 4; off > 0; off >>= 1) rpart = fmax(rpart, __shfl_xor(rpart, off, 64));
    if (tid % 8 == 0) {
        rs[tid / 8] = rpart;
        rinv[tid / 8] = rpart >= DBL_MIN ? 1.0 / rpart : 0.0;
    }
    // columns: the 8 parts are 32 threads apart; combine them through the
    // power buffer (free until the first p)
    ap[tid] = cpart;
    __syncthreads();
    if (tid < kSmTile) {
        double mx = ap[tid];
        for (int q = 1; q < kSmThreads / kSmTile; ++q) mx = fmax(mx, ap[tid + q * kSmTile]);
        cs[tid] = mx;
        cinv[tid] = mx >= DBL_MIN ? 1.0 / mx : 0.0;
    }
    __syncthreads();

    // this thread's entries: rows 2 ty + di, columns 2 tx + dj; bit 2 di + dj
    // of `open` is set while the entry has no p yet (entries outside C never)
    const int tx = tid % 16, ty = tid / 16;
    uint32_t open = 0;
    for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj)
            if (row0 + 2 * ty + di < m && col0 + 2 * tx + dj < n) open |= 1u << (2 * di + dj);

    // the tile stays in LDS for every p when the inner dimension fits; it is
    // scaled in place once (the scaled inputs a / r, b / c of H')
    const bool resident = k <= kSmKR;
    if (resident) {
        constexpr int L = kSmTile * kSmKR / kSmThreads;
#pragma unroll
        for (int s = 0; s < L; ++s) {
            const int e = tid + s * kSmThreads;
            const int i = e / kSmKR, kk = e % kSmKR;
            ar[i * (kSmKR + 1) + kk] = sm_scaled(ar[i * (kSmKR + 1) + kk], rs[i], rinv[i]);
            const int kb = e / kSmTile, j = e % kSmTile;
            br[kb * kSmTile + j] = sm_scaled(br[kb * kSmTile + j], cs[j], cinv[j]);
        }
        __syncthreads();
    }
    int visited = 0;
    for (int q = spec.n - 1; q >= 0; --q) {  // the largest p first
        ++visited;
        const int p = spec.p[q];
        double acc00 = 0.0, acc01 = 0.0, acc10 = 0.0, acc11 = 0.0;
        for (int64_t kr0 = 0; kr0 < k; kr0 += kSmKR) {
            if (!resident) {
                load_raw(kr0, true);
                __syncthreads();
            }
            const int kr_len = k - kr0 < kSmKR ? (int)(k - kr0) : kSmKR;
            for (int kc = 0; kc < kr_len; kc += kSmK) {
                // stage (a / r)^p and (b / c)^p of inner indices kc .. kc + 31:
                // this thread's 8 values raised together by binary powering
                constexpr int SE = kSmTile * kSmK / kSmThreads;
                double xa[SE], xb[SE], ya[SE], yb[SE];
#pragma unroll
                for (int t = 0; t < SE; ++t) {
                    const int e = tid + t * kSmThreads;
                    xa[t] = ar[(e / kSmK) * (kSmKR + 1) + kc + e % kSmK];
                    xb[t] = br[(kc + e / kSmTile) * kSmTile + e % kSmTile];
                    ya[t] = 1.0;
                    yb[t] = 1.0;
                }
                for (int pp = p; pp; pp >>= 1) {
                    if (pp & 1) {
#pragma unroll
                        for (int t = 0; t < SE; ++t) {
                            ya[t] *= xa[t];
                            yb[t] *= xb[t];
                        }
                    }
#pragma unroll
                    for (int t = 0; t < SE; ++t) {
                        xa[t] *= xa[t];
                        xb[t] *= xb[t];
                    }
                }
#pragma unroll
                for (int t = 0; t < SE; ++t) {
                    const int e = tid + t * kSmThreads;
                    ap[(e / kSmK) * (kSmK + 1) + e % kSmK] = ya[t];
                    bp[(e / kSmTile) * kSmTile + e % kSmTile] = yb[t];
                }
                __syncthreads();
#pragma unroll
                for (int kk = 0; kk < kSmK; ++kk) {
                    const double a0 = ap[(2 * ty) * (kSmK + 1) + kk], a1 = ap[(2 * ty + 1) * (kSmK + 1) + kk];
                    const double2 bv = *(const double2*)&bp[kk * kSmTile + 2 * tx];
                    acc00 = fma(a0, bv.x, acc00);
                    acc01 = fma(a0, bv.y, acc01);
                    acc10 = fma(a1, bv.x, acc10);
                    acc11 = fma(a1, bv.y, acc11);
                }
                __syncthreads();
            }
        }
        const bool last = q == 0;
        const double accs[4] = {acc00, acc01, acc10, acc11};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (!(open & (1u << e))) continue;
            const double S = accs[e];
            const bool stable = S >= spec.tau;
            if (!stable && !last) continue;
            open &= ~(1u << e);
            const int li = 2 * ty + (e >> 1), lj = 2 * tx + (e & 1);
            const double root = p == 1 ? S : (S > 0.0 ? exp(log(S) / (double)p) : 0.0);
            double v = rs[li] * cs[lj] * root * spec.corr[q];
            if (spec.clamp) v = fmin(v, 1.0);
            const int64_t o = (bi * m + row0 + li) * n + col0 + lj;
            C[o] = (TO)v;
            if (pstar) pstar[o] = stable ? (uint8_t)q : (uint8_t)MT_PSTAR_NONE;
        }
        if (!__syncthreads_or(open != 0)) break;
    }
    if (work && tid == 0) {
        // timed launch: 2 k flops per output entry of the tile and p visited,
        // and the end (every wave has passed the last vote)
        const int64_t rows = m - row0 < kSmTile ? m - row0 : kSmTile;
        const int64_t cols = n - col0 < kSmTile ? n - col0 : kSmTile;
        atomicAdd(work, (unsigned long long)(2 * rows * cols * k * visited));
        timing_span_end(work);
    }
}

}  // namespace

hipError_t launch_small_product_f64(const void* A, const void* B, int in_f64, int64_t b, int64_t m, int64_t k,
                                    int64_t n, const SmallSpec& spec, void* C, int out_f64, uint8_t* pstar,
                                    hipStream_t st) {
    if (b <= 0 || m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kSmTile - 1) / kSmTile), (unsigned)((m + kSmTile - 1) / kSmTile),
                    (unsigned)b);
    // the dynamic-LDS limit is a per-device attribute of each instance
    static std::atomic<uint64_t> attr_set[4];
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    const int inst = (in_f64 ? 2 : 0) + (out_f64 ? 1 : 0);
    if (!(attr_set[inst].load() & bit)) {
        const void* fn = in_f64 ? (out_f64 ? (const void*)mt_small_product_f64_kernel<double, double>
                                           : (const void*)mt_small_product_f64_kernel<double, float>)
                                : (out_f64 ? (const void*)mt_small_product_f64_kernel<float, double>
                                           : (const void*)mt_small_product_f64_kernel<float, float>);
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kSmLdsBytes);
        if (e != hipSuccess) return e;
        attr_set[inst].fetch_or(bit);
    }
    timing_before("mt_small_product_f64", st);
    unsigned long long* work = timing_work_slot();
#define MT_SMALL(TS, TO)                                                                             \
    hipLaunchKernelGGL((mt_small_product_f64_kernel<TS, TO>), grid, dim3(kSmThreads), kSmLdsBytes, st,    \
                       (const TS*)A, (const TS*)B, m, k, n, spec, (TO*)C, pstar, work)
    if (in_f64) {
        if (out_f64) MT_SMALL(double, double); else MT_SMALL(double, float);
    } else {
        if (out_f64) MT_SMALL(float, double); else MT_SMALL(float, float);
    }
#undef MT_SMALL
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
