// Exact (max, x) matrix product on the vector ALUs (Alg. 2, Sec. 2.2):
// E_ij = max_k A_ik B_kj, E starting at 0.  Products are formed in the input
// precision (one rounding), the max is exact.  Used to measure the error of
// the estimate and as the exact-product throughput beside it.
//
// 64 x 64 output tile per 256-thread workgroup, 4 x 4 outputs per thread,
// K step 16 staged through LDS.
#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;
constexpr int TM = 64, TK = 16;

template <typename T>
__global__ __launch_bounds__(kThreads) void mt_exact_maxtimes_kernel(const T* __restrict__ A,
                                                                     const T* __restrict__ B,
                                                                     T* __restrict__ E, int64_t m,
                                                                     int64_t k, int64_t n) {
    __shared__ T As[TK][TM + 1];
    __shared__ T Bs[TK][TM];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t bi = blockIdx.z;
    const int64_t i0 = (int64_t)blockIdx.y * TM, j0 = (int64_t)blockIdx.x * TM;
    const T* a = A + bi * m * k;
    const T* b = B + bi * k * n;
    T acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
    for (int64_t k0 = 0; k0 < k; k0 += TK) {
        for (int e = tid; e < TM * TK; e += kThreads) {
            const int r = e / TK, kk = e % TK;  // A tile: 64 rows x 16 k, read along k
            const int64_t gi = i0 + r, gk = k0 + kk;
            As[kk][r] = (gi < m && gk < k) ? a[gi * k + gk] : T(0);
            const int kb = e / TM, c = e % TM;  // B tile: 16 k x 64 cols, read along n
            const int64_t gkb = k0 + kb, gj = j0 + c;
            Bs[kb][c] = (gkb < k && gj < n) ? b[gkb * n + gj] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            T av[4], bv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) av[i] = As[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmax(acc[i][j], av[i] * bv[j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t gi = i0 + ty * 4 + i;
        if (gi >= m) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gj = j0 + tx * 4 + j;
            if (gj < n) E[(bi * m + gi) * n + gj] = acc[i][j];
        }
    }
}

}  // namespace

hipError_t launch_exact_maxtimes(const void* A, const void* B, int f64, int64_t b, int64_t m,
                                 int64_t k, int64_t n, void* E, hipStream_t st) {
    if (b <= 0 || m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)((m + TM - 1) / TM), (unsigned)b);
    timing_before("mt_exact_maxtimes", st);
    if (f64)
        hipLaunchKernelGGL(mt_exact_maxtimes_kernel<double>, grid, dim3(kThreads), 0, st,
                           (const double*)A, (const double*)B, (double*)E, m, k, n);
    else
        hipLaunchKernelGGL(mt_exact_maxtimes_kernel<float>, grid, dim3(kThreads), 0, st,
                           (const float*)A, (const float*)B, (float*)E, m, k, n);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
