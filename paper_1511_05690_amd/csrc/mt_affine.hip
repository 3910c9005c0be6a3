// Exact distances from a few sources and the affine correction of the APSP
// estimate (Sec. 4: exact distances for a small number of vertex pairs, e.g.
// by Dijkstra's algorithm, and an affine model fitted on them to correct the
// estimate's numerical error).
//
// Exact rows: Bellman-Ford on the dense weights in FP64.  D_0[q][v] is the
// edge weight from source q to v (0 at the source); a round forms
// D'[q][v] = min(D[q][v], min_u D[q][u] + W[u][v]) and flags any change.
// After at most n - 1 rounds nothing changes and D holds the shortest-path
// distances (weights are nonnegative: no negative cycles).
//
// Fit: least squares d_exact = a d_est + b over the pairs (source, v),
// v != source, where both are finite, in two passes (means, then centred
// sums) with per-block partials added in a fixed order.

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;
constexpr int TM = 64, TK = 16;
constexpr int kFitBlocks = 256;

// A source outside 0 .. n - 1 gives a row of +inf and sets *bad.
__global__ __launch_bounds__(kThreads) void exact_rows_init_kernel(const float* __restrict__ W, int64_t n,
                                                                   const int32_t* __restrict__ src, int32_t nsrc,
                                                                   double* __restrict__ D, int32_t* __restrict__ bad) {
    const int64_t total = (int64_t)nsrc * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = e / n, v = e % n;
        const int64_t s = src[q];
        if (s < 0 || s >= n) {
            D[e] = INFINITY;
            atomicOr(bad, 1);
            continue;
        }
        D[e] = v == s ? 0.0 : (double)W[s * n + v];
    }
}

// One round: Dn = min(D, D (min,+) W) for a 64 x 64 block of (source, v);
// *changed |= any entry decreased.
__global__ __launch_bounds__(kThreads) void exact_rows_round_kernel(const double* __restrict__ D,
                                                                    const float* __restrict__ W, int64_t n,
                                                                    int32_t nsrc, double* __restrict__ Dn,
                                                                    int32_t* __restrict__ changed) {
    __shared__ double Ds[TK][TM + 1];
    __shared__ double Ws[TK][TM];
    const int tid = threadIdx.x;
    const int tx = tid & 15, ty = tid >> 4;
    const int64_t q0 = (int64_t)blockIdx.y * TM, v0 = (int64_t)blockIdx.x * TM;
    double acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = INFINITY;
    for (int64_t k0 = 0; k0 < n; k0 += TK) {
        for (int e = tid; e < TM * TK; e += kThreads) {
            const int r = e / TK, kk = e % TK;
            const int64_t gq = q0 + r, gk = k0 + kk;
            Ds[kk][r] = (gq < nsrc && gk < n) ? D[gq * n + gk] : INFINITY;
            const int kb = e / TM, c = e % TM;
            const int64_t gkb = k0 + kb, gv = v0 + c;
            Ws[kb][c] = (gkb < n && gv < n) ? (double)W[gkb * n + gv] : INFINITY;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; ++kk) {
            double dv[4], wv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) dv[i] = Ds[kk][ty * 4 + i];
#pragma unroll
            for (int j = 0; j < 4; ++j) wv[j] = Ws[kk][tx * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmin(acc[i][j], dv[i] + wv[j]);
        }
        __syncthreads();
    }
    bool any = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t gq = q0 + ty * 4 + i;
        if (gq >= nsrc) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t gv = v0 + tx * 4 + j;
            if (gv >= n) continue;
            const double old = D[gq * n + gv];
            const double nv = acc[i][j] < old ? acc[i][j] : old;
            any |= nv < old;
            Dn[gq * n + gv] = nv;
        }
    }
    if (__any(any) && (tid & 63) == 0) atomicOr(changed, 1);
}

// Pair p of the fit: source q = p / n, vertex v = p % n.
template <typename T>
__device__ __forceinline__ bool fit_pair(const T* Dest, int64_t n, const int32_t* src, const double* ex, int64_t p,
                                         double& x, double& y) {
    const int64_t q = p / n, v = p % n;
    const int64_t s = src[q];
    if (v == s || s < 0 || s >= n) return false;  // a source outside the graph has no pairs
    x = (double)Dest[s * n + v];
    y = ex[p];
    return x < INFINITY && y < INFINITY;
}

// Pass 1 (mode 0): partial count, sum x, sum y.  Pass 2 (mode 1), around the
// means in stats[0..2]: partial sum (x - mx)^2, sum (x - mx)(y - my).
template <typename T>
__global__ __launch_bounds__(kThreads) void fit_partial_kernel(const T* __restrict__ Dest, int64_t n,
                                                               const int32_t* __restrict__ src, int32_t nsrc,
                                                               const double* __restrict__ ex, int mode,
                                                               const double* __restrict__ stats,
                                                               double* __restrict__ part) {
    __shared__ double red[3][kThreads];
    const int tid = threadIdx.x;
    const int64_t total = (int64_t)nsrc * n;
    const int64_t per = (total + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min<int64_t>(lo + per, total);
    double a0 = 0, a1 = 0, a2 = 0;
    const double mx = mode ? stats[1] : 0.0, my = mode ? stats[2] : 0.0;
    for (int64_t p = lo + tid; p < hi; p += kThreads) {
        double x, y;
        if (!fit_pair(Dest, n, src, ex, p, x, y)) continue;
        if (mode == 0) {
            a0 += 1.0;
            a1 += x;
            a2 += y;
        } else {
            a1 += (x - mx) * (x - mx);
            a2 += (x - mx) * (y - my);
        }
    }
    red[0][tid] = a0;
    red[1][tid] = a1;
    red[2][tid] = a2;
    __syncthreads();
    for (int d = kThreads / 2; d > 0; d >>= 1) {
        if (tid < d)
            for (int c = 0; c < 3; ++c) red[c][tid] += red[c][tid + d];
        __syncthreads();
    }
    if (tid < 3) part[blockIdx.x * 3 + tid] = red[tid][0];
}

// Adds the block partials in order.  mode 0: stats = (count, mean x, mean y);
// mode 1: ab = (a, b) (a = 1, b = 0 without pairs; a = 1 when every x is
// equal).
__global__ void fit_finish_kernel(const double* __restrict__ part, int nblocks, int mode, double* __restrict__ stats,
                                  double* __restrict__ ab) {
    if (threadIdx.x != 0) return;
    double s0 = 0, s1 = 0, s2 = 0;
    for (int b = 0; b < nblocks; ++b) {
        s0 += part[b * 3 + 0];
        s1 += part[b * 3 + 1];
        s2 += part[b * 3 + 2];
    }
    if (mode == 0) {
        stats[0] = s0;
        stats[1] = s0 > 0 ? s1 / s0 : 0.0;
        stats[2] = s0 > 0 ? s2 / s0 : 0.0;
        return;
    }
    const double cnt = stats[0], mx = stats[1], my = stats[2];
    double a = 1.0, b = 0.0;
    if (cnt > 0) {
        if (s1 > 0) a = s2 / s1;
        b = my - a * mx;
    }
    ab[0] = a;
    ab[1] = b;
}

// D <- max(0, a D + b) on every finite off-diagonal entry.
template <typename T>
__global__ __launch_bounds__(kThreads) void affine_apply_kernel(T* __restrict__ D, int64_t n,
                                                                const double* __restrict__ ab) {
    const double a = ab[0], b = ab[1];
    const int64_t total = n * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const double d = (double)D[e];
        if (e / n == e % n || !(d < INFINITY)) continue;
        const double c = a * d + b;
        D[e] = (T)(c > 0.0 ? c : 0.0);
    }
}

unsigned grid_of(int64_t items) {
    int64_t g = (items + kThreads - 1) / kThreads;
    if (g > 4096) g = 4096;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace

// Workspace: the second row buffer, then kExactRowsChunk round flags and
// the bad-source flag.
size_t exact_rows_workspace(int64_t n, int32_t nsrc) {
    const size_t rows = ((size_t)nsrc * n * 8 + 255) / 256 * 256;
    return rows + 256 * (((kExactRowsChunk + 1) * 4 + 255) / 256);
}

hipError_t launch_exact_rows(const float* W, int64_t n, const int32_t* src, int32_t nsrc, double* D, uint8_t* ws,
                             hipStream_t st, int64_t* rounds_out, int32_t* bad_out) {
    *rounds_out = 0;
    *bad_out = 0;
    if (n <= 0 || nsrc <= 0) return hipSuccess;
    double* Db = (double*)ws;
    int32_t* flags = (int32_t*)(ws + ((size_t)nsrc * n * 8 + 255) / 256 * 256);
    int32_t* bad = flags + kExactRowsChunk;
    hipError_t e = launch_fill_zero_u32(bad, 1, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(exact_rows_init_kernel, dim3(grid_of((int64_t)nsrc * n)), dim3(kThreads), 0, st, W, n, src,
                       nsrc, D, bad);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = hipMemcpyAsync(bad_out, bad, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
    if (*bad_out) return hipSuccess;
    const dim3 grid((unsigned)((n + TM - 1) / TM), (unsigned)((nsrc + TM - 1) / TM));
    double* cur = D;
    double* nxt = Db;
    int64_t r = 0;
    const int64_t max_rounds = n > 1 ? n - 1 : 0;
    while (r < max_rounds) {
        const int chunk = (int)std::min<int64_t>(kExactRowsChunk, max_rounds - r);
        e = launch_fill_zero_u32(flags, chunk, st);
        if (e != hipSuccess) return e;
        timing_before("mt_exact_rows", st);
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(exact_rows_round_kernel, grid, dim3(kThreads), 0, st, cur, W, n, nsrc, nxt, flags + c);
            std::swap(cur, nxt);
        }
        timing_after(st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        r += chunk;
        int32_t last = 1;
        if ((e = hipMemcpyAsync(&last, flags + chunk - 1, 4, hipMemcpyDeviceToHost, st)) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        if (!last) break;  // the last round changed nothing: converged
    }
    *rounds_out = r;
    if (cur != D) {
        if ((e = hipMemcpyAsync(D, cur, (size_t)nsrc * n * 8, hipMemcpyDeviceToDevice, st)) != hipSuccess) return e;
    }
    return hipSuccess;
}

size_t affine_workspace() { return 256 * (((size_t)kFitBlocks * 3 * 8 + 255) / 256) + 256; }

hipError_t launch_affine_correct(void* D, int f64, int64_t n, const int32_t* src, int32_t nsrc, const double* ex,
                                 double* ab, uint8_t* ws, int apply, hipStream_t st) {
    double* part = (double*)ws;
    double* stats = (double*)(ws + 256 * (((size_t)kFitBlocks * 3 * 8 + 255) / 256));
    timing_before("mt_affine", st);
    for (int mode = 0; mode < 2; ++mode) {
        if (f64)
            hipLaunchKernelGGL(fit_partial_kernel<double>, dim3(kFitBlocks), dim3(kThreads), 0, st, (const double*)D,
                               n, src, nsrc, ex, mode, stats, part);
        else
            hipLaunchKernelGGL(fit_partial_kernel<float>, dim3(kFitBlocks), dim3(kThreads), 0, st, (const float*)D, n,
                               src, nsrc, ex, mode, stats, part);
        hipLaunchKernelGGL(fit_finish_kernel, dim3(1), dim3(64), 0, st, part, kFitBlocks, mode, stats, ab);
    }
    if (apply) {
        if (f64)
            hipLaunchKernelGGL(affine_apply_kernel<double>, dim3(grid_of(n * n)), dim3(kThreads), 0, st, (double*)D,
                               n, ab);
        else
            hipLaunchKernelGGL(affine_apply_kernel<float>, dim3(grid_of(n * n)), dim3(kThreads), 0, st, (float*)D, n,
                               ab);
    }
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
