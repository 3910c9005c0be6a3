// Adjoint of the p-norm estimate with p* held fixed per entry: the per-entry
// weights that enter the two gradient products, and the p* histogram that
// lets the adjoint GEMMs skip the p no entry uses.
//
// With C' = C / (r_i c_j) and p = p*_ij (the smallest p of the family where
// no p was stable), the derivative of C_ij = (sum_k A_ik^p B_kj^p)^(1/p) gives
//   dL/dA = sum_p A'^(p-1) .* (Gt_p  B'^p^T),  Gt_p  = [p* = p] G c_j C'^(1-p)
//   dL/dB = sum_p B'^(p-1) .* (A'^p^T Gt'_p),  Gt'_p = [p* = p] G r_i C'^(1-p)
// (the paper notes the p-norm rings are continuous and differentiable,
// Sec. 4).  Entries with C = 0 contribute nothing.
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kThreads = 256;

__device__ inline uint16_t bf16_rne(float x) {
    // Round to nearest even on the bit pattern (finite x).
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_float(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// hist[q] = number of entries whose p is family index q (MT_PSTAR_NONE -> 0).
__global__ __launch_bounds__(kThreads) void mt_pstar_hist_kernel(const uint8_t* __restrict__ ps,
                                                                 int64_t total, int n_p,
                                                                 int32_t* __restrict__ hist) {
    __shared__ int32_t h[MT_MAX_P];
    for (int i = threadIdx.x; i < MT_MAX_P; i += kThreads) h[i] = 0;
    __syncthreads();
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        int q = ps[e];
        if (q == MT_PSTAR_NONE || q >= n_p) q = 0;
        atomicAdd(&h[q], 1);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n_p; i += kThreads)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

// Per batch item, the binary exponents of the largest row scale and of the
// largest column scale: ex[bi] = e with max_i r_i < 2^e, ex[b + bi] the
// same for c.  The BF16 adjoint planes carry r_i / 2^ex and c_j / 2^ex, which
// lie in (0, 1] whatever the range of the inputs, and the adjoint GEMMs
// multiply their sums back by 2^ex.
__global__ __launch_bounds__(kThreads) void mt_scale_exp_kernel(const double* __restrict__ r,
                                                                const double* __restrict__ c, int64_t m,
                                                                int64_t n, int32_t* __restrict__ ex) {
    __shared__ double red[2][kThreads / 64];
    const int64_t bi = blockIdx.x;
    double mr = 0.0, mc = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += kThreads) mr = fmax(mr, r[bi * m + i]);
    for (int64_t j = threadIdx.x; j < n; j += kThreads) mc = fmax(mc, c[bi * n + j]);
    for (int off = 32; off > 0; off >>= 1) {
        mr = fmax(mr, __shfl_xor(mr, off, 64));
        mc = fmax(mc, __shfl_xor(mc, off, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = mr;
        red[1][threadIdx.x >> 6] = mc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) {
            mr = fmax(mr, red[0][w]);
            mc = fmax(mc, red[1][w]);
        }
        int er = 0, ec = 0;
        if (mr > 0.0) (void)frexp(mr, &er);
        if (mc > 0.0) (void)frexp(mc, &ec);
        ex[bi] = er;
        ex[gridDim.x + bi] = ec;
    }
}

// Adjoint planes for one 64 x 64 (i, j) tile of one batch item.
//   XA: [b][plane][m_pad][n_kpad]  Gt_p   (rows i, inner j)  -> dA product
//   YB: [b][plane][n_pad][m_kpad]  Gt'_p^T (rows j, inner i) -> dB product
// For the BF16 path each p has a hi and a lo plane (planes 2q, 2q + 1);
// for FP64 one plane (q).  Planes of p that no entry uses are not written.
template <typename T, bool kBf16>
__global__ __launch_bounds__(kThreads) void mt_adjoint_prep_kernel(
    const T* __restrict__ G, const T* __restrict__ C, const uint8_t* __restrict__ pstar,
    const double* __restrict__ r, const double* __restrict__ c, const int32_t* __restrict__ ex, int64_t m,
    int64_t n, AdjPrepSpec spec, const int32_t* __restrict__ hist, void* __restrict__ XA,
    void* __restrict__ YB) {
    __shared__ double gw[64][65];  // G * C'^(1-p), 0 where C = 0 or outside
    __shared__ uint8_t qq[64][68];  // family index of p*
    __shared__ double rsh[64], csh[64];  // r_i and c_j as the planes take them (/ 2^ex on the BF16 path)
    __shared__ double rm[64], cm[64];    // mantissas of r_i and c_j
    __shared__ int re[64], ce[64];       // and their exponents
    const int64_t bi = blockIdx.z;
    const int64_t i0 = (int64_t)blockIdx.y * 64, j0 = (int64_t)blockIdx.x * 64;
    const int64_t base = bi * m * n;
    if (threadIdx.x < 128) {
        const bool is_r = threadIdx.x < 64;
        const int t = threadIdx.x & 63;
        const int64_t idx = (is_r ? i0 : j0) + t;
        const double v = is_r ? (idx < m ? r[bi * m + idx] : 0.0) : (idx < n ? c[bi * n + idx] : 0.0);
        int e = 0;
        const double mv = v > 0.0 ? frexp(v, &e) : 0.0;
        const double vs = ex ? ldexp(v, -ex[(is_r ? 0 : gridDim.z) + bi]) : v;
        if (is_r) {
            rsh[t] = vs;
            rm[t] = mv;
            re[t] = e;
        } else {
            csh[t] = vs;
            cm[t] = mv;
            ce[t] = e;
        }
    }
    __syncthreads();

    // 1. per-entry weights (FP64), coalesced along j
    for (int e = threadIdx.x; e < 64 * 64; e += kThreads) {
        const int ii = e >> 6, jj = e & 63;
        const int64_t i = i0 + ii, j = j0 + jj;
        double w = 0.0;
        int q = 0;
        if (i < m && j < n) {
            const int64_t o = base + i * n + j;
            const int code = pstar[o];
            q = (code == MT_PSTAR_NONE || code >= spec.n_p) ? 0 : code;
            // C' = C / (r_i c_j), formed as (C 2^-(e_r + e_c)) / (m_r m_c)
            // so that r_i c_j itself never has to be representable
            const double mrc = rm[ii] * cm[jj];
            const double cs = mrc > 0.0 ? ldexp((double)C[o], -(re[ii] + ce[jj])) / mrc : 0.0;
            if (cs > 0.0) {
                const int p = spec.p[q];
                w = (double)G[o] * (p == 1 ? 1.0 : exp((double)(1 - p) * log(cs)));  // G C'^(1-p)
            }
        }
        gw[ii][jj] = w;
        qq[ii][jj] = (uint8_t)q;
    }
    __syncthreads();

    // 2. XA planes (rows i, inner j): 8 consecutive j per task
    for (int task = threadIdx.x; task < 64 * 8; task += kThreads) {
        const int ii = task >> 3, ch = task & 7;
        const int64_t i = i0 + ii, j = j0 + ch * 8;
        if (i >= spec.xa_rows_pad || j >= spec.xa_cols_pad) continue;
        for (int q = 0; q < spec.n_p; ++q) {
            if (hist[q] == 0) continue;
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = qq[ii][ch * 8 + t] == q ? gw[ii][ch * 8 + t] * csh[ch * 8 + t] : 0.0;
            if (kBf16) {
                uint16_t* pl = (uint16_t*)XA + ((bi * spec.planes + 2 * q) * spec.xa_rows_pad + i) * spec.xa_cols_pad + j;
                u32x4 hi, lo;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float f0 = (float)v[2 * t], f1 = (float)v[2 * t + 1];
                    const uint16_t h0 = bf16_rne(f0), h1 = bf16_rne(f1);
                    hi[t] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    lo[t] = (uint32_t)bf16_rne(f0 - bf16_to_float(h0)) |
                            ((uint32_t)bf16_rne(f1 - bf16_to_float(h1)) << 16);
                }
                *(u32x4*)pl = hi;
                *(u32x4*)(pl + spec.xa_rows_pad * spec.xa_cols_pad) = lo;
            } else {
                double* pl = (double*)XA + ((bi * spec.planes + q) * spec.xa_rows_pad + i) * spec.xa_cols_pad + j;
#pragma unroll
                for (int t = 0; t < 8; t += 2) *(double2*)(pl + t) = double2{v[t], v[t + 1]};
            }
        }
    }

    // 3. YB planes (rows j, inner i): 8 consecutive i per task (transposed)
    for (int task = threadIdx.x; task < 64 * 8; task += kThreads) {
        const int jj = task >> 3, ch = task & 7;
        const int64_t j = j0 + jj, i = i0 + ch * 8;
        if (j >= spec.yb_rows_pad || i >= spec.yb_cols_pad) continue;
        for (int q = 0; q < spec.n_p; ++q) {
            if (hist[q] == 0) continue;
            double v[8];
#pragma unroll
            for (int t = 0; t < 8; ++t) v[t] = qq[ch * 8 + t][jj] == q ? gw[ch * 8 + t][jj] * rsh[ch * 8 + t] : 0.0;
            if (kBf16) {
                uint16_t* pl = (uint16_t*)YB + ((bi * spec.planes + 2 * q) * spec.yb_rows_pad + j) * spec.yb_cols_pad + i;
                u32x4 hi, lo;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float f0 = (float)v[2 * t], f1 = (float)v[2 * t + 1];
                    const uint16_t h0 = bf16_rne(f0), h1 = bf16_rne(f1);
                    hi[t] = (uint32_t)h0 | ((uint32_t)h1 << 16);
                    lo[t] = (uint32_t)bf16_rne(f0 - bf16_to_float(h0)) |
                            ((uint32_t)bf16_rne(f1 - bf16_to_float(h1)) << 16);
                }
                *(u32x4*)pl = hi;
                *(u32x4*)(pl + spec.yb_rows_pad * spec.yb_cols_pad) = lo;
            } else {
                double* pl = (double*)YB + ((bi * spec.planes + q) * spec.yb_rows_pad + j) * spec.yb_cols_pad + i;
#pragma unroll
                for (int t = 0; t < 8; t += 2) *(double2*)(pl + t) = double2{v[t], v[t + 1]};
            }
        }
    }
}

}  // namespace

hipError_t launch_pstar_hist(const uint8_t* ps, int64_t total, int n_p, int32_t* hist,
                             hipStream_t st) {
    if (total <= 0) return hipSuccess;
    int64_t g = (total + kThreads * 16 - 1) / (kThreads * 16);
    if (g > 2048) g = 2048;
    timing_before("mt_pstar_hist", st);
    hipLaunchKernelGGL(mt_pstar_hist_kernel, dim3((unsigned)g), dim3(kThreads), 0, st, ps, total, n_p, hist);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_scale_exp(const double* r, const double* c, int64_t b, int64_t m, int64_t n, int32_t* ex,
                            hipStream_t st) {
    if (b <= 0) return hipSuccess;
    timing_before("mt_scale_exp", st);
    hipLaunchKernelGGL(mt_scale_exp_kernel, dim3((unsigned)b), dim3(kThreads), 0, st, r, c, m, n, ex);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_adjoint_prep(const void* G, const void* C, const uint8_t* pstar, int io_f64,
                               const double* r, const double* c, const int32_t* ex, int64_t b, int64_t m,
                               int64_t n, const AdjPrepSpec& spec, const int32_t* hist, int bf16, void* XA,
                               void* YB, hipStream_t st) {
    const int64_t rows_cover = spec.xa_rows_pad > spec.yb_cols_pad ? spec.xa_rows_pad : spec.yb_cols_pad;
    const int64_t cols_cover = spec.xa_cols_pad > spec.yb_rows_pad ? spec.xa_cols_pad : spec.yb_rows_pad;
    const dim3 grid((unsigned)((cols_cover + 63) / 64), (unsigned)((rows_cover + 63) / 64), (unsigned)b);
#define MT_PREP(T, BF)                                                                              \
    hipLaunchKernelGGL((mt_adjoint_prep_kernel<T, BF>), grid, dim3(kThreads), 0, st, (const T*)G,  \
                       (const T*)C, pstar, r, c, ex, m, n, spec, hist, XA, YB)
    timing_before("mt_adjoint_prep", st);
    if (io_f64) {
        if (bf16) MT_PREP(double, true); else MT_PREP(double, false);
    } else {
        if (bf16) MT_PREP(float, true); else MT_PREP(float, false);
    }
#undef MT_PREP
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
