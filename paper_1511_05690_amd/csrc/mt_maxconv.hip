// Max-convolution (Sec. 1).
//
// Estimate: z[t] = max_i x[i] y[t - i] from the norm sequence
// S_p[t] = (x'^p * y'^p)[t] with x' = x / max x, y' = y / max y (terms in
// [0, 1], the scaling of Sec. 2.1), computed by FFT convolution in FP64 (the
// fast ring kernel H, Sec. 2.1, whose threshold there is tau = 1e-12); per
// index the largest p of the family with S_p >= tau, and
// z = max x max y S_{p*}^(1/p*).
//
// One workgroup per batch item runs the whole family in LDS: for each p,
// largest first, it loads x'^p + i y'^p at bit-reversed positions, runs an
// in-place radix-2 FFT of N = 2^ceil(log2(n + m - 1)) points, separates the
// two real transforms (X_k = (Z_k + conj Z_{N-k}) / 2, Y_k = (Z_k - conj
// Z_{N-k}) / 2i), multiplies them, and transforms back as the forward FFT of
// the conjugate.  Indices decided at a larger p keep their value and the
// group stops once every index of its item is decided.  LDS: 16 N bytes of
// data and 8 N of twiddles, so N <= 4096 (96 KB).
//
// Exact: z[t] = max_i x[i] y[t - i] by the definition, one thread per output
// index, products in the input precision.

#include <atomic>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kConvMaxThreads = 512;
// each thread owns the output indices tid + j * blockDim.x, one bit of a mask each
static_assert(kMaxConvN / kConvMaxThreads <= 32, "decided mask holds 32 indices");

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__device__ __forceinline__ double ipow_d(double v, int p) {
    double r = 1.0;
    while (p) {
        if (p & 1) r *= v;
        v *= v;
        p >>= 1;
    }
    return r;
}

__device__ __forceinline__ int brev_n(int t, int logN) { return (int)(__brev((unsigned)t) >> (32 - logN)); }

// In-place radix-2 decimation in time: input in bit-reversed order, output in
// natural order; tw[k] = exp(-2 pi i k / N), k < N / 2.
__device__ void fft_radix2(double2* buf, const double2* tw, int logN) {
    const int N = 1 << logN;
    for (int s = 1; s <= logN; ++s) {
        const int h = 1 << (s - 1);
        const int step = N >> s;
        for (int f = threadIdx.x; f < N / 2; f += blockDim.x) {
            const int j = f & (h - 1);
            const int i0 = ((f >> (s - 1)) << s) + j, i1 = i0 + h;
            const double2 t = cmul(tw[j * step], buf[i1]);
            const double2 a = buf[i0];
            buf[i0] = make_double2(a.x + t.x, a.y + t.y);
            buf[i1] = make_double2(a.x - t.x, a.y - t.y);
        }
        __syncthreads();
    }
}

template <typename T>
__global__ __launch_bounds__(kConvMaxThreads) void mt_maxconv_kernel(const T* __restrict__ x,
                                                                     const T* __restrict__ y, int64_t n,
                                                                     int64_t m, int logN, MaxconvSpec spec,
                                                                     T* __restrict__ z,
                                                                     uint8_t* __restrict__ pstar) {
    extern __shared__ double2 lds[];
    const int N = 1 << logN;
    double2* buf = lds;
    double2* tw = lds + N;
    __shared__ double red[2][kConvMaxThreads / 64];
    const int tid = threadIdx.x, nthr = blockDim.x, lane = tid & 63, wave = tid >> 6;
    const int64_t bi = blockIdx.x;
    const int L = (int)(n + m - 1);
    const T* xb = x + bi * n;
    const T* yb = y + bi * m;
    T* zb = z + bi * (int64_t)L;
    uint8_t* pb = pstar ? pstar + bi * (int64_t)L : nullptr;

    // scales: max x, max y
    double mx = 0.0, my = 0.0;
    for (int i = tid; i < n; i += nthr) mx = fmax(mx, (double)xb[i]);
    for (int i = tid; i < m; i += nthr) my = fmax(my, (double)yb[i]);
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    if (lane == 0) {
        red[0][wave] = mx;
        red[1][wave] = my;
    }
    for (int k = tid; k < N / 2; k += nthr) {
        double sn, cs;
        sincospi(-2.0 * (double)k / (double)N, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
    __syncthreads();
    double rx = 0.0, ry = 0.0;
    for (int w = 0; w < nthr / 64; ++w) {
        rx = fmax(rx, red[0][w]);
        ry = fmax(ry, red[1][w]);
    }
    const double inv_n = 1.0 / (double)N;
    const double rxy = rx * ry;
    // output index tid + j * nthr is decided once bit j is set
    uint32_t decided = 0u;

    for (int q = spec.n - 1; q >= 0; --q) {
        const int p = spec.p[q];
        for (int t = tid; t < N; t += nthr) {
            const double a = (t < n && rx > 0.0) ? ipow_d((double)xb[t] / rx, p) : 0.0;
            const double b = (t < m && ry > 0.0) ? ipow_d((double)yb[t] / ry, p) : 0.0;
            buf[brev_n(t, logN)] = make_double2(a, b);
        }
        __syncthreads();
        fft_radix2(buf, tw, logN);
        // W_k = X_k Y_k; W_{N-k} = conj W_k.  Stored conjugated (the inverse
        // transform is the forward transform of the conjugate), then put in
        // bit-reversed order for the second pass.
        for (int k = tid; k <= N / 2; k += nthr) {
            const int kn = (N - k) & (N - 1);
            const double2 Zk = buf[k], Zn = buf[kn];
            const double2 Xk = make_double2(0.5 * (Zk.x + Zn.x), 0.5 * (Zk.y - Zn.y));
            const double2 Yk = make_double2(0.5 * (Zk.y + Zn.y), -0.5 * (Zk.x - Zn.x));
            const double2 Wk = cmul(Xk, Yk);
            buf[k] = make_double2(Wk.x, -Wk.y);
            buf[kn] = Wk;
        }
        __syncthreads();
        for (int t = tid; t < N; t += nthr) {
            const int r = brev_n(t, logN);
            if (t < r) {
                const double2 a = buf[t];
                buf[t] = buf[r];
                buf[r] = a;
            }
        }
        __syncthreads();
        fft_radix2(buf, tw, logN);
        // S_p[t] = Re(FFT(conj W))[t] / N
        int open = 0;
        for (int j = 0, t = tid; t < L; ++j, t += nthr) {
            if (decided & (1u << j)) continue;
            const double S = buf[t].x * inv_n;
            const bool stable = S >= spec.tau;
            if (!stable && q > 0) {
                open = 1;
                continue;
            }
            // stable, or the smallest p with none stable (its root of max(S, 0))
            decided |= 1u << j;
            double root = 0.0;
            if (S > 0.0) root = p == 1 ? S : exp(log(S) / (double)p);
            zb[t] = (T)(rxy * root);
            if (pb) pb[t] = stable ? (uint8_t)q : (uint8_t)MT_PSTAR_NONE;
        }
        if (!__syncthreads_or(open)) break;
    }
}

template <typename T>
__global__ __launch_bounds__(256) void mt_maxconv_exact_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                              int64_t b, int64_t n, int64_t m,
                                                              T* __restrict__ z) {
    const int64_t L = n + m - 1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b * L) return;
    const int64_t bi = g / L, t = g - bi * L;
    const T* xb = x + bi * n;
    const T* yb = y + bi * m;
    const int64_t lo = t - (m - 1) > 0 ? t - (m - 1) : 0;
    const int64_t hi = t < n - 1 ? t : n - 1;
    T best = 0;
    for (int64_t i = lo; i <= hi; ++i) {
        const T v = xb[i] * yb[t - i];
        best = v > best ? v : best;
    }
    z[g] = best;
}

}  // namespace

int maxconv_log_size(int64_t n, int64_t m) {
    const int64_t L = n + m - 1;
    int logN = 1;
    while ((int64_t(1) << logN) < L) ++logN;
    return logN;
}

hipError_t launch_maxconv(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                          const MaxconvSpec& spec, void* z, uint8_t* pstar, hipStream_t st) {
    if (b <= 0 || n <= 0 || m <= 0) return hipSuccess;
    const int logN = maxconv_log_size(n, m);
    if (logN > kMaxConvLog) return hipErrorInvalidValue;
    const int N = 1 << logN;
    int threads = N / 2 < 64 ? 64 : N / 2;
    if (threads > kConvMaxThreads) threads = kConvMaxThreads;
    const size_t lds = (size_t)N * sizeof(double2) + (size_t)(N / 2) * sizeof(double2);
    // the dynamic-LDS limit is a per-device attribute of each kernel
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_set.load() & bit)) {
        const int max_lds = kMaxConvN * (int)sizeof(double2) * 3 / 2;
        e = hipFuncSetAttribute((const void*)mt_maxconv_kernel<double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e == hipSuccess)
            e = hipFuncSetAttribute((const void*)mt_maxconv_kernel<float>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, max_lds);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    timing_before("mt_maxconv", st);
    if (f64)
        hipLaunchKernelGGL(mt_maxconv_kernel<double>, dim3((unsigned)b), dim3(threads), lds, st,
                           (const double*)x, (const double*)y, n, m, logN, spec, (double*)z, pstar);
    else
        hipLaunchKernelGGL(mt_maxconv_kernel<float>, dim3((unsigned)b), dim3(threads), lds, st,
                           (const float*)x, (const float*)y, n, m, logN, spec, (float*)z, pstar);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_maxconv_exact(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                                void* z, hipStream_t st) {
    const int64_t total = b * (n + m - 1);
    if (b <= 0 || n <= 0 || m <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    timing_before("mt_maxconv_exact", st);
    if (f64)
        hipLaunchKernelGGL(mt_maxconv_exact_kernel<double>, dim3(blocks), dim3(256), 0, st, (const double*)x,
                           (const double*)y, b, n, m, (double*)z);
    else
        hipLaunchKernelGGL(mt_maxconv_exact_kernel<float>, dim3(blocks), dim3(256), 0, st, (const float*)x,
                           (const float*)y, b, n, m, (float*)z);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
