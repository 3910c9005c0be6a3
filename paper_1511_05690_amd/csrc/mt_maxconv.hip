// Max-convolution (Sec. 1) and the top k of x + y (Sec. 2.3) on FFT ring
// results.
//
// Estimate: z[t] = max_i x[i] y[t - i] from the norm sequence
// S_p[t] = (x'^p * y'^p)[t] with x' = x / max x, y' = y / max y (terms in
// [0, 1], the scaling of Sec. 2.1), computed by FFT convolution in FP64 (the
// fast ring kernel H, Sec. 2.1, whose threshold there is tau = 1e-12); per
// index the largest p of the family with S_p >= tau, and
// z = max x max y S_{p*}^(1/p*).
//
// LDS path (n + m - 1 <= 4096): a transform of N = max(16, 2^ceil(log2(n + m
// - 1))) points is done by N / 16 threads that hold 16 complex values each in
// registers (N = 4096: 256 threads, one pair per workgroup; smaller N packs
// 4096 / N pairs into a workgroup).  Passes are Stockham radix-16 (the last
// one radix 2, 4 or 8 when log2 N is not a multiple of 4), natural order in
// and out, through one LDS buffer per pair padded by one element every 16
// (the stride-16 writes of the first pass then hit distinct banks).
// Twiddles exp(-2 pi i m / N) come from one LDS table of cos and sin of
// 2 pi k / N for k <= N / 8 (the other octants by symmetry); a thread looks up
// w and w^4 of its butterflies once and forms the other powers by products.
// Per p, largest first:
//   forward: x'^p + i y'^p (x, y re-read per p, times 1 / max), so both real
//            transforms come out of one complex FFT;
//   product: thread t reads Z_t and Z_{N-t} and forms conj(W_t),
//            W = X Y with X_t = (Z_t + conj Z_{N-t}) / 2, Y_t = (Z_t - conj
//            Z_{N-t}) / 2i (the first pass of the inverse reads these pairs);
//   inverse: the forward FFT of conj(W), whose real part / N is S_p; the
//            last pass leaves S in registers at the positions the thread
//            owns, where the p* test runs.
// Indices decided at a larger p keep their S; a workgroup stops once every
// index of its pairs is decided, and the roots are taken once per index.
// When every index still open has at most kDirectTerms terms (they sit at
// the ends of the output, where few products meet), the workgroup finishes
// them by direct sums of x'^p y'^p for the remaining p instead of further
// transforms.
//
// Global path (n + m - 1 <= 16384): the same passes through two buffers in
// the workspace, one thread per butterfly, kernel boundaries between passes,
// the whole batch one p at a time.
//
// Top k of x + y: the ring results of both runs (y and y reversed) for every
// p by either path, the initial estimates, a one-wave NormQueue per run and
// the index pairing.
//
// Exact: z[t] = max_i x[i] y[t - i] by the definition, one thread per output
// index, products in the input precision.

#include <atomic>
#include <climits>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kConvThreads = 256;  // kMaxConvN / 16
static_assert(kConvThreads * 16 == kMaxConvN, "16 values per thread at the largest N");
constexpr int kConvMinLog = 4;
// padded LDS elements per workgroup: one buffer of N + N / 16 per pair, 4096 / N pairs
constexpr int kConvLdsElems = kMaxConvN + kMaxConvN / 16;
// twiddle octant: cos and sin of 2 pi k / N, k = 0 .. N / 8
constexpr int kConvTwElems = kMaxConvN / 8 + 1;

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
// -i a
__device__ __forceinline__ double2 cmul_mi(double2 a) { return make_double2(a.y, -a.x); }

__device__ __forceinline__ double ipow_d(double v, int p) {
    double r = 1.0;
    while (p) {
        if (p & 1) r *= v;
        v *= v;
        p >>= 1;
    }
    return r;
}

// v[i] <- v[i]^p componentwise for the 16 values of a thread.  A power of two
// is one loop of squarings over all values (uniform, in place); other p go
// value by value (a second array of 16 would not fit beside the rest).  The
// same products in the same order as ipow_d either way.
__device__ __forceinline__ void pow_all(double2 (&v)[16], int p) {
    if ((p & (p - 1)) == 0) {
        for (int e = p; e > 1; e >>= 1) {
#pragma unroll
            for (int i = 0; i < 16; ++i) v[i] = make_double2(v[i].x * v[i].x, v[i].y * v[i].y);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = make_double2(ipow_d(v[i].x, p), ipow_d(v[i].y, p));
}

__device__ __forceinline__ int padi(int i) { return i + (i >> 4); }

// An empty asm that claims to change v: values derived from it are then
// recomputed where they are used instead of being hoisted out of the p loop
// and held in registers for all of it.
__device__ __forceinline__ void opaque(double2& v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

// cos(pi / 8), sin(pi / 8), sqrt(2) / 2
constexpr double kC8 = 0.92387953251128674;
constexpr double kS8 = 0.38268343236508978;
constexpr double kH = 0.70710678118654752;

__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
    const double2 t0 = cadd(a0, a2), t1 = csub(a0, a2), t2 = cadd(a1, a3), t3 = cmul_mi(csub(a1, a3));
    a0 = cadd(t0, t2);
    a1 = cadd(t1, t3);
    a2 = csub(t0, t2);
    a3 = csub(t1, t3);
}

// Forward DFT of the R values v[o + s * e], e = 0 .. R - 1, in place.  Output
// k ends in register o + s * oreg<R>(k).
template <int R>
__device__ __forceinline__ constexpr int oreg(int k) {
    if constexpr (R == 16) return (k >> 2) + 4 * (k & 3);
    if constexpr (R == 8) return 2 * (k & 3) + (k >> 2);
    return k;
}

template <int R>
__device__ __forceinline__ void dft(double2 (&v)[16], int o, int s) {
    if constexpr (R == 2) {
        const double2 a = v[o], b = v[o + s];
        v[o] = cadd(a, b);
        v[o + s] = csub(a, b);
    } else if constexpr (R == 4) {
        dft4(v[o], v[o + s], v[o + 2 * s], v[o + 3 * s]);
    } else if constexpr (R == 8) {
        // e = c + 2 n2, k = k1 + 4 k2: two DFT4 over n2, twiddle W8^(c k1), DFT2 over c
#pragma unroll
        for (int c = 0; c < 2; ++c) dft4(v[o + s * c], v[o + s * (c + 2)], v[o + s * (c + 4)], v[o + s * (c + 6)]);
        // u[c][k1] sits at c + 2 k1
        v[o + s * 3] = make_double2(kH * (v[o + s * 3].x + v[o + s * 3].y), kH * (v[o + s * 3].y - v[o + s * 3].x));
        v[o + s * 5] = cmul_mi(v[o + s * 5]);
        v[o + s * 7] = make_double2(kH * (v[o + s * 7].y - v[o + s * 7].x), -kH * (v[o + s * 7].x + v[o + s * 7].y));
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            const double2 a = v[o + s * (2 * k1)], b = v[o + s * (2 * k1 + 1)];
            v[o + s * (2 * k1)] = cadd(a, b);
            v[o + s * (2 * k1 + 1)] = csub(a, b);
        }
    } else {
        static_assert(R == 16, "radix 2, 4, 8 or 16");
        // e = c + 4 n2, k = k1 + 4 k2: four DFT4 over n2, twiddle W16^(c k1), four DFT4 over c
#pragma unroll
        for (int c = 0; c < 4; ++c) dft4(v[o + s * c], v[o + s * (c + 4)], v[o + s * (c + 8)], v[o + s * (c + 12)]);
        // u[c][k1] sits at c + 4 k1; W16^1 = (C, -S), ^2 = (H, -H), ^3 = (S, -C), ^4 = -i,
        // ^6 = (-H, -H), ^9 = (-C, S)
        const double2 w1 = make_double2(kC8, -kS8), w3 = make_double2(kS8, -kC8), w9 = make_double2(-kC8, kS8);
        v[o + s * 5] = cmul(v[o + s * 5], w1);                                                         // c1 k1 1
        v[o + s * 9] = make_double2(kH * (v[o + s * 9].x + v[o + s * 9].y), kH * (v[o + s * 9].y - v[o + s * 9].x));  // c1 k2
        v[o + s * 13] = cmul(v[o + s * 13], w3);                                                       // c1 k3
        v[o + s * 6] = make_double2(kH * (v[o + s * 6].x + v[o + s * 6].y), kH * (v[o + s * 6].y - v[o + s * 6].x));  // c2 k1
        v[o + s * 10] = cmul_mi(v[o + s * 10]);                                                        // c2 k2
        v[o + s * 14] = make_double2(kH * (v[o + s * 14].y - v[o + s * 14].x), -kH * (v[o + s * 14].x + v[o + s * 14].y));  // c2 k3
        v[o + s * 7] = cmul(v[o + s * 7], w3);                                                         // c3 k1
        v[o + s * 11] = make_double2(kH * (v[o + s * 11].y - v[o + s * 11].x), -kH * (v[o + s * 11].x + v[o + s * 11].y));  // c3 k2
        v[o + s * 15] = cmul(v[o + s * 15], w9);                                                       // c3 k3
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1)
            dft4(v[o + s * (4 * k1)], v[o + s * (4 * k1 + 1)], v[o + s * (4 * k1 + 2)], v[o + s * (4 * k1 + 3)]);
    }
}

template <int LOGN>
struct Fft {
    static constexpr int N = 1 << LOGN;
    static constexpr int T = N / 16;               // threads per pair
    static constexpr int G = kConvThreads / T;     // pairs per workgroup
    static constexpr int NP = N + N / 16;          // padded buffer
    static constexpr int NPASS = (LOGN + 3) / 4;
    static constexpr int radix(int pass) { return pass < LOGN / 4 ? 16 : (1 << (LOGN % 4)); }
    static constexpr int span(int pass) {
        int s = 1;
        for (int i = 0; i < pass; ++i) s *= radix(i);
        return s;
    }
};

// One Stockham pass on the thread's registers: butterfly g (j = tl + g T) takes
// the values at j + e N / R (registers g + e B), twiddles them by
// exp(-2 pi i k e / (Ns R)), k = j mod Ns, and transforms.
// exp(-2 pi i mm / N), 0 <= mm < N, from the octant table tw[k] = (cos, sin)(2 pi k / N):
// mm = q N / 4 + r gives (-i)^q w^r, and w^r = (-i) conj(w^(N/4 - r)) above N / 8.
template <int LOGN>
__device__ __forceinline__ double2 twiddle(const double2* tw, int mm) {
    constexpr int N4 = (1 << LOGN) / 4;
    const int q = mm / N4, r = mm & (N4 - 1);
    const bool refl = r > N4 / 2;
    const double2 t = tw[refl ? N4 - r : r];
    double a = refl ? t.y : t.x, b = refl ? -t.x : -t.y;
    if (q & 1) {
        const double c = a;
        a = b;
        b = -c;
    }
    if (q & 2) {
        a = -a;
        b = -b;
    }
    return make_double2(a, b);
}

// The thread's base twiddles, the same for every p and both directions:
// w1[PASS][g] = exp(-2 pi i k / (Ns R)) for butterfly g (k = j mod Ns) and
// w4[PASS][g] = its fourth power, looked up once (unused entries vanish).
template <int LOGN>
struct PassTwiddles {
    double2 w1[Fft<LOGN>::NPASS][16];
    double2 w4[Fft<LOGN>::NPASS][16];
};

template <int LOGN, int PASS>
__device__ __forceinline__ void load_twiddles(PassTwiddles<LOGN>& pt, int tl, const double2* tw) {
    using F = Fft<LOGN>;
    if constexpr (PASS < F::NPASS) {
        constexpr int R = F::radix(PASS), Ns = F::span(PASS), B = 16 / R;
#pragma unroll
        for (int g = 0; g < B; ++g) {
            const int j = tl + g * F::T;
            const int step = (j & (Ns - 1)) * (F::N / (Ns * R));
            pt.w1[PASS][g] = twiddle<LOGN>(tw, step);
            if constexpr (R >= 8) pt.w4[PASS][g] = twiddle<LOGN>(tw, 4 * step);
        }
        load_twiddles<LOGN, PASS + 1>(pt, tl, tw);
    }
}

// One Stockham pass on the thread's registers: butterfly g (j = tl + g T) takes
// the values at j + e N / R (registers g + e B), twiddles them by w^e,
// w = exp(-2 pi i k / (Ns R)), k = j mod Ns, and transforms.
template <int LOGN, int PASS>
__device__ __forceinline__ void pass_compute(double2 (&v)[16], const PassTwiddles<LOGN>& pt) {
    using F = Fft<LOGN>;
    constexpr int R = F::radix(PASS), Ns = F::span(PASS), B = 16 / R;
    if constexpr (Ns > 1) {
        // w^e from w and w^4 by at most three products each (about 10 ulp)
#pragma unroll
        for (int g = 0; g < B; ++g) {
            double2 w1 = pt.w1[PASS][g];
            opaque(w1);
            v[g + B] = cmul(v[g + B], w1);
            if constexpr (R >= 4) {
                const double2 w2 = cmul(w1, w1), w3 = cmul(w2, w1);
                v[g + 2 * B] = cmul(v[g + 2 * B], w2);
                v[g + 3 * B] = cmul(v[g + 3 * B], w3);
                if constexpr (R >= 8) {
                    double2 w4 = pt.w4[PASS][g];
                    opaque(w4);
                    const double2 w5 = cmul(w4, w1), w6 = cmul(w4, w2), w7 = cmul(w4, w3);
                    v[g + 4 * B] = cmul(v[g + 4 * B], w4);
                    v[g + 5 * B] = cmul(v[g + 5 * B], w5);
                    v[g + 6 * B] = cmul(v[g + 6 * B], w6);
                    v[g + 7 * B] = cmul(v[g + 7 * B], w7);
                    if constexpr (R == 16) {
                        const double2 w8 = cmul(w4, w4);
                        v[g + 8 * B] = cmul(v[g + 8 * B], w8);
                        v[g + 9 * B] = cmul(v[g + 9 * B], cmul(w8, w1));
                        v[g + 10 * B] = cmul(v[g + 10 * B], cmul(w8, w2));
                        v[g + 11 * B] = cmul(v[g + 11 * B], cmul(w8, w3));
                        v[g + 12 * B] = cmul(v[g + 12 * B], cmul(w8, w4));
                        v[g + 13 * B] = cmul(v[g + 13 * B], cmul(w8, w5));
                        v[g + 14 * B] = cmul(v[g + 14 * B], cmul(w8, w6));
                        v[g + 15 * B] = cmul(v[g + 15 * B], cmul(w8, w7));
                    }
                }
            }
        }
    }
#pragma unroll
    for (int g = 0; g < B; ++g) dft<R>(v, g, B);
}

// Output k of butterfly g goes to (j - k0) R + k0 + k Ns, k0 = j mod Ns.
// The padded index of base + k * stride for k = 0 .. 15, as padi(base) plus a
// constant where the stride is a multiple of 16 (or 1 with base a multiple of 16).
template <int STRIDE>
__device__ __forceinline__ int pad_step(int base_padded, int base, int k) {
    if constexpr (STRIDE % 16 == 0)
        return base_padded + k * (STRIDE / 16 * 17);
    else
        return padi(base + k * STRIDE);
}

template <int LOGN, int PASS>
__device__ __forceinline__ void pass_store(const double2 (&v)[16], int tl, double2* buf) {
    using F = Fft<LOGN>;
    constexpr int R = F::radix(PASS), Ns = F::span(PASS), B = 16 / R;
#pragma unroll
    for (int g = 0; g < B; ++g) {
        const int j = tl + g * F::T;
        const int k0 = j & (Ns - 1);
        const int base = (j - k0) * R + k0;
        const int bp = padi(base);
        if constexpr (Ns == 1 && R == 16) {
            // base = 16 j: the 16 outputs are contiguous after padding
#pragma unroll
            for (int k = 0; k < R; ++k) buf[bp + k] = v[g + B * oreg<R>(k)];
        } else {
#pragma unroll
            for (int k = 0; k < R; ++k) buf[pad_step<Ns>(bp, base, k)] = v[g + B * oreg<R>(k)];
        }
    }
}

// Every pass reads the thread's positions tl + i T into register i.
template <int LOGN>
__device__ __forceinline__ void pass_load(double2 (&v)[16], int tl, const double2* buf) {
    constexpr int TP = Fft<LOGN>::T;
    const int bp = padi(tl);
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = buf[pad_step<TP>(bp, tl, i)];
}

// Passes 1 .. NPASS - 2 (or - 1): load, compute, barrier, store, barrier.
template <int LOGN, int PASS, int END>
__device__ __forceinline__ void middle_passes(double2 (&v)[16], int tl, double2* buf,
                                              const PassTwiddles<LOGN>& pt) {
    if constexpr (PASS < END) {
        pass_load<LOGN>(v, tl, buf);
        pass_compute<LOGN, PASS>(v, pt);
        __syncthreads();
        pass_store<LOGN, PASS>(v, tl, buf);
        __syncthreads();
        middle_passes<LOGN, PASS + 1, END>(v, tl, buf, pt);
    }
}

// Register holding position tl + i T after the last pass.
template <int LOGN>
__device__ __forceinline__ constexpr int last_reg(int i) {
    using F = Fft<LOGN>;
    constexpr int R = F::radix(F::NPASS - 1), B = 16 / R;
    return (i % B) + B * oreg<R>(i / B);
}

// Maxima of mx and my over the threads of one slot (contiguous lanes; several
// waves when TP > 64); red holds one pair per wave.
template <int TP>
__device__ __forceinline__ void slot_max(double& mx, double& my, double (*red)[kConvThreads / 64]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int d = (TP < 64 ? TP : 64) / 2; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    if constexpr (TP > 64) {
        if (lane == 0) {
            red[0][wave] = mx;
            red[1][wave] = my;
        }
        __syncthreads();
        constexpr int WPI = TP / 64;
        const int w0 = (wave / WPI) * WPI;
#pragma unroll
        for (int w = 0; w < WPI; ++w) {
            mx = fmax(mx, red[0][w0 + w]);
            my = fmax(my, red[1][w0 + w]);
        }
    }
}

// The octant table cos / sin (2 pi k / N), k = 0 .. N / 8.
template <int LOGN>
__device__ __forceinline__ void build_twiddle_table(double2* tw) {
    constexpr int N = 1 << LOGN;
    for (int k = threadIdx.x; k <= N / 8; k += kConvThreads) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)N, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
}

// One pair's convolution of the two real sequences held as v[i] = (a, b) at
// the thread's positions tl + i T (a = x'^p, b = y'^p, zero beyond the
// lists): the forward transform of a + i b, the product W = X Y formed from
// Z_t and Z_(N-t), and the inverse as the forward transform of conj(W).  On
// return v[last_reg(i)].x * 0.25 / N is (a * b)[tl + i T].  Every thread of
// the workgroup calls it (it holds barriers).
template <int LOGN>
__device__ __forceinline__ void convolve_pair(double2 (&v)[16], int tl, double2* buf,
                                              const PassTwiddles<LOGN>& pt) {
    using F = Fft<LOGN>;
    constexpr int N = F::N, TP = F::T;
    pass_compute<LOGN, 0>(v, pt);
    pass_store<LOGN, 0>(v, tl, buf);
    __syncthreads();
    middle_passes<LOGN, 1, F::NPASS>(v, tl, buf, pt);
    // conj(4 W_t), 4 W_t = (Z_t + conj Z_-t)(Z_t - conj Z_-t) / i
    const int bp = padi(tl), bn = padi(N - tl);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        int ik, in;
        if constexpr (TP % 16 == 0) {
            // t = tl + i TP > 0 for i > 0
            ik = bp + i * (TP / 16 * 17);
            in = i == 0 ? padi((N - tl) & (N - 1)) : bn - i * (TP / 16 * 17);
        } else {
            const int t = tl + i * TP;
            ik = padi(t);
            in = padi((N - t) & (N - 1));
        }
        const double2 zk = buf[ik], zn = buf[in];
        const double2 a = make_double2(zk.x + zn.x, zk.y - zn.y);
        const double2 c = make_double2(zk.y + zn.y, zn.x - zk.x);
        const double2 w = cmul(a, c);
        v[i] = make_double2(w.x, -w.y);
    }
    // the last pass leaves position tl + i TP in register last_reg(i)
    pass_compute<LOGN, 0>(v, pt);
    if constexpr (F::NPASS > 1) {
        __syncthreads();
        pass_store<LOGN, 0>(v, tl, buf);
        __syncthreads();
        middle_passes<LOGN, 1, F::NPASS - 1>(v, tl, buf, pt);
        pass_load<LOGN>(v, tl, buf);
        pass_compute<LOGN, F::NPASS - 1>(v, pt);
    }
}

// An open index with at most this many terms is finished by direct sums.
constexpr int kDirectTerms = 64;

// x^p for p >= 1 by binary powering (p uniform)
__device__ __forceinline__ double pow_int(double x, int p) {
    double r = 1.0;
    for (; p; p >>= 1) {
        if (p & 1) r *= x;
        x *= x;
    }
    return r;
}

template <typename T, int LOGN>
__global__ __launch_bounds__(kConvThreads, 2) void mt_maxconv_kernel(const T* __restrict__ x,
                                                                  const T* __restrict__ y, int64_t b, int64_t n,
                                                                  int64_t m, MaxconvSpec spec,
                                                                  T* __restrict__ z,
                                                                  uint8_t* __restrict__ pstar,
                                                                  unsigned long long* work) {
    using F = Fft<LOGN>;
    constexpr int N = F::N, TP = F::T;
    extern __shared__ double2 lds[];
    __shared__ double red[2][kConvThreads / 64];
    double2* tw = lds;  // kConvTwElems
    const int tid = threadIdx.x;
    if (work && tid == 0) timing_span_begin(work);
    const int slot = tid / TP, tl0 = tid % TP;
    const int64_t item = (int64_t)blockIdx.x * F::G + slot;
    const bool active = item < b;
    const int L = (int)(n + m - 1);
    double2* buf = lds + kConvTwElems + slot * F::NP;
    const T* xi = x + item * n;
    const T* yi = y + item * m;

    // the thread owns positions tl + i TP, i = 0 .. 15
    double mx = 0.0, my = 0.0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int t = tl0 + i * TP;
        if (active && t < n) mx = fmax(mx, (double)xi[t]);
        if (active && t < m) my = fmax(my, (double)yi[t]);
    }
    build_twiddle_table<LOGN>(tw);
    slot_max<TP>(mx, my, red);
    __syncthreads();
    PassTwiddles<LOGN> pt;
    load_twiddles<LOGN, 1>(pt, tl0, tw);
    const double rxy = mx * my;
    const double ix = mx > 0.0 ? 1.0 / mx : 0.0, iy = my > 0.0 ? 1.0 / my : 0.0;
    // 1 / N and the 1 / 4 of X Y (both halves carry 1 / 2)
    const double scale = 0.25 / (double)N;
    uint32_t decided = 0u;  // bit i: position tl + i TP
    double s_sel[16];       // S at the selected p
    uint32_t q_sel[4];      // its family index (byte i % 4 of word i / 4; MT_PSTAR_NONE if none stable)
#pragma unroll
    for (int i = 0; i < 16; ++i) s_sel[i] = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) q_sel[i] = 0u;
    int iters = 0;

    for (int q = spec.n - 1; q >= 0; --q) {
        ++iters;
        const int p = spec.p[q];
        // re-derive the addresses per p instead of holding them across the loop
        int tl = tl0;
        asm volatile("" : "+v"(tl));
        double2 v[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int t = tl + i * TP;
            const double a = (active && t < n) ? (double)xi[t] * ix : 0.0;
            const double c = (active && t < m) ? (double)yi[t] * iy : 0.0;
            v[i] = make_double2(a, c);
        }
        pow_all(v, p);
        convolve_pair<LOGN>(v, tl, buf, pt);
        // p* test: the first stable p from the top decides an index; the
        // smallest p decides what is left (its S, no p stable)
        int open = 0, open_far = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int t = tl + i * TP;
            const double S = v[last_reg<LOGN>(i)].x * scale;
            const bool live = active && t < L && !(decided & (1u << i));
            const bool stable = S >= spec.tau;
            const bool dec = live && (stable || q == 0);
            open |= live && !dec;
            // terms of index t: x[j] y[t - j] for max(0, t - m + 1) <= j <= min(t, n - 1)
            const int nterms = min(t, (int)n - 1) - max(0, t - (int)m + 1) + 1;
            open_far |= live && !dec && nterms > kDirectTerms;
            s_sel[i] = dec ? S : s_sel[i];
            const uint32_t code = stable ? (uint32_t)q : (uint32_t)MT_PSTAR_NONE;
            q_sel[i / 4] = dec ? (q_sel[i / 4] & ~(0xffu << (8 * (i % 4)))) | (code << (8 * (i % 4))) : q_sel[i / 4];
            decided |= dec ? 1u << i : 0u;
        }
        if (!__syncthreads_or(open)) break;
        if (!__syncthreads_or(open_far)) {
            // every open index has few terms: its S for the remaining p as a
            // direct sum (the exact S the transforms approximate), the same
            // selection.  x' and y' go to the pair's LDS buffer first (free
            // after the barrier above; n + m - 1 <= N doubles fit in it).
            double* sx = (double*)buf;
            double* sy = sx + n;
            for (int j = tl; j < (int)n; j += TP) sx[j] = active ? (double)xi[j] * ix : 0.0;
            for (int j = tl; j < (int)m; j += TP) sy[j] = active ? (double)yi[j] * iy : 0.0;
            __syncthreads();
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int t = tl + i * TP;
                if (!(active && t < L && !(decided & (1u << i)))) continue;
                const int j0 = max(0, t - (int)m + 1), j1 = min(t, (int)n - 1);
                for (int qq = q - 1; qq >= 0; --qq) {
                    const int pp = spec.p[qq];
                    double S = 0.0;
                    for (int j = j0; j <= j1; ++j) S = fma(pow_int(sx[j], pp), pow_int(sy[t - j], pp), S);
                    const bool stable = S >= spec.tau;
                    if (!(stable || qq == 0)) continue;
                    s_sel[i] = S;
                    const uint32_t code = stable ? (uint32_t)qq : (uint32_t)MT_PSTAR_NONE;
                    q_sel[i / 4] = (q_sel[i / 4] & ~(0xffu << (8 * (i % 4)))) | (code << (8 * (i % 4)));
                    decided |= 1u << i;
                    break;
                }
            }
            // the roots below reuse the buffer
            __syncthreads();
            break;
        }
    }
    // roots, once per index: the selected S goes to the thread's own LDS
    // positions, then one index at a time (the buffer is free after the loop's
    // last barrier)
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[padi(tl0 + i * TP)].x = s_sel[i];
    if (active) {
#pragma unroll 1
        for (int i = 0; i < 16; ++i) {
            const int t = tl0 + i * TP;
            if (t >= L) break;
            const double S = buf[padi(t)].x;
            const uint32_t code = (q_sel[i / 4] >> (8 * (i % 4))) & 0xffu;
            const int p = spec.p[code == MT_PSTAR_NONE ? 0 : code];
            double root = 0.0;
            if (S > 0.0) {
                if ((p & (p - 1)) == 0) {
                    root = S;
                    for (int e = p; e > 1; e >>= 1) root = sqrt(root);
                } else {
                    root = exp(log(S) / (double)p);
                }
            }
            z[item * L + t] = (T)(rxy * root);
            if (pstar) pstar[item * L + t] = (uint8_t)code;
        }
    }
    if (work) {
        // timed launch: two complex transforms per p, 5 N log2 N flops each
        // (the usual FFT count), and the end once every wave is done
        __syncthreads();
        if (tid == 0) {
            const int64_t pairs = b - (int64_t)blockIdx.x * F::G < F::G ? b - (int64_t)blockIdx.x * F::G : F::G;
            atomicAdd(work, (unsigned long long)iters * (unsigned long long)pairs * (10ull * N * LOGN));
            timing_span_end(work);
        }
    }
}

// Top k of x + y (Sec. 2.3).  The ring results sigma^(p) = x'^p * y'^p with
// x' = e^(x - max x), y' = e^(y - max y) (terms in (0, 1]), for every p of the
// family and both runs (run 0 with y, run 1 with y reversed): one convolution
// per slot, slot = run |P| + q.  sigma is (2, |P|, 2n - 1), FP64.
template <typename T, int LOGN>
__global__ __launch_bounds__(kConvThreads, 2) void mt_xy_sigma_kernel(const T* __restrict__ x,
                                                                   const T* __restrict__ y, int64_t n,
                                                                   MaxconvSpec spec, double* __restrict__ sigma) {
    using F = Fft<LOGN>;
    constexpr int N = F::N, TP = F::T;
    extern __shared__ double2 lds[];
    __shared__ double red[2][kConvThreads / 64];
    double2* tw = lds;  // kConvTwElems
    const int tid = threadIdx.x;
    const int slot = tid / TP, tl = tid % TP;
    const int item = (int)blockIdx.x * F::G + slot;
    const bool active = item < 2 * spec.n;
    const int run = active ? item / spec.n : 0, q = active ? item % spec.n : 0;
    const int L = (int)(2 * n - 1);
    double2* buf = lds + kConvTwElems + slot * F::NP;

    double mx = -INFINITY, my = -INFINITY;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int t = tl + i * TP;
        if (active && t < n) {
            mx = fmax(mx, (double)x[t]);
            my = fmax(my, (double)y[t]);
        }
    }
    build_twiddle_table<LOGN>(tw);
    slot_max<TP>(mx, my, red);
    __syncthreads();
    PassTwiddles<LOGN> pt;
    load_twiddles<LOGN, 1>(pt, tl, tw);
    const int p = spec.p[q];
    double2 v[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const int t = tl + i * TP;
        double a = 0.0, c = 0.0;
        if (active && t < n) {
            a = exp((double)x[t] - mx);
            c = exp((double)y[run ? n - 1 - t : t] - my);
        }
        v[i] = make_double2(a, c);
    }
    pow_all(v, p);
    convolve_pair<LOGN>(v, tl, buf, pt);
    if (active) {
        double* out = sigma + ((int64_t)run * spec.n + q) * L;
        const double scale = 0.25 / (double)N;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int t = tl + i * TP;
            if (t < L) out[t] = v[last_reg<LOGN>(i)].x * scale;
        }
    }
}

// psi for every diagonal of both runs before any pop: the root at the largest
// p with sigma^(p)[m] >= tau, 0 if none.  One thread per (run, m).
__global__ __launch_bounds__(256) void mt_xy_psi_kernel(const double* __restrict__ sigma, int64_t L,
                                                       MaxconvSpec spec, double* __restrict__ psi) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= 2 * L) return;
    const int64_t run = g / L, m = g - run * L;
    const double* col = sigma + run * spec.n * L + m;
    double s[MT_MAX_P];
#pragma unroll
    for (int q = 0; q < MT_MAX_P; ++q) s[q] = q < spec.n ? col[q * L] : 0.0;
    int qh = -1;
#pragma unroll
    for (int q = 0; q < MT_MAX_P; ++q) qh = (q < spec.n && s[q] >= spec.tau) ? q : qh;
    double sh = 0.0;
#pragma unroll
    for (int q = 0; q < MT_MAX_P; ++q) sh = q == qh ? s[q] : sh;
    psi[g] = qh >= 0 ? pow(sh, 1.0 / (double)spec.p[qh]) : 0.0;
}

// ---- wave-wide argmax for the queues ----------------------------------
//
// DPP row shifts and row broadcasts (register moves between lanes, no LDS
// round trip) carry the maximum to lane 63 in six steps; lanes a move has no
// source for keep their own value, the identity of max.

template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_i32(int x) {
    return __builtin_amdgcn_update_dpp(x, x, kCtrl, kRowMask, 0xf, false);
}

template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_i32<kCtrl, kRowMask>((int)b);
    const int hi = dpp_i32<kCtrl, kRowMask>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double x, int l) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// row_shr:1, 2, 4, 8 leave each row's maximum in its lane 15; row_bcast:15
// into rows 1 and 3 and row_bcast:31 into rows 2 and 3 bring all four to
// lane 63.
__device__ __forceinline__ double wave_max_f64(double m) {
    m = fmax(m, dpp_f64<0x111, 0xf>(m));
    m = fmax(m, dpp_f64<0x112, 0xf>(m));
    m = fmax(m, dpp_f64<0x114, 0xf>(m));
    m = fmax(m, dpp_f64<0x118, 0xf>(m));
    m = fmax(m, dpp_f64<0x142, 0xa>(m));
    m = fmax(m, dpp_f64<0x143, 0xc>(m));
    return readlane_f64(m, 63);
}

__device__ __forceinline__ int wave_min_i32(int m) {
    m = min(m, dpp_i32<0x111, 0xf>(m));
    m = min(m, dpp_i32<0x112, 0xf>(m));
    m = min(m, dpp_i32<0x114, 0xf>(m));
    m = min(m, dpp_i32<0x118, 0xf>(m));
    m = min(m, dpp_i32<0x142, 0xa>(m));
    m = min(m, dpp_i32<0x143, 0xc>(m));
    return __builtin_amdgcn_readlane(m, 63);
}

// The largest v over the wave and, among the lanes holding it, the smallest
// s; every lane receives both.  v must not be NaN.
__device__ __forceinline__ void wave_argmax(double& v, int& s) {
    const double vm = wave_max_f64(v);
    const uint64_t tied = __ballot(v == vm);
    if (__popcll(tied) == 1)
        s = __builtin_amdgcn_readlane(s, (int)__ffsll((unsigned long long)tied) - 1);
    else
        s = wave_min_i32(v == vm ? s : INT_MAX);
    v = vm;
}

constexpr int kQueueGroups = 16;

// The NormQueue of Sec. 2.3 for one run (block = run), one wave: psi[m] is the
// root at the largest stable p of diagonal m (0 if none); k times the largest
// psi (lowest m on ties) is reported as max x + max y + log(psi) and its
// diagonal, psi^p is subtracted from every sigma^(p)[m] (in place) and psi[m]
// is estimated again.  Within a pop the powers and roots go through one
// log psi (exp(p log psi), exp(log S / p)): the same values as pow to a few
// ulp, at half its cost on this serial path.
template <typename T>
__global__ __launch_bounds__(64) void mt_xy_queue_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                       int64_t n, MaxconvSpec spec, double* __restrict__ sigma,
                                                       const double* __restrict__ psi0, int32_t k,
                                                       double* __restrict__ values0,
                                                       double* __restrict__ values1, int32_t* __restrict__ diag0,
                                                       int32_t* __restrict__ diag1) {
    extern __shared__ double psi[];  // 2n - 1
    __shared__ double gv[64 * kQueueGroups];
    __shared__ int gm[64 * kQueueGroups];
    const int lane = threadIdx.x, run = blockIdx.x;
    const int L = (int)(2 * n - 1), np = spec.n;
    double* sg = sigma + (int64_t)run * np * L;
    double* values = run ? values1 : values0;
    int32_t* diag = run ? diag1 : diag0;

    double mx = -INFINITY, my = -INFINITY;
    for (int i = lane; i < n; i += 64) {
        mx = fmax(mx, (double)x[i]);
        my = fmax(my, (double)y[i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    const double shift = mx + my;
    for (int m = lane; m < L; m += 64) psi[m] = psi0[(int64_t)run * L + m];
    __syncthreads();
    // The lane owns m = lane + 64 c, c < C, in kQueueGroups groups of GS
    // consecutive c; gv / gm hold each group's largest psi and its m (lowest m
    // on ties), bv / bm the lane's.  A pop rescans one group.
    const int C = (L + 63) / 64;
    const int GS = (C + kQueueGroups - 1) / kQueueGroups;
    double* gvl = gv + lane * kQueueGroups;
    int* gml = gm + lane * kQueueGroups;
    auto group_scan = [&](int g) {
        double v = -1.0;
        int mm = L;
        const int c1 = (g + 1) * GS < C ? (g + 1) * GS : C;
        for (int c = g * GS; c < c1; ++c) {
            const int m = lane + 64 * c;
            if (m < L) {
                const double e = psi[m];
                if (e > v) {
                    v = e;
                    mm = m;
                }
            }
        }
        gvl[g] = v;
        gml[g] = mm;
    };
    double bv = -1.0;
    int bm = L;
    auto lane_best = [&]() {
        bv = -1.0;
        bm = L;
#pragma unroll
        for (int g = 0; g < kQueueGroups; ++g) {
            const double v = gvl[g];
            if (v > bv) {
                bv = v;
                bm = gml[g];
            }
        }
    };
    for (int g = 0; g < kQueueGroups; ++g) group_scan(g);
    lane_best();
    for (int r = 0; r < k; ++r) {
        double a = bv;
        int ms = bm;
        wave_argmax(a, ms);
        // log psi once for the value and every power (psi = 0: -inf, power 0)
        const double la = a > 0.0 ? log(a) : -INFINITY;
        if (lane == 0) {
            values[r] = shift + la;
            diag[r] = ms;
        }
        double s = 0.0;
        bool st = false;
        if (lane < np) {
            double* cell = sg + (int64_t)lane * L + ms;
            s = *cell - exp(la * (double)spec.p[lane]);
            *cell = s;
            st = s >= spec.tau;
        }
        const uint64_t mask = __ballot(st);
        double e = 0.0;
        if (mask) {
            const int qh = 63 - __clzll(mask);
            e = exp(log(__shfl(s, qh)) * (1.0 / (double)spec.p[qh]));
        }
        if (lane == 0) psi[ms] = e;
        __syncthreads();
        if (lane == (ms & 63)) {
            group_scan((ms >> 6) / GS);
            lane_best();
        }
    }
}

// Index recovery (Sec. 2.3): rank r has diagonal m1 = i + j in run 0 and
// anti-diagonal m2 = i + (n - 1 - j) in run 1, so i = (m1 + m2 - n + 1) / 2,
// j = m1 - i; -1 where that is not an integer pair in the n x n grid.
__global__ __launch_bounds__(256) void mt_xy_index_kernel(const int32_t* __restrict__ d0,
                                                         const int32_t* __restrict__ d1, int32_t k, int64_t n,
                                                         int32_t* __restrict__ diag, int32_t* __restrict__ ii,
                                                         int32_t* __restrict__ jj) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= k) return;
    const int64_t m1 = d0[r], m2 = d1[r];
    const int64_t sum = m1 + m2 - (n - 1);
    int64_t i = (sum & 1) == 0 ? sum / 2 : -1;
    int64_t j = i >= 0 ? m1 - i : -1;
    if (!(i >= 0 && i < n && j >= 0 && j < n)) i = j = -1;
    if (diag) diag[r] = (int32_t)m1;
    if (ii) ii[r] = (int32_t)i;
    if (jj) jj[r] = (int32_t)j;
}

// ---- the paired queue (Discussion) -------------------------------------
//
// Within k pops a run only ever pops diagonals among the K = min(k, 2n - 1)
// largest initial estimates (lowest m on ties): an estimate changes only
// when its diagonal is popped, so a diagonal's first pop takes the largest
// never-popped estimate, and at most k diagonals are popped.  The paired
// queue therefore works on those K candidates per run, held in LDS.

constexpr int kSelThreads = 1024;
constexpr int kSelPer = kLongConvN / kSelThreads;  // covers 2n - 1 < kLongConvN

// Block-wide exclusive sum of v over threads in thread order; every thread
// of the block calls it.
__device__ __forceinline__ uint32_t block_sum_before(uint32_t v, uint32_t* wtot) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(inc, o);
        if (lane >= o) inc += t;
    }
    if (lane == 63) wtot[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
#pragma unroll
    for (int w2 = 0; w2 < kSelThreads / 64; ++w2) before += w2 < wv ? wtot[w2] : 0u;
    return before + inc - v;
}

// The K candidates of each run (block = run): the K largest psi, lowest m
// on ties, written in ascending m with their sigma columns
// (cand_cols[(run np + q) K + slot]).  psi >= 0, so its bit pattern orders as
// its value; the K-th largest key is found by an 8-bit radix select, then
// the keys above it and the first keys equal to it (in m order) are kept.
__global__ __launch_bounds__(kSelThreads) void mt_xy_select_kernel(const double* __restrict__ psi, int L, int K,
                                                                   const double* __restrict__ sigma, int np,
                                                                   int32_t* __restrict__ cand_m,
                                                                   double* __restrict__ cand_psi,
                                                                   double* __restrict__ cand_cols) {
    __shared__ uint32_t hist[256];
    __shared__ int s_bin, s_above;
    __shared__ uint32_t wtot[kSelThreads / 64];
    __shared__ int taken_m[kPairedMaxK];
    const int tid = threadIdx.x, run = blockIdx.x, lane = tid & 63;
    const double* ps = psi + (int64_t)run * L;
    if (tid == 0) s_bin = s_above = 0;
    uint64_t key[kSelPer];
    // thread tid owns m = kSelPer tid + c: thread order is m order
#pragma unroll
    for (int c = 0; c < kSelPer; ++c) {
        const int m = kSelPer * tid + c;
        key[c] = m < L ? (uint64_t)__double_as_longlong(ps[m]) : 0ull;
    }
    uint64_t prefix = 0, mask = 0;
    int need = K;  // keys still to take among those matching prefix
    for (int d = 7; d >= 0; --d) {
        const int shift = 8 * d;
        if (tid < 256) hist[tid] = 0u;
        __syncthreads();
        // the high digits of psi's bits are shared by almost every key: when
        // a wave's counted keys all fall in one bin, one lane adds them
#pragma unroll
        for (int c = 0; c < kSelPer; ++c) {
            const bool counted = kSelPer * tid + c < L && (key[c] & mask) == prefix;
            const uint32_t bin = (uint32_t)(key[c] >> shift) & 255u;
            const uint64_t act = __ballot(counted);
            if (act == 0) continue;
            const uint32_t b0 = (uint32_t)__builtin_amdgcn_readlane((int)bin, (int)__ffsll((unsigned long long)act) - 1);
            if (__ballot(counted && bin == b0) == act) {
                if (lane == 0) atomicAdd(&hist[b0], (uint32_t)__popcll(act));
            } else if (counted) {
                atomicAdd(&hist[bin], 1u);
            }
        }
        __syncthreads();
        if (tid < 64) {
            // lane l holds bins 255 - 4l .. 252 - 4l (descending)
            int h[4], tot = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                h[u] = (int)hist[255 - 4 * lane - u];
                tot += h[u];
            }
            int inc = tot;
            for (int o = 1; o < 64; o <<= 1) {
                const int t = __shfl_up(inc, o);
                if (lane >= o) inc += t;
            }
            const int exc = inc - tot;
            if (exc < need && inc >= need) {
                int cum = exc, b = -1;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (b < 0) {
                        if (cum + h[u] >= need)
                            b = 255 - 4 * lane - u;
                        else
                            cum += h[u];
                    }
                }
                s_bin = b;
                s_above = cum;
            }
        }
        __syncthreads();
        prefix |= (uint64_t)s_bin << shift;
        mask |= 255ull << shift;
        need -= s_above;
        __syncthreads();
    }
    // keys above the threshold, and the first `need` keys equal to it in m
    // order: one block scan of the per-thread counts (above | equal << 16)
    uint32_t n_gt = 0, n_eq = 0;
#pragma unroll
    for (int c = 0; c < kSelPer; ++c) {
        const bool ok = kSelPer * tid + c < L;
        n_gt += ok && key[c] > prefix ? 1u : 0u;
        n_eq += ok && key[c] == prefix ? 1u : 0u;
    }
    const uint32_t before = block_sum_before(n_gt | (n_eq << 16), wtot);
    const int gt_before = (int)(before & 0xffffu), eq_before = (int)(before >> 16);
    int pos = gt_before + (eq_before < need ? eq_before : need), eq_rank = eq_before;
#pragma unroll
    for (int c = 0; c < kSelPer; ++c) {
        const int m = kSelPer * tid + c;
        const bool ok = m < L;
        const bool gt = ok && key[c] > prefix, eq = ok && key[c] == prefix;
        const bool take = gt || (eq && eq_rank < need);
        eq_rank += eq ? 1 : 0;
        if (take && pos < K) {
            cand_m[(int64_t)run * K + pos] = m;
            cand_psi[(int64_t)run * K + pos] = __longlong_as_double((long long)key[c]);
            taken_m[pos] = m;
        }
        pos += take ? 1 : 0;
    }
    __syncthreads();
    // the candidates' columns, every thread gathering (q, slot) cells
    const double* sg = sigma + (int64_t)run * np * L;
    double* cc = cand_cols + (int64_t)run * np * K;
    for (int u = tid; u < np * K; u += kSelThreads) {
        const int q = u / K, slot = u - q * K;
        cc[u] = sg[(int64_t)q * L + taken_m[slot]];
    }
}

__device__ __forceinline__ int diag_len(int m, int n) { return (m < 2 * n - 2 - m ? m : 2 * n - 2 - m) + 1; }

// A lane's candidate slots held in registers (slot u * 32 + q of its run in
// entry u, q = lane % 32): the largest log psi, the first valid slot on ties
// and all -inf.
template <int kS>
__device__ __forceinline__ void slots_best(const double (&rv)[kS], const int (&rm)[kS], int q, int K, double& bv,
                                           int& bs, int& bm) {
    bv = -INFINITY;
    bs = K;
    bm = 0;
#pragma unroll
    for (int u = 0; u < kS; ++u) {
        const int s = u * 32 + q;
        if (s < K && (bs == K || rv[u] > bv)) {
            bv = rv[u];
            bs = s;
            bm = rm[u];
        }
    }
}

template <int kS>
__device__ __forceinline__ void slots_set(double (&rv)[kS], int u, double e) {
#pragma unroll
    for (int w = 0; w < kS; ++w)
        if (w == u) rv[w] = e;
}

// The largest v of each half wave (lanes 0..31 and 32..63) and, among the
// lanes of that half holding it, the smallest s: row_shr 1, 2, 4, 8 leave
// each row's maximum in its lane 15, row_bcast:15 into rows 1 and 3 brings
// the two rows of a half together in lanes 31 and 63.  v must not be NaN.
__device__ __forceinline__ void half_argmax(double v, int s, double& a0, int& s0, double& a1, int& s1) {
    double m = v;
    m = fmax(m, dpp_f64<0x111, 0xf>(m));
    m = fmax(m, dpp_f64<0x112, 0xf>(m));
    m = fmax(m, dpp_f64<0x114, 0xf>(m));
    m = fmax(m, dpp_f64<0x118, 0xf>(m));
    m = fmax(m, dpp_f64<0x142, 0xa>(m));
    a0 = readlane_f64(m, 31);
    a1 = readlane_f64(m, 63);
    const bool tie = v == ((threadIdx.x & 32) ? a1 : a0);
    const uint64_t t = __ballot(tie);
    const uint32_t t0 = (uint32_t)t, t1 = (uint32_t)(t >> 32);
    if (__popc(t0) == 1 && __popc(t1) == 1) {
        s0 = __builtin_amdgcn_readlane(s, __ffs(t0) - 1);
        s1 = __builtin_amdgcn_readlane(s, 32 + __ffs(t1) - 1);
        return;
    }
    int w = tie ? s : INT_MAX;
    w = min(w, dpp_i32<0x111, 0xf>(w));
    w = min(w, dpp_i32<0x112, 0xf>(w));
    w = min(w, dpp_i32<0x114, 0xf>(w));
    w = min(w, dpp_i32<0x118, 0xf>(w));
    w = min(w, dpp_i32<0x142, 0xa>(w));
    s0 = __builtin_amdgcn_readlane(w, 31);
    s1 = __builtin_amdgcn_readlane(w, 63);
}

// Both runs' NormQueues in lockstep, one wave, over the candidates: each
// rank pops run 0 (diagonals i + j) and run 1 (anti-diagonals
// i + n - 1 - j) together.  Plain (Sec. 2.3): each run subtracts its own
// estimate and the indices are recovered from the two diagonals.  Paired
// (Discussion): the pair (i, j) the two diagonals meet in is accurate when it
// lies in the grid, no earlier rank reported it (a list in LDS, scanned by
// every lane), and its scaled value v = e^(x_i - max x + y_j - max y) is at
// least psi len^(-1/p*) on both diagonals (the smallest largest term their
// norms admit; none on a diagonal without a stable p); an accurate rank
// reports x_i + y_j and (i, j) and subtracts v^p from both runs, any other
// reports run 0's estimate and i = j = -1, and each run subtracts its own
// estimate.  Lanes 0..31 hold run 0's powers and candidates, lanes 32..63
// run 1's; candidate slot s of run t belongs to lane 32 t + s % 32.  The
// candidates' sigma
// columns are updated in LDS when they fit (kColsLds), else in the
// workspace copy; with kRegS > 0 (K <= 32 kRegS) a lane's slots, estimates
// and diagonals, stay in registers.  The log diagonal lengths of the paired
// acceptance test are kept in LDS when they fit (kLenLds), else taken from
// the popped diagonals each rank (the same values).
template <typename T, bool kPaired, bool kColsLds, int kRegS, bool kLenLds>
__global__ __launch_bounds__(64) void mt_xy_lockstep_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                          int64_t n, MaxconvSpec spec,
                                                          const int32_t* __restrict__ cand_m,
                                                          const double* __restrict__ cand_psi,
                                                          double* __restrict__ cand_cols, int K, int32_t k,
                                                          double* __restrict__ values, int32_t* __restrict__ diag,
                                                          int32_t* __restrict__ anti, int32_t* __restrict__ ii,
                                                          int32_t* __restrict__ jj) {
    // LDS: 2K log estimates, [2K log diagonal lengths], [2 np K column
    // cells], 2K diagonals, [k reported pairs (paired)].  The queue keeps log psi: the argmax
    // order is psi's, the reported value needs the log, the subtraction
    // exp(p log psi) and the new root exp(log S / p) then need no log or exp
    // of their own.
    extern __shared__ double cv[];
    const int lane = threadIdx.x;
    const int np = spec.n, nn = (int)n;
    constexpr int kLen = kPaired && kLenLds ? 1 : 0;
    double* cl = cv + 2 * K;  // used when kLen
    double* cols = kColsLds ? cv + (2 + 2 * kLen) * K : cand_cols;
    int* cm = (int*)(cv + (2 + 2 * kLen) * K + (kColsLds ? 2 * np * K : 0));
    int* done = cm + 2 * K;  // paired only
    int n_done = 0;
    double mx = -INFINITY, my = -INFINITY;
    for (int i = lane; i < nn; i += 64) {
        mx = fmax(mx, (double)x[i]);
        my = fmax(my, (double)y[i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    const double shift = mx + my;
    for (int s = lane; s < 2 * K; s += 64) {
        const double e = cand_psi[s];
        const int m = cand_m[s];
        cv[s] = e > 0.0 ? log(e) : -INFINITY;
        if (kLen) cl[s] = log((double)diag_len(m, nn));
        cm[s] = m;
    }
    if (kColsLds)
        for (int s = lane; s < 2 * np * K; s += 64) cols[s] = cand_cols[s];
    __syncthreads();
    const int half = lane >> 5, q = lane & 31;
    const int S = (K + 31) / 32;
    // the lane's largest log psi of its run and its slot (the first valid
    // slot always counts, so a run whose estimates are all -inf still names
    // its lowest)
    auto lane_best = [&](double& bv, int& bs) {
        bv = -INFINITY;
        bs = K;
        for (int u = 0; u < S; ++u) {
            const int s = u * 32 + q;
            if (s < K) {
                const double e = cv[half * K + s];
                if (bs == K || e > bv) {
                    bv = e;
                    bs = s;
                }
            }
        }
    };
    constexpr int kSR = kRegS > 0 ? kRegS : 1;
    double rv[kSR];
    int rm[kSR];
    double bv;
    int bs, bm;
    if (kRegS > 0) {
#pragma unroll
        for (int u = 0; u < kSR; ++u) {
            const int s = u * 32 + q;
            rv[u] = s < K ? cv[half * K + s] : -INFINITY;
            rm[u] = s < K ? cm[half * K + s] : 0;
        }
        slots_best(rv, rm, q, K, bv, bs, bm);
    } else {
        lane_best(bv, bs);
        bm = bs < K ? cm[half * K + bs] : 0;
    }
    const bool mine = q < np;
    // this lane's power and its reciprocal; a rank picks other lanes' by readlane
    const double pw = mine ? (double)spec.p[q] : 1.0, ipw = 1.0 / pw;
    for (int r = 0; r < k; ++r) {
        double a0, a1;
        int s0, s1;
        half_argmax(bv, bs, a0, s0, a1, s1);
        const int m1 = __builtin_amdgcn_readlane(bm, s0 & 31), m2 = __builtin_amdgcn_readlane(bm, 32 + (s1 & 31));
        const int sd = m1 + m2 - (nn - 1);
        const int i = sd >> 1, j = m1 - i;
        bool valid = (sd & 1) == 0 && sd >= 0 && i < nn && j >= 0 && j < nn;
        double* cp = cols + (half * np + q) * K + (half ? s1 : s0);
        double cell = 0.0;
        if (mine) cell = *cp;
        const double la0 = a0, la1 = a1;
        bool acc = false;
        double xi = 0.0, yj = 0.0, lv = 0.0;
        const int id = i * nn + j;
        if (kPaired) {
            if (valid) {
                xi = (double)x[i];
                yj = (double)y[j];
            }
            bool seen = false;
            if (valid)
                for (int u = lane; u < n_done; u += 64) seen |= done[u] == id;
            valid = valid && __ballot(seen) == 0;
            const uint64_t st = __ballot(mine && cell >= spec.tau);
            const uint32_t lo_b = (uint32_t)st, hi_b = (uint32_t)(st >> 32);
            const int q0 = lo_b ? 31 - __clz(lo_b) : -1, q1 = hi_b ? 31 - __clz(hi_b) : -1;
            // in logs: log v >= log psi - log(len) / p* on both diagonals
            lv = (xi - mx) + (yj - my);
            const double ll0 = kLen ? cl[s0] : log((double)diag_len(m1, nn));
            const double ll1 = kLen ? cl[K + s1] : log((double)diag_len(m2, nn));
            acc = valid && q0 >= 0 && q1 >= 0 && lv >= la0 - ll0 * readlane_f64(ipw, q0 >= 0 ? q0 : 0) &&
                  lv >= la1 - ll1 * readlane_f64(ipw, q1 >= 0 ? 32 + q1 : 32);
        }
        const double la = acc ? lv : (half ? la1 : la0);
        double s = 0.0;
        bool ns = false;
        if (mine) {
            s = cell - exp(la * pw);
            *cp = s;
            ns = s >= spec.tau;
        }
        const uint64_t nm = __ballot(ns);
        const uint32_t nlo = (uint32_t)nm, nhi = (uint32_t)(nm >> 32);
        const int h0 = nlo ? 31 - __clz(nlo) : -1, h1 = nhi ? 31 - __clz(nhi) : -1;
        const int l0 = h0 >= 0 ? h0 : 0, l1 = h1 >= 0 ? 32 + h1 : 32;
        // both runs' new roots in one log: half 0 takes run 0's sum, half 1 run 1's
        const double sh = half ? readlane_f64(s, l1) : readlane_f64(s, l0);
        const double ih = half ? readlane_f64(ipw, l1) : readlane_f64(ipw, l0);
        const double lr = log(sh) * ih;
        const double e0 = h0 >= 0 ? readlane_f64(lr, 0) : -INFINITY;
        const double e1 = h1 >= 0 ? readlane_f64(lr, 32) : -INFINITY;
        if (lane == 0) {
            values[r] = acc ? xi + yj : shift + la0;
            if (diag) diag[r] = m1;
            anti[r] = m2;
            const bool give = kPaired ? acc : valid;
            if (ii) ii[r] = give ? i : -1;
            if (jj) jj[r] = give ? j : -1;
            if (kPaired && acc) done[n_done] = id;
        }
        n_done += acc ? 1 : 0;
        // the owner of each popped slot (one lane per half) takes its new
        // estimate and rescans its slots
        const int so = half ? s1 : s0;
        if (q == (so & 31)) {
            const double e = half ? e1 : e0;
            if (kRegS > 0) {
                slots_set(rv, so >> 5, e);
                slots_best(rv, rm, q, K, bv, bs, bm);
            } else {
                cv[half * K + so] = e;
                lane_best(bv, bs);
                bm = cm[half * K + bs];
            }
        }
    }
}

// Long transforms (N = 8192 or 16384, up to kLongConvN): every transform of
// the batch in a global buffer [slot][N], the four-step transform below
// going through two such buffers.

// exp(-2 pi i mm / N), 0 <= mm < N, from the octant table (runtime N, N4 = N / 4).
__device__ __forceinline__ double2 twiddle_rt(const double2* tw, int mm, int N4) {
    const int q = mm / N4, r = mm & (N4 - 1);
    const bool refl = r > N4 / 2;
    const double2 t = tw[refl ? N4 - r : r];
    double a = refl ? t.y : t.x, b = refl ? -t.x : -t.y;
    if (q & 1) {
        const double c = a;
        a = b;
        b = -c;
    }
    if (q & 2) {
        a = -a;
        b = -b;
    }
    return make_double2(a, b);
}

// cos / sin (2 pi k / N), k = 0 .. N / 8; the maxima of x and y in mxy[0], mxy[1].
template <typename T>
__global__ __launch_bounds__(1024) void mt_xy_long_setup_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                               int64_t n, int N, double2* __restrict__ tw,
                                                               double* __restrict__ mxy) {
    __shared__ double red[2][16];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int k = tid; k <= N / 8; k += 1024) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)N, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
    double mx = -INFINITY, my = -INFINITY;
    for (int64_t i = tid; i < n; i += 1024) {
        mx = fmax(mx, (double)x[i]);
        my = fmax(my, (double)y[i]);
    }
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    if (lane == 0) {
        red[0][wave] = mx;
        red[1][wave] = my;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 16; ++w) {
            mx = fmax(mx, red[0][w]);
            my = fmax(my, red[1][w]);
        }
        mxy[0] = mx;
        mxy[1] = my;
    }
}

// cos / sin (2 pi k / N), k = 0 .. N / 8.
__global__ __launch_bounds__(256) void mt_twiddle_octant_kernel(double2* __restrict__ tw, int N) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > N / 8) return;
    double sn, cs;
    sincospi(2.0 * (double)k / (double)N, &sn, &cs);
    tw[k] = make_double2(cs, sn);
}

// buf[slot][t] = (x'^p, y'^p) for slot = run |P| + q, zero for t >= n.
template <typename T>
__global__ __launch_bounds__(256) void mt_xy_long_load_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                             int64_t n, int logN, MaxconvSpec spec,
                                                             const double* __restrict__ mxy,
                                                             double2* __restrict__ buf) {
    const int N = 1 << logN;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (int64_t)2 * spec.n * N) return;
    const int slot = (int)(g >> logN), t = (int)(g & (N - 1));
    const int run = slot / spec.n, p = spec.p[slot % spec.n];
    double a = 0.0, c = 0.0;
    if (t < n) {
        a = ipow_d(exp((double)x[t] - mxy[0]), p);
        c = ipow_d(exp((double)y[run ? n - 1 - t : t] - mxy[1]), p);
    }
    buf[g] = make_double2(a, c);
}

// Four-step transform of the long lengths (N = N1 N2, N1 = 128, N2 = 64 or
// 128): with n = N2 n1 + n2 and k = k1 + N1 k2,
//   X[k] = sum_n2 W_N2^(n2 k2) W_N^(n2 k1) sum_n1 x[N2 n1 + n2] W_N1^(n1 k1),
// so one kernel transforms the N2 columns (length N1, stride N2) and applies
// W_N^(n2 k1), storing Y[k1 N2 + n2]; a second transforms the N1 rows of Y
// (length N2, contiguous) and stores X[k1 + N1 k2].  Each workgroup holds
// kF4Cols transforms of M points in LDS and runs Stockham stages there, so a
// direction reads and writes the buffer twice instead of once per radix pass.
constexpr int kF4Cols = 8;
constexpr int kF4Threads = 128;

template <int M, int R>
__device__ __forceinline__ void f4_stage(double2* buf, int Ns, int N, const double2* tw) {
    constexpr int MR = M / R;
    const int t = threadIdx.x;
    const bool act = t < kF4Cols * MR;
    double2 v[16];
    int c = 0, j = 0, k0 = 0;
    if (act) {
        c = t / MR;
        j = t - c * MR;
        k0 = j & (Ns - 1);
#pragma unroll
        for (int e = 0; e < R; ++e) v[e] = buf[c * (M + 1) + j + e * MR];
        if (Ns > 1) {
            const int step = k0 * (N / (Ns * R));
#pragma unroll
            for (int e = 1; e < R; ++e) v[e] = cmul(v[e], twiddle_rt(tw, step * e, N / 4));
        }
        dft<R>(v, 0, 1);
    }
    __syncthreads();
    if (act) {
        const int base = (j - k0) * R + k0;
#pragma unroll
        for (int e = 0; e < R; ++e) buf[c * (M + 1) + base + e * Ns] = v[oreg<R>(e)];
    }
    __syncthreads();
}

// One step of the four-step transform for every transform of the batch:
// workgroup g takes transform g / groups_per_tr and its kF4Cols consecutive
// columns (or rows) from (g % groups_per_tr) kF4Cols.  Element i of line c
// is in[i s_in + c c_in]; result k of line c goes to out[k s_out + c]
// (multiplied by W_N^(c k) when twiddle).  Lines are contiguous in memory
// when c_in = 1 (columns) and elements are when s_in = 1 (rows).
template <int M>
__global__ __launch_bounds__(kF4Threads) void mt_fft4_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                    int logN, int groups_per_tr, int s_in, int c_in, int s_out,
                                                    int twiddle, const double2* __restrict__ tw) {
    __shared__ double2 buf[kF4Cols * (M + 1)];
    const int t = threadIdx.x;
    const int N = 1 << logN;
    const int64_t tr = blockIdx.x / groups_per_tr;
    const int c0 = (int)(blockIdx.x - tr * groups_per_tr) * kF4Cols;
    const double2* src = in + tr * N;
    double2* dst = out + tr * N;
    for (int idx = t; idx < kF4Cols * M; idx += kF4Threads) {
        const int i = c_in == 1 ? idx / kF4Cols : idx % M;
        const int c = c_in == 1 ? idx % kF4Cols : idx / M;
        buf[c * (M + 1) + i] = src[i * s_in + (c0 + c) * c_in];
    }
    __syncthreads();
    f4_stage<M, 16>(buf, 1, N, tw);
    f4_stage<M, M / 16>(buf, 16, N, tw);
    for (int idx = t; idx < kF4Cols * M; idx += kF4Threads) {
        const int k = idx / kF4Cols, c = idx % kF4Cols;
        double2 v = buf[c * (M + 1) + k];
        if (twiddle) v = cmul(v, twiddle_rt(tw, ((c0 + c) * k) & (N - 1), N / 4));
        dst[k * s_out + c0 + c] = v;
    }
}

// conj(4 W_t) of every transform from Z_t and Z_(N-t) (see convolve_pair).
__global__ __launch_bounds__(256) void mt_fft_product_kernel(const double2* __restrict__ Z, double2* __restrict__ out,
                                                            int logN, int64_t total) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total) return;
    const int N = 1 << logN;
    const int64_t base = g & ~(int64_t)(N - 1);
    const int t = (int)(g & (N - 1));
    const double2 zk = Z[g], zn = Z[base + ((N - t) & (N - 1))];
    const double2 a = make_double2(zk.x + zn.x, zk.y - zn.y);
    const double2 c = make_double2(zk.y + zn.y, zn.x - zk.x);
    const double2 w = cmul(a, c);
    out[g] = make_double2(w.x, -w.y);
}

// sigma[slot][t] = Re(result)[t] * 0.25 / N for t < L.
__global__ __launch_bounds__(256) void mt_xy_long_store_kernel(const double2* __restrict__ res, int logN, int64_t L,
                                                              int64_t slots, double* __restrict__ sigma) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= slots * L) return;
    const int64_t slot = g / L, t = g - slot * L;
    sigma[g] = res[(slot << logN) + t].x * (0.25 / (double)(1 << logN));
}

// Max-convolution of long vectors (kMaxConvN < N <= kLongConvN): the batch of
// pairs through the four-step transforms in global buffers, one p at a time
// (largest first); every index keeps the S of its first stable p (code = its
// family index) and the roots are taken at the end.  No early exit.
constexpr uint8_t kCodeOpen = 254;

// Per pair: rxy[pair] = max x max y, inv[2 pair] = 1 / max x, inv[2 pair + 1] = 1 / max y.
template <typename T>
__global__ __launch_bounds__(256) void mt_maxconv_long_scale_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                                   int64_t n, int64_t m, double* __restrict__ rxy,
                                                                   double* __restrict__ inv) {
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t pair = blockIdx.x;
    double mx = 0.0, my = 0.0;
    for (int64_t i = tid; i < n; i += 256) mx = fmax(mx, (double)x[pair * n + i]);
    for (int64_t i = tid; i < m; i += 256) my = fmax(my, (double)y[pair * m + i]);
    for (int d = 32; d >= 1; d >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, d));
        my = fmax(my, __shfl_xor(my, d));
    }
    if (lane == 0) {
        red[0][wave] = mx;
        red[1][wave] = my;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < 4; ++w) {
            mx = fmax(mx, red[0][w]);
            my = fmax(my, red[1][w]);
        }
        rxy[pair] = mx * my;
        inv[2 * pair] = mx > 0.0 ? 1.0 / mx : 0.0;
        inv[2 * pair + 1] = my > 0.0 ? 1.0 / my : 0.0;
    }
}

// buf[pair][t] = (x'^p, y'^p), zero beyond the vectors.
template <typename T>
__global__ __launch_bounds__(256) void mt_maxconv_long_load_kernel(const T* __restrict__ x, const T* __restrict__ y,
                                                                  int64_t b, int64_t n, int64_t m, int logN, int p,
                                                                  const double* __restrict__ inv,
                                                                  double2* __restrict__ buf) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= (b << logN)) return;
    const int64_t pair = g >> logN;
    const int64_t t = g & ((1 << logN) - 1);
    const double a = t < n ? ipow_d((double)x[pair * n + t] * inv[2 * pair], p) : 0.0;
    const double c = t < m ? ipow_d((double)y[pair * m + t] * inv[2 * pair + 1], p) : 0.0;
    buf[g] = make_double2(a, c);
}

// The p* test of family index q for every index still open.
__global__ __launch_bounds__(256) void mt_maxconv_long_select_kernel(const double2* __restrict__ res, int logN,
                                                                    int64_t b, int64_t L, int q, double tau,
                                                                    double* __restrict__ s_sel,
                                                                    uint8_t* __restrict__ code) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b * L) return;
    if (code[g] != kCodeOpen) return;
    const int64_t pair = g / L, t = g - pair * L;
    const double S = res[(pair << logN) + t].x * (0.25 / (double)(1 << logN));
    const bool stable = S >= tau;
    if (stable || q == 0) {
        s_sel[g] = S;
        code[g] = stable ? (uint8_t)q : (uint8_t)MT_PSTAR_NONE;
    }
}

__global__ __launch_bounds__(256) void mt_fill_u8_kernel(uint8_t* __restrict__ p, int64_t count, uint8_t v) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g < count) p[g] = v;
}

// z = max x max y S^(1/p) at the selected p (the smallest p with S clamped
// at 0 where none was stable), p* = its code.
template <typename T>
__global__ __launch_bounds__(256) void mt_maxconv_long_root_kernel(const double* __restrict__ s_sel,
                                                                  const uint8_t* __restrict__ code,
                                                                  const double* __restrict__ rxy, int64_t b,
                                                                  int64_t L, MaxconvSpec spec, T* __restrict__ z,
                                                                  uint8_t* __restrict__ pstar) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= b * L) return;
    const uint8_t c = code[g];
    const int p = spec.p[c == MT_PSTAR_NONE ? 0 : c];
    const double S = s_sel[g];
    double root = 0.0;
    if (S > 0.0) {
        if ((p & (p - 1)) == 0) {
            root = S;
            for (int e = p; e > 1; e >>= 1) root = sqrt(root);
        } else {
            root = exp(log(S) / (double)p);
        }
    }
    z[g] = (T)(rxy[g / L] * root);
    if (pstar) pstar[g] = c;
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
    int logN = kConvMinLog;
    while ((int64_t(1) << logN) < L) ++logN;
    return logN;
}

namespace {

template <typename T, int LOGN>
hipError_t launch_maxconv_n(const T* x, const T* y, int64_t b, int64_t n, int64_t m, const MaxconvSpec& spec,
                            T* z, uint8_t* pstar, hipStream_t st) {
    auto kern = mt_maxconv_kernel<T, LOGN>;
    const int lds = (kConvTwElems + kConvLdsElems) * (int)sizeof(double2);
    // the dynamic-LDS limit is a per-device attribute of each kernel
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
    constexpr int G = Fft<LOGN>::G;
    const int64_t blocks = (b + G - 1) / G;
    timing_before("mt_maxconv", st);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kConvThreads), lds, st, x, y, b, n, m, spec, z, pstar,
                       timing_work_slot());
    timing_after(st);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_maxconv_t(const T* x, const T* y, int64_t b, int64_t n, int64_t m, const MaxconvSpec& spec,
                            T* z, uint8_t* pstar, hipStream_t st) {
    switch (maxconv_log_size(n, m)) {
        case 4: return launch_maxconv_n<T, 4>(x, y, b, n, m, spec, z, pstar, st);
        case 5: return launch_maxconv_n<T, 5>(x, y, b, n, m, spec, z, pstar, st);
        case 6: return launch_maxconv_n<T, 6>(x, y, b, n, m, spec, z, pstar, st);
        case 7: return launch_maxconv_n<T, 7>(x, y, b, n, m, spec, z, pstar, st);
        case 8: return launch_maxconv_n<T, 8>(x, y, b, n, m, spec, z, pstar, st);
        case 9: return launch_maxconv_n<T, 9>(x, y, b, n, m, spec, z, pstar, st);
        case 10: return launch_maxconv_n<T, 10>(x, y, b, n, m, spec, z, pstar, st);
        case 11: return launch_maxconv_n<T, 11>(x, y, b, n, m, spec, z, pstar, st);
        case 12: return launch_maxconv_n<T, 12>(x, y, b, n, m, spec, z, pstar, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace


namespace {

template <typename T, int LOGN>
hipError_t launch_xy_sigma_n(const T* x, const T* y, int64_t n, const MaxconvSpec& spec, double* sigma,
                             hipStream_t st) {
    auto kern = mt_xy_sigma_kernel<T, LOGN>;
    const int lds = (kConvTwElems + kConvLdsElems) * (int)sizeof(double2);
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
    constexpr int G = Fft<LOGN>::G;
    const int blocks = (2 * spec.n + G - 1) / G;
    timing_before("mt_xy_sigma", st);
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(kConvThreads), lds, st, x, y, n, spec, sigma);
    timing_after(st);
    return hipGetLastError();
}

// The convolution step of every transform of a batch held in cur (count
// transforms of N = 2^logN points, (a, b) packed as a + i b): the forward
// passes, the product conj(4 X Y) and the inverse passes.  On return cur holds
// the result (real part 4 N (a * b)); nxt is scratch.
hipError_t long_convolve(double2*& cur, double2*& nxt, int logN, int64_t count, const double2* tw,
                         const char* pass_name, const char* product_name, hipStream_t st) {
    const int64_t total = count << logN;
    auto blocks = [](int64_t c) { return dim3((unsigned)((c + 255) / 256)); };
    auto swap = [&]() {
        double2* t = cur;
        cur = nxt;
        nxt = t;
    };
    // N = 8192 or 16384: the four-step transform (columns of 128, rows of N2)
    auto transform4 = [&]() -> hipError_t {
        const int N2 = 1 << (logN - 7);
        timing_before(pass_name, st);
        hipLaunchKernelGGL(mt_fft4_kernel<128>, dim3((unsigned)(count * (N2 / kF4Cols))), dim3(kF4Threads), 0, st, cur,
                           nxt, logN, N2 / kF4Cols, N2, 1, N2, 1, tw);
        timing_after(st);
        hipError_t pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
        swap();
        timing_before(pass_name, st);
        if (N2 == 128)
            hipLaunchKernelGGL(mt_fft4_kernel<128>, dim3((unsigned)(count * (128 / kF4Cols))), dim3(kF4Threads), 0, st,
                               cur, nxt, logN, 128 / kF4Cols, 1, N2, 128, 0, tw);
        else
            hipLaunchKernelGGL(mt_fft4_kernel<64>, dim3((unsigned)(count * (128 / kF4Cols))), dim3(kF4Threads), 0, st, cur,
                               nxt, logN, 128 / kF4Cols, 1, N2, 128, 0, tw);
        timing_after(st);
        pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
        swap();
        return hipSuccess;
    };
    if (logN != 13 && logN != 14) return hipErrorInvalidValue;
    hipError_t e = transform4();
    if (e != hipSuccess) return e;
    timing_before(product_name, st);
    hipLaunchKernelGGL(mt_fft_product_kernel, blocks(total), dim3(256), 0, st, cur, nxt, logN, total);
    timing_after(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    swap();
    return transform4();
}

// Max-convolution of long vectors through the global buffers of ws.
template <typename T>
hipError_t launch_maxconv_long(const T* x, const T* y, int64_t b, int64_t n, int64_t m, const MaxconvSpec& spec,
                               T* z, uint8_t* pstar, const MaxconvWorkspace& w, hipStream_t st) {
    const int logN = maxconv_log_size(n, m);
    const int N = 1 << logN;
    const int64_t L = n + m - 1;
    auto blocks = [](int64_t c) { return dim3((unsigned)((c + 255) / 256)); };
    timing_before("mt_maxconv_long_setup", st);
    hipLaunchKernelGGL(mt_twiddle_octant_kernel, blocks(N / 8 + 1), dim3(256), 0, st, w.tw, N);
    hipLaunchKernelGGL(mt_maxconv_long_scale_kernel<T>, dim3((unsigned)b), dim3(256), 0, st, x, y, n, m, w.rxy,
                       w.inv);
    hipLaunchKernelGGL(mt_fill_u8_kernel, blocks(b * L), dim3(256), 0, st, w.code, b * L, kCodeOpen);
    timing_after(st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int q = spec.n - 1; q >= 0; --q) {
        double2* cur = w.buf0;
        double2* nxt = w.buf1;
        timing_before("mt_maxconv_long_load", st);
        hipLaunchKernelGGL(mt_maxconv_long_load_kernel<T>, blocks(b << logN), dim3(256), 0, st, x, y, b, n, m, logN,
                           spec.p[q], w.inv, cur);
        timing_after(st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = long_convolve(cur, nxt, logN, b, w.tw, "mt_maxconv_long_pass", "mt_maxconv_long_product", st)) !=
            hipSuccess)
            return e;
        timing_before("mt_maxconv_long_select", st);
        hipLaunchKernelGGL(mt_maxconv_long_select_kernel, blocks(b * L), dim3(256), 0, st, cur, logN, b, L, q,
                           spec.tau, w.s_sel, w.code);
        timing_after(st);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    timing_before("mt_maxconv_long_root", st);
    hipLaunchKernelGGL(mt_maxconv_long_root_kernel<T>, blocks(b * L), dim3(256), 0, st, w.s_sel, w.code, w.rxy, b,
                       L, spec, z, pstar);
    timing_after(st);
    return hipGetLastError();
}

// The ring results of long lists (N > kMaxConvN) through global buffers.
template <typename T>
hipError_t launch_xy_long(const T* x, const T* y, int64_t n, const MaxconvSpec& spec, const XyWorkspace& w,
                          hipStream_t st) {
    const int logN = maxconv_log_size(n, n);
    const int N = 1 << logN;
    const int64_t slots = 2 * (int64_t)spec.n, total = slots * N, L = 2 * n - 1;
    auto blocks = [](int64_t count) { return dim3((unsigned)((count + 255) / 256)); };
    timing_before("mt_xy_sigma_setup", st);
    hipLaunchKernelGGL(mt_xy_long_setup_kernel<T>, dim3(1), dim3(1024), 0, st, x, y, n, N, w.tw, w.mxy);
    timing_after(st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_before("mt_xy_sigma_load", st);
    hipLaunchKernelGGL(mt_xy_long_load_kernel<T>, blocks(total), dim3(256), 0, st, x, y, n, logN, spec, w.mxy,
                       w.buf0);
    timing_after(st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    double2* cur = w.buf0;
    double2* nxt = w.buf1;
    if ((e = long_convolve(cur, nxt, logN, slots, w.tw, "mt_xy_sigma_pass", "mt_xy_sigma_product", st)) != hipSuccess)
        return e;
    timing_before("mt_xy_sigma_store", st);
    hipLaunchKernelGGL(mt_xy_long_store_kernel, blocks(slots * L), dim3(256), 0, st, cur, logN, L, slots, w.sigma);
    timing_after(st);
    return hipGetLastError();
}

// LDS bytes of the lockstep queue: log estimates and diagonals of 2K
// candidates; paired: the reported pairs and, when kept there, the log
// lengths; the 2 |P| K column cells when they are kept there.
size_t lockstep_lds(int K, int k, int np, bool paired, bool cols, bool lens) {
    return (size_t)2 * K * (sizeof(double) + sizeof(int)) +
           (paired ? (size_t)k * sizeof(int) + (lens ? (size_t)2 * K * sizeof(double) : 0) : 0) +
           (cols ? (size_t)2 * np * K * sizeof(double) : 0);
}
constexpr size_t kLdsBytes = 160 * 1024;

template <typename T, bool kPaired, bool kColsLds, int kRegS, bool kLenLds = true>
hipError_t launch_lockstep(const T* x, const T* y, int64_t n, int32_t k, int K, const MaxconvSpec& spec,
                           double* values, int32_t* diag, int32_t* ii, int32_t* jj, const XyWorkspace& w,
                           hipStream_t st) {
    auto queue = mt_xy_lockstep_kernel<T, kPaired, kColsLds, kRegS, kLenLds>;
    const size_t lds = lockstep_lds(K, k, spec.n, kPaired, kColsLds, kLenLds);
    if (lds > kLdsBytes) return hipErrorInvalidValue;
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_set.load() & bit)) {
        e = hipFuncSetAttribute((const void*)queue, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kLdsBytes);
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    timing_before(kPaired ? "mt_xy_paired" : "mt_xy_queue", st);
    hipLaunchKernelGGL(queue, dim3(1), dim3(64), lds, st, x, y, n, spec, w.cand_m,
                       w.cand_psi, w.cand_cols, K, k, values, diag, w.diag1, ii, jj);
    timing_after(st);
    return hipGetLastError();
}

// k <= kPairedMaxK: both runs in lockstep over their K = min(k, 2n - 1)
// candidates (plain or paired).
template <typename T>
hipError_t launch_xy_candidates(const T* x, const T* y, int64_t n, int32_t k, const MaxconvSpec& spec, bool paired,
                                double* values, int32_t* diag, int32_t* ii, int32_t* jj, const XyWorkspace& w,
                                hipStream_t st) {
    const int L = (int)(2 * n - 1), K = k < L ? k : L;
    if (k > kPairedMaxK || L >= kLongConvN || spec.n > 32) return hipErrorInvalidValue;
    timing_before("mt_xy_select", st);
    hipLaunchKernelGGL(mt_xy_select_kernel, dim3(2), dim3(kSelThreads), 0, st, w.psi, L, K, w.sigma, spec.n,
                       w.cand_m, w.cand_psi, w.cand_cols);
    timing_after(st);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // K <= 256: the columns always fit (at most 2 x 32 x 256 x 8 B plus
    // 40 K + 4 k bytes), and a lane's 8 slots of its run stay in registers.
    // The largest case, K = k = 4096, needs 40 K = 160 KiB plain and
    // 24 K + 4 k paired with the log lengths taken per rank.
    const bool cols = lockstep_lds(K, k, spec.n, paired, true, true) <= kLdsBytes;
    const bool regs = K <= 256 && cols;
    if (paired) {
        if (regs) return launch_lockstep<T, true, true, 8>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
        if (cols) return launch_lockstep<T, true, true, 0>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
        if (lockstep_lds(K, k, spec.n, true, false, true) <= kLdsBytes)
            return launch_lockstep<T, true, false, 0>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
        return launch_lockstep<T, true, false, 0, false>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
    }
    if (regs) return launch_lockstep<T, false, true, 8>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
    return cols ? launch_lockstep<T, false, true, 0>(x, y, n, k, K, spec, values, diag, ii, jj, w, st)
                : launch_lockstep<T, false, false, 0>(x, y, n, k, K, spec, values, diag, ii, jj, w, st);
}

template <typename T>
hipError_t launch_xy_t(const T* x, const T* y, int64_t n, int32_t k, const MaxconvSpec& spec, bool paired,
                       double* values, int32_t* diag, int32_t* ii, int32_t* jj, const XyWorkspace& w,
                       hipStream_t st) {
    hipError_t e = hipErrorInvalidValue;
    switch (maxconv_log_size(n, n)) {
        case 4: e = launch_xy_sigma_n<T, 4>(x, y, n, spec, w.sigma, st); break;
        case 5: e = launch_xy_sigma_n<T, 5>(x, y, n, spec, w.sigma, st); break;
        case 6: e = launch_xy_sigma_n<T, 6>(x, y, n, spec, w.sigma, st); break;
        case 7: e = launch_xy_sigma_n<T, 7>(x, y, n, spec, w.sigma, st); break;
        case 8: e = launch_xy_sigma_n<T, 8>(x, y, n, spec, w.sigma, st); break;
        case 9: e = launch_xy_sigma_n<T, 9>(x, y, n, spec, w.sigma, st); break;
        case 10: e = launch_xy_sigma_n<T, 10>(x, y, n, spec, w.sigma, st); break;
        case 11: e = launch_xy_sigma_n<T, 11>(x, y, n, spec, w.sigma, st); break;
        case 12: e = launch_xy_sigma_n<T, 12>(x, y, n, spec, w.sigma, st); break;
        case 13:
        case 14: e = launch_xy_long<T>(x, y, n, spec, w, st); break;
        default: break;
    }
    if (e != hipSuccess) return e;
    if (k <= 0) return hipSuccess;
    const int64_t L = 2 * n - 1;
    timing_before("mt_xy_psi", st);
    hipLaunchKernelGGL(mt_xy_psi_kernel, dim3((unsigned)((2 * L + 255) / 256)), dim3(256), 0, st, w.sigma, L, spec,
                       w.psi);
    timing_after(st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (k <= kPairedMaxK) return launch_xy_candidates<T>(x, y, n, k, spec, paired, values, diag, ii, jj, w, st);
    if (paired) return hipErrorInvalidValue;
    // psi of one run in LDS: up to 8 (kLongConvN - 1) bytes
    auto queue = mt_xy_queue_kernel<T>;
    static std::atomic<uint64_t> attr_set{0};
    int dev = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    const uint64_t bit = 1ull << (dev & 63);
    if (!(attr_set.load() & bit)) {
        e = hipFuncSetAttribute((const void*)queue, hipFuncAttributeMaxDynamicSharedMemorySize,
                                kLongConvN * (int)sizeof(double));
        if (e != hipSuccess) return e;
        attr_set.fetch_or(bit);
    }
    timing_before("mt_xy_queue", st);
    hipLaunchKernelGGL(queue, dim3(2), dim3(64), (size_t)L * sizeof(double), st, x, y, n, spec, w.sigma, w.psi, k,
                       values, w.values1, w.diag0, w.diag1);
    timing_after(st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    timing_before("mt_xy_index", st);
    hipLaunchKernelGGL(mt_xy_index_kernel, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, st, w.diag0, w.diag1, k,
                       n, diag, ii, jj);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_maxconv(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                          const MaxconvSpec& spec, void* z, uint8_t* pstar, const MaxconvWorkspace& w,
                          hipStream_t st) {
    if (b <= 0 || n <= 0 || m <= 0) return hipSuccess;
    const int logN = maxconv_log_size(n, m);
    if (logN > kLongConvLog) return hipErrorInvalidValue;
    if (logN > kMaxConvLog) {
        if (f64)
            return launch_maxconv_long<double>((const double*)x, (const double*)y, b, n, m, spec, (double*)z, pstar,
                                               w, st);
        return launch_maxconv_long<float>((const float*)x, (const float*)y, b, n, m, spec, (float*)z, pstar, w, st);
    }
    if (f64)
        return launch_maxconv_t<double>((const double*)x, (const double*)y, b, n, m, spec, (double*)z, pstar, st);
    return launch_maxconv_t<float>((const float*)x, (const float*)y, b, n, m, spec, (float*)z, pstar, st);
}

hipError_t launch_xy_topk(const void* x, const void* y, int f64, int64_t n, int32_t k, const MaxconvSpec& spec,
                          bool paired, double* values, int32_t* diag, int32_t* ii, int32_t* jj,
                          const XyWorkspace& w, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (maxconv_log_size(n, n) > kLongConvLog) return hipErrorInvalidValue;
    if (f64)
        return launch_xy_t<double>((const double*)x, (const double*)y, n, k, spec, paired, values, diag, ii, jj, w,
                                   st);
    return launch_xy_t<float>((const float*)x, (const float*)y, n, k, spec, paired, values, diag, ii, jj, w, st);
}

hipError_t launch_maxconv_exact(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                                void* z, hipStream_t st) {
    const int64_t total = b * (n + m - 1);
    if (b <= 0 || n <= 0 || m <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((total + 255) / 256);
    timing_before("mt_exact_maxconv", st);
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
