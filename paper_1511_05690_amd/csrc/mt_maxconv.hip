// Max-convolution (Sec. 1).
//
// Estimate: z[t] = max_i x[i] y[t - i] from the norm sequence
// S_p[t] = (x'^p * y'^p)[t] with x' = x / max x, y' = y / max y (terms in
// [0, 1], the scaling of Sec. 2.1), computed by FFT convolution in FP64 (the
// fast ring kernel H, Sec. 2.1, whose threshold there is tau = 1e-12); per
// index the largest p of the family with S_p >= tau, and
// z = max x max y S_{p*}^(1/p*).
//
// Layout: a transform of N = max(16, 2^ceil(log2(n + m - 1))) points is
// done by N / 16 threads that hold 16 complex values each in registers
// (N <= 4096: 256 threads, one pair per workgroup; smaller N packs 4096 / N
// pairs into a workgroup).  Passes are Stockham radix-16 (the last one radix
// 2, 4 or 8 when log2 N is not a multiple of 4), natural order in and out,
// through one LDS buffer per pair padded by one element every 16 (the
// stride-16 writes of the first pass then hit distinct banks).  Twiddles
// exp(-2 pi i m / N) come from one LDS table of cos and sin of 2 pi k / N for
// k <= N / 8 (the other octants by symmetry); a butterfly looks up w and w^4
// and forms the other powers by products.
// Per p, largest first:
//   forward: x'^p + i y'^p (x, y re-read per p, times 1 / max), so both real
//            transforms come out of one complex FFT;
//   product: thread t reads Z_t and Z_{N-t} and forms conj(W_t),
//            W = X Y with X_t = (Z_t + conj Z_{N-t}) / 2, Y_t = (Z_t - conj
//            Z_{N-t}) / 2i (the first pass of the inverse reads these pairs);
//   inverse: the forward FFT of conj(W), whose real part / N is S_p; the
//            last pass leaves S in registers at the positions the thread
//            owns, where the p* test and the root run without another LDS
//            trip.
// Indices decided at a larger p keep their value; a workgroup stops once
// every index of its pairs is decided.
//
// Exact: z[t] = max_i x[i] y[t - i] by the definition, one thread per output
// index, products in the input precision.

#include <atomic>

#include "mt_internal.h"

namespace mt {
namespace {

constexpr int kConvThreads = 256;  // kMaxConvN / 16
static_assert(kConvThreads * 16 == kMaxConvN, "16 values per thread at the largest N");
constexpr int kConvMinLog = 4;
// per log2 N: transform the powers in pairs (one inverse for two p)
constexpr bool kPairInverse[kMaxConvLog + 1] = {false, false, false, false, false, false, false,
                                                false, false, false, false, false, false};
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

template <typename T, int LOGN, bool PAIR>
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
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int slot = tid / TP, tl0 = tid % TP;
    const int tl = tl0;
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
        const int t = tl + i * TP;
        if (active && t < n) mx = fmax(mx, (double)xi[t]);
        if (active && t < m) my = fmax(my, (double)yi[t]);
    }
    for (int k = tid; k <= N / 8; k += kConvThreads) {
        double sn, cs;
        sincospi(2.0 * (double)k / (double)N, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
    // maxima over the pair's threads (contiguous lanes; several waves when TP > 64)
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
    __syncthreads();
    PassTwiddles<LOGN> pt;
    load_twiddles<LOGN, 1>(pt, tl, tw);
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
    int ffts = 0;

    // With PAIR, powers go in pairs (p_a, p_b) = (P[q], P[q - 1]): two forward
    // transforms and one inverse of V = W_a + i W_b, whose real and imaginary
    // parts are S_a and S_b (both ring results are real).
    for (int q = spec.n - 1; q >= 0; q -= PAIR ? 2 : 1) {
        const bool two = PAIR && q > 0;
        ffts += two ? 3 : 2;
        // re-derive the addresses per step instead of holding them across the loop
        int tl = tl0;
        asm volatile("" : "+v"(tl));
        const int bp = padi(tl), bn = padi(N - tl);
        // forward transform of x'^p + i y'^p into the LDS buffer (natural order)
        auto forward = [&](int p, double2 (&w)[16]) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
                const int t = tl + i * TP;
                const double a = (active && t < n) ? (double)xi[t] * ix : 0.0;
                const double c = (active && t < m) ? (double)yi[t] * iy : 0.0;
                w[i] = make_double2(ipow_d(a, p), ipow_d(c, p));
            }
            pass_compute<LOGN, 0>(w, pt);
            pass_store<LOGN, 0>(w, tl, buf);
            __syncthreads();
            middle_passes<LOGN, 1, F::NPASS>(w, tl, buf, pt);
        };
        // 4 W_t = (Z_t + conj Z_-t)(Z_t - conj Z_-t) / i at the thread's position i
        auto product = [&](int i) {
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
            return cmul(a, c);
        };
        double2 v[16];
        forward(spec.p[q], v);
        // the inverse is the forward transform of conj(V) = conj(W_a) - i conj(W_b)
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double2 w = product(i);
            v[i] = make_double2(w.x, -w.y);
        }
        if constexpr (PAIR) {
            if (two) {
                double2 u[16];
                __syncthreads();
                forward(spec.p[q - 1], u);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const double2 w = product(i);
                    v[i] = make_double2(v[i].x - w.y, v[i].y - w.x);
                }
            }
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
        // p* test: the first stable p from the top decides an index; the
        // smallest p decides what is left (its S, no p stable).  S_a = Re / N,
        // S_b = -Im / N (with the 1 / 4 of X Y).
        const bool lastp = two ? q == 1 : q == 0;
        int open = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int t = tl + i * TP;
            const double2 r = v[last_reg<LOGN>(i)];
            const double sa = r.x * scale, sb = -r.y * scale;
            const bool live = active && t < L && !(decided & (1u << i));
            const bool st_a = sa >= spec.tau, st_b = two && sb >= spec.tau;
            const bool dec = live && (st_a || st_b || lastp);
            open |= live && !dec;
            s_sel[i] = dec ? (st_a || !two ? sa : sb) : s_sel[i];
            const uint32_t code = st_a ? (uint32_t)q : st_b ? (uint32_t)(q - 1) : (uint32_t)MT_PSTAR_NONE;
            q_sel[i / 4] = dec ? (q_sel[i / 4] & ~(0xffu << (8 * (i % 4)))) | (code << (8 * (i % 4))) : q_sel[i / 4];
            decided |= dec ? 1u << i : 0u;
        }
        if (!__syncthreads_or(open)) break;
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
    if (work && tid == 0) {
        // 5 N log2 N flops per complex transform (the usual FFT count)
        const int64_t pairs = b - (int64_t)blockIdx.x * F::G < F::G ? b - (int64_t)blockIdx.x * F::G : F::G;
        atomicAdd(work, (unsigned long long)ffts * (unsigned long long)pairs * (5ull * N * LOGN));
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
    int logN = kConvMinLog;
    while ((int64_t(1) << logN) < L) ++logN;
    return logN;
}

namespace {

template <typename T, int LOGN>
hipError_t launch_maxconv_n(const T* x, const T* y, int64_t b, int64_t n, int64_t m, const MaxconvSpec& spec,
                            T* z, uint8_t* pstar, hipStream_t st) {
    auto kern = mt_maxconv_kernel<T, LOGN, kPairInverse[LOGN]>;
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

hipError_t launch_maxconv(const void* x, const void* y, int f64, int64_t b, int64_t n, int64_t m,
                          const MaxconvSpec& spec, void* z, uint8_t* pstar, hipStream_t st) {
    if (b <= 0 || n <= 0 || m <= 0) return hipSuccess;
    if (maxconv_log_size(n, m) > kMaxConvLog) return hipErrorInvalidValue;
    if (f64)
        return launch_maxconv_t<double>((const double*)x, (const double*)y, b, n, m, spec, (double*)z, pstar, st);
    return launch_maxconv_t<float>((const float*)x, (const float*)y, b, n, m, spec, (float*)z, pstar, st);
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
