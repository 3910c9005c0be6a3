// HBM-bound kernels of the p-norm (max, x) path on gfx950:
//   * row / column maxima of the inputs with the domain check (the scaled
//     ring call H' of Sec. 2.1: inputs divided by their maximum);
//   * power planes: (A/r)^p and (B/c)^p for every p of the family, written
//     once in the layout the MFMA GEMM reads (K contiguous, zero padded),
//     as BF16 hi/lo pairs or FP64 (the powered inputs of Alg. 5);
//   * the (+, min) <-> (x, max) transforms of Sec. 2.2.
#include <cfloat>
#include <cmath>

#include "mt_internal.h"

namespace mt {

namespace {

constexpr int kThreads = 256;

// Two values to BF16 by the hardware conversion, round to nearest even (the
// same bits as rounding the FP32 bit pattern to nearest even: checked for
// every finite nonnegative FP32 value), a in the low half.
typedef float mt_f32x2 __attribute__((ext_vector_type(2)));
typedef __bf16 mt_bf16x2 __attribute__((ext_vector_type(2)));
__device__ inline uint32_t bf16x2_rne(float a, float b) {
    const mt_f32x2 v = {a, b};
    return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, mt_bf16x2));
}

template <typename T>
__device__ inline bool bad_value(T x) {
    // negative, NaN or +inf
    return !(x >= T(0)) || !(x <= (T)(sizeof(T) == 8 ? DBL_MAX : FLT_MAX));
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t value, int64_t words) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < words; i += stride) p[i] = value;
}

// ---------------------------------------------------------------- tail sort
// Counting sort of the sparse-tail list by row bucket and state: counts, an exclusive
// scan of the counts (one block), then each entry to its bucket's next slot.
// The order inside a bucket is whatever the atomics give; each entry's
// result does not depend on it.
// Bucket of an entry: its row bucket, and within it the open entries after
// the others (entries of one row with one state are then adjacent).
__device__ __forceinline__ int64_t tail_key(const TailEntry& te, int64_t rows, int shift) {
    return ((((int64_t)te.bi * rows + te.i) >> shift) << 1) | (te.state == kTailOpen ? 1 : 0);
}

__global__ void tail_hist_kernel(const TailEntry* __restrict__ in, const uint32_t* __restrict__ count,
                                 int64_t rows, int shift, int32_t* __restrict__ bucket) {
    const int64_t nent = *count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nent; i += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&bucket[tail_key(in[i], rows, shift)], 1);
}

// Exclusive prefix sum of bucket[0 .. nb) in place, one block of
// kScanThreads: thread t scans a contiguous run of the buckets (a multiple of
// 4 long, read and written as int4; the bucket array is 16-byte aligned and
// padded to a multiple of 4 entries).
constexpr int kScanThreads = 1024;
__global__ __launch_bounds__(kScanThreads) void tail_scan_kernel(int32_t* __restrict__ bucket, int32_t nb) {
    __shared__ int32_t part[kScanThreads];
    const int t = threadIdx.x;
    const int nb4 = (nb + 3) / 4;
    const int per4 = (nb4 + kScanThreads - 1) / kScanThreads;
    const int lo = min(t * per4, nb4), hi = min(lo + per4, nb4);
    int4* b4 = (int4*)bucket;
    int32_t sum = 0;
    for (int i = lo; i < hi; ++i) {
        const int4 v = b4[i];
        sum += v.x + v.y + v.z + v.w;
    }
    part[t] = sum;
    __syncthreads();
    for (int d = 1; d < kScanThreads; d <<= 1) {
        const int32_t y = t >= d ? part[t - d] : 0;
        __syncthreads();
        part[t] += y;
        __syncthreads();
    }
    int32_t run = part[t] - sum;
    for (int i = lo; i < hi; ++i) {
        const int4 v = b4[i];
        int4 o;
        o.x = run;
        o.y = run + v.x;
        o.z = o.y + v.y;
        o.w = o.z + v.z;
        run = o.w + v.w;
        b4[i] = o;
    }
}

__global__ void tail_scatter_kernel(const TailEntry* __restrict__ in, const uint32_t* __restrict__ count,
                                    int64_t rows, int shift, int32_t* __restrict__ bucket,
                                    TailEntry* __restrict__ out) {
    const int64_t nent = *count;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nent; i += (int64_t)gridDim.x * blockDim.x) {
        const TailEntry te = in[i];
        out[atomicAdd(&bucket[tail_key(te, rows, shift)], 1)] = te;
    }
}

// One wave per row: r[row] = max_k A[row, k] (times mul[batch, k] when
// kMul: the balanced row maximum, rpb rows per batch item); flags invalid
// entries.
template <typename T, bool kMul = false>
__global__ __launch_bounds__(kThreads) void mt_rowmax_kernel(const T* __restrict__ A, int64_t rows,
                                                             int64_t k, double* __restrict__ r,
                                                             int32_t* __restrict__ flag,
                                                             const double* __restrict__ mul = nullptr,
                                                             int64_t rpb = 1) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (row >= rows) return;
    const T* a = A + row * k;
    const double* mu = kMul ? mul + (row / rpb) * k : nullptr;
    auto val = [&](T v, int64_t j) { return kMul ? (double)v * mu[j] : (double)v; };
    double mx = 0.0;
    bool bad = false;
    int64_t j = lane;
    constexpr int V = 16 / sizeof(T);
    if (k % V == 0) {
        // 16-byte loads: lane l reads elements V*l .. V*l+V-1 of each chunk
        typedef T vecT __attribute__((ext_vector_type(V)));
        for (int64_t j0 = (int64_t)lane * V; j0 < k; j0 += 64 * V) {
            const vecT v = *(const vecT*)(a + j0);
#pragma unroll
            for (int q = 0; q < V; ++q) {
                bad |= bad_value(v[q]);
                mx = fmax(mx, val(v[q], j0 + q));
            }
        }
        j = k;
    }
    for (; j + 192 < k; j += 256) {
        T v0 = a[j], v1 = a[j + 64], v2 = a[j + 128], v3 = a[j + 192];
        bad |= bad_value(v0) | bad_value(v1) | bad_value(v2) | bad_value(v3);
        mx = fmax(mx, fmax(fmax(val(v0, j), val(v1, j + 64)), fmax(val(v2, j + 128), val(v3, j + 192))));
    }
    for (; j < k; j += 64) {
        T v = a[j];
        bad |= bad_value(v);
        mx = fmax(mx, val(v, j));
    }
    mx = wave_max(mx);
    if (lane == 0) r[row] = mx;
    if (bad) atomicOr(flag, 1);
}

// c[b, j] = max_k B[b, k, j] (times mul[b, k] when kMul: the balanced column
// maximum): each thread owns kColVec consecutive columns (one 16-byte load
// per row when n allows it), 64 rows per block, combined with an integer
// atomic max on the bit pattern (exact for >= 0).
template <typename T, bool kMul>
__device__ __forceinline__ void colmax_block(const T* __restrict__ B, int64_t k, int64_t n, double* __restrict__ c,
                                             int32_t* __restrict__ flag, const double* __restrict__ mul,
                                             int64_t bx, int64_t by, int64_t bz) {
    constexpr int V = 16 / sizeof(T);
    const int64_t j0 = (bx * kThreads + threadIdx.x) * V;
    const int64_t k0 = by * 64;
    const int64_t bi = bz;
    if (j0 >= n) return;
    const T* bb = B + bi * k * n + j0;
    double mx[V];
#pragma unroll
    for (int q = 0; q < V; ++q) mx[q] = 0.0;
    bool bad = false;
    const int64_t k1 = k0 + 64 < k ? k0 + 64 : k;
    if (j0 + V <= n && (n % V) == 0) {
        typedef T vecT __attribute__((ext_vector_type(V)));
#pragma unroll 8
        for (int64_t kk = k0; kk < k1; ++kk) {
            const vecT v = *(const vecT*)(bb + kk * n);
            const double f = kMul ? mul[bi * k + kk] : 1.0;
#pragma unroll
            for (int q = 0; q < V; ++q) {
                bad |= bad_value(v[q]);
                mx[q] = fmax(mx[q], kMul ? (double)v[q] * f : (double)v[q]);
            }
        }
    } else {
        for (int64_t kk = k0; kk < k1; ++kk) {
            const double f = kMul ? mul[bi * k + kk] : 1.0;
#pragma unroll
            for (int q = 0; q < V; ++q)
                if (j0 + q < n) {
                    const T v = bb[kk * n + q];
                    bad |= bad_value(v);
                    mx[q] = fmax(mx[q], kMul ? (double)v * f : (double)v);
                }
        }
    }
    if (bad) atomicOr(flag, 1);
#pragma unroll
    for (int q = 0; q < V; ++q)
        if (j0 + q < n && (mx[q] > 0.0 || mx[q] != mx[q]))
            atomicMax((unsigned long long*)(c + bi * n + j0 + q), (unsigned long long)__double_as_longlong(mx[q]));
}

template <typename T, bool kMul = false>
__global__ __launch_bounds__(kThreads) void mt_colmax_kernel(const T* __restrict__ B, int64_t k,
                                                             int64_t n, double* __restrict__ c,
                                                             int32_t* __restrict__ flag,
                                                             const double* __restrict__ mul = nullptr) {
    colmax_block<T, kMul>(B, k, n, c, flag, mul, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Inner-index balancing: d = sqrt(b / a) per inner index (a = largest entry
// of the column of A, b = of the row of B), 1 where either is 0; dinv = 1 / d.
__global__ void mt_balance_kernel(const double* __restrict__ a, const double* __restrict__ b, int64_t count,
                                  double* __restrict__ d, double* __restrict__ dinv) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double av = a[i], bv = b[i];
        const double f = (av > 0.0 && bv > 0.0) ? sqrt(bv / av) : 1.0;
        d[i] = f;
        dinv[i] = 1.0 / f;
    }
}

template <typename T>
__device__ inline T ipow(T x, int p) {
    T r = T(1);
    while (p) {
        if (p & 1) r *= x;
        x *= x;
        p >>= 1;
    }
    return r;
}

// Power planes.  Tile: 64 plane rows x 64 plane columns per block.
//   transpose == 0: plane row t = src row t (src is rows x cols)
//   transpose == 1: plane row t = src column t (src is cols x rows)
// Plane element (t, u) is src / (scale_rows[t] * scale_cols[u]) (each scale
// optional; a zero scale gives 0), the scaled input of Sec. 2.1's H'.
// Every thread produces 8 consecutive plane columns (one 16-byte BF16 chunk)
// of two plane rows.
// Powers of one 8-element chunk of scaled values x (plane row position
// `pos` = t * cols_pad + u) to every plane of the family: squaring where p
// doubles the previous power, binary powering otherwise; BF16 planes take
// hi = RNE(power) and, for a split p, lo = RNE(power - hi) in the next plane.
template <typename TC, bool kBf16>
__device__ __forceinline__ void write_power_chunk(const TC (&x)[8], const PlaneSpec& spec, void* __restrict__ planes,
                                                  int64_t bi, int64_t plane_elems, int64_t pos) {
    TC pw[8];
    int prev = 0;
    for (int q = 0; q < spec.n_p; ++q) {
        const int p = spec.p[q];
        if (prev > 0 && p == 2 * prev) {
#pragma unroll
            for (int i = 0; i < 8; ++i) pw[i] = pw[i] * pw[i];
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) pw[i] = ipow(x[i], p);
        }
        prev = p;
        // powers whose planes are not wanted are still formed: the next
        // power may square them
        if (!((spec.write_mask >> q) & 1u)) continue;
        const int64_t pl = spec.first_plane[q];
        const int64_t off = (bi * spec.n_planes + pl) * plane_elems + pos;
        if (kBf16) {
            uint16_t* base = (uint16_t*)planes;
            u32x4 hi, lo;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float f0 = (float)pw[2 * i], f1 = (float)pw[2 * i + 1];
                const uint32_t h = bf16x2_rne(f0, f1);
                hi[i] = h;
                if (spec.split[q])
                    lo[i] = bf16x2_rne(f0 - __uint_as_float(h << 16), f1 - __uint_as_float(h & 0xFFFF0000u));
            }
            // streaming stores: the planes are read back only by the GEMM,
            // long after (measured: the GEMM 1.5 % faster, the planes even)
            __builtin_nontemporal_store(hi, (u32x4*)(base + off));
            if (spec.split[q]) __builtin_nontemporal_store(lo, (u32x4*)(base + off + plane_elems));
        } else {
            double* base = (double*)planes;
#pragma unroll
            for (int i = 0; i < 8; i += 2) {
                double2 v2;
                v2.x = (double)pw[i];
                v2.y = (double)pw[i + 1];
                *(double2*)(base + off + i) = v2;
            }
        }
    }
}

// A workgroup covers PlaneTile::T plane rows x PlaneTile::U plane columns:
// through an LDS transpose (FP32 sources kTrRows x kTrCols, FP64 64 x 64),
// or 16 rows x 256 columns straight from the rows (512 contiguous bytes per
// row and BF16 plane written).
constexpr int kTrRows = 64, kTrCols = 64;
template <typename TS, bool kTranspose>
struct PlaneTile {
    static constexpr int T = kTranspose ? (sizeof(TS) == 4 ? kTrRows : 64) : 16;
    static constexpr int U = kTranspose ? (sizeof(TS) == 4 ? kTrCols : 64) : 256;
    static constexpr int CHUNKS = U / 8;  // 8-column chunks per plane row
    static constexpr int TASKS = T * CHUNKS;
    static_assert(TASKS % kThreads == 0, "whole tasks per thread");
};

// The workgroup of plane tile (bx, by) of batch item bz.
template <typename TS, bool kBf16, bool kTranspose>
__device__ __forceinline__ void power_planes_block(const TS* __restrict__ src, int64_t rows, int64_t cols,
                                                   int64_t rows_pad, int64_t cols_pad,
                                                   const double* __restrict__ scale_rows,
                                                   const double* __restrict__ scale_cols,
                                                   const double* __restrict__ col_mul, const PlaneSpec& spec,
                                                   void* __restrict__ planes, int64_t bx, int64_t by, int64_t bz) {
    using PT = PlaneTile<TS, kTranspose>;
    __shared__ TS tile[kTranspose ? PT::T : 1][kTranspose ? PT::U + 1 : 1];
    const int64_t bi = bz;
    const int64_t t0 = by * PT::T;  // plane row
    const int64_t u0 = bx * PT::U;  // plane column
    const TS* s = src + bi * rows * cols;

    if (kTranspose) {
        // src[u][t]: read U (u) x T (t) coalesced along t.
        for (int e = threadIdx.x; e < PT::T * PT::U; e += kThreads) {
            const int uu = e / PT::T, tt = e % PT::T;
            const int64_t u = u0 + uu, t = t0 + tt;
            tile[tt][uu] = (u < cols && t < rows) ? s[u * rows + t] : TS(0);
        }
        __syncthreads();
    }

    typedef typename std::conditional<kBf16, float, double>::type TC;
    const int64_t plane_elems = rows_pad * cols_pad;
    for (int rep = 0; rep < PT::TASKS / kThreads; ++rep) {
        const int task = threadIdx.x + rep * kThreads;
        const int tt = task / PT::CHUNKS, ch = task % PT::CHUNKS;
        const int64_t t = t0 + tt;
        const int64_t u = u0 + ch * 8;
        if (t >= rows_pad || u >= cols_pad) continue;
        TC x[8];
        double sc = 1.0;
        if (scale_rows != nullptr && t < rows) sc = scale_rows[bi * rows + t];
        const bool zero_row = (t >= rows) || (sc == 0.0);
        if (scale_cols == nullptr && !zero_row && sc >= DBL_MIN && u + 8 <= cols &&
            (kTranspose || (cols & 3) == 0)) {
            // whole chunk inside the row and (untransposed) 16-byte aligned:
            // vector loads and one reciprocal per row instead of 8 divisions
            // (the scaled value may differ from src / scale by one FP64 ulp;
            // a subnormal scale, whose reciprocal overflows, divides below)
            TS v[8];
            if (kTranspose) {
#pragma unroll
                for (int i = 0; i < 8; ++i) v[i] = tile[tt][ch * 8 + i];
            } else {
                typedef TS vec4 __attribute__((ext_vector_type(4)));
                const vec4 a0 = *(const vec4*)(s + t * cols + u);
                const vec4 a1 = *(const vec4*)(s + t * cols + u + 4);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    v[i] = a0[i];
                    v[4 + i] = a1[i];
                }
            }
            const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
            if (col_mul != nullptr) {
                // balanced input: (src d_u) / scale_rows, the product first
                // (it is at most the row's balanced maximum)
                const double* cm = col_mul + bi * cols + u;
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = (TC)(((double)v[i] * cm[i]) * inv);
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i) x[i] = (TC)((double)v[i] * inv);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                double v = 0.0;
                if (!zero_row && u + i < cols) {
                    v = kTranspose ? (double)tile[tt][ch * 8 + i] : (double)s[t * cols + u + i];
                    if (col_mul != nullptr) v *= col_mul[bi * cols + u + i];
                    double d = sc;
                    if (scale_cols != nullptr) d *= scale_cols[bi * cols + u + i];
                    v = d > 0.0 ? v / d : 0.0;
                }
                x[i] = (TC)v;
            }
        }
        write_power_chunk<TC, kBf16>(x, spec, planes, bi, plane_elems, t * cols_pad + u);
    }
}

template <typename TS, bool kBf16, bool kTranspose>
__global__ __launch_bounds__(kThreads) void mt_power_planes_kernel(
    const TS* __restrict__ src, int64_t rows, int64_t cols, int64_t rows_pad, int64_t cols_pad,
    const double* __restrict__ scale_rows, const double* __restrict__ scale_cols,
    const double* __restrict__ col_mul, PlaneSpec spec, void* __restrict__ planes) {
    power_planes_block<TS, kBf16, kTranspose>(src, rows, cols, rows_pad, cols_pad, scale_rows, scale_cols,
                                              col_mul, spec, planes, blockIdx.x, blockIdx.y, blockIdx.z);
}

// Both operands' planes of spec.write_mask (BF16 or FP64), only when *cond is
// set: A's untransposed plane tiles first, then B's transposed ones, a fixed
// grid striding over them.
struct PlanesIfOperand {
    const void* src;
    int64_t rows, cols, rows_pad, cols_pad;
    const double* scale_rows;
    const double* col_mul;
    void* planes;
    int64_t gx, gy, blocks;  // plane tiles along columns, along rows, in all
};
// With marks (b x tiles_m x tiles_n output tiles of side tile_bm, nonzero:
// the tile runs again), only the plane rows of marked tiles are written: A's
// rows of a tile row with a marked tile, B's of a tile column with one.
struct PlanesIfMarks {
    const uint32_t* marks;  // null: every plane row
    int64_t tiles_m, tiles_n, tile_bm;
};
template <typename TS, bool kBf16>
__global__ __launch_bounds__(kThreads) void mt_planes_if_kernel(const int32_t* __restrict__ cond, PlanesIfOperand a,
                                                                PlanesIfOperand b, PlaneSpec spec, PlanesIfMarks mk) {
    if (*cond == 0) return;
    for (int64_t v = blockIdx.x; v < a.blocks + b.blocks; v += gridDim.x) {
        const bool is_a = v < a.blocks;
        const int64_t w = is_a ? v : v - a.blocks;
        const PlanesIfOperand& o = is_a ? a : b;
        const int64_t bx = w % o.gx, by = (w / o.gx) % o.gy, bz = w / (o.gx * o.gy);
        if (mk.marks != nullptr) {
            // plane rows by * T.. of this block lie in one tile row (A) or
            // tile column (B): any marked tile along it?
            const int64_t tr = by * (is_a ? PlaneTile<TS, false>::T : PlaneTile<TS, true>::T) / mk.tile_bm;
            const int64_t len = is_a ? mk.tiles_n : mk.tiles_m;
            int hit = 0;
            for (int64_t i = threadIdx.x; i < len; i += kThreads) {
                const int64_t tm = is_a ? tr : i, tn = is_a ? i : tr;
                hit |= mk.marks[(bz * mk.tiles_m + tm) * mk.tiles_n + tn] != 0u;
            }
            if (!__syncthreads_or(hit)) continue;
        }
        if (is_a) {
            power_planes_block<TS, kBf16, false>((const TS*)a.src, a.rows, a.cols, a.rows_pad, a.cols_pad,
                                                 a.scale_rows, nullptr, a.col_mul, spec, a.planes, bx, by, bz);
        } else {
            power_planes_block<TS, kBf16, true>((const TS*)b.src, b.rows, b.cols, b.rows_pad, b.cols_pad,
                                                b.scale_rows, nullptr, b.col_mul, spec, b.planes, bx, by, bz);
        }
        // the transposed tile in LDS is refilled by the next iteration
        __syncthreads();
    }
}

// Row maxima and power planes of a row-major FP32 operand in one pass, for
// rows of at most kFusedRowMaxK padded inner elements: one workgroup per
// plane row holds the row in registers (kFusedChunks chunks of 8 per thread),
// takes r = max_k A_ik (Sec. 2.1 scaling; the domain check of the row-max
// kernel included), then writes the planes of A / r with the plane kernel's
// arithmetic (the FP64 reciprocal of r for whole 8-element chunks of rows
// whose length allows 16-byte loads, a division otherwise).  Padding rows
// and columns get zeros; r is written for the real rows.
constexpr int kFusedChunks = (int)(kFusedRowMaxK / 8 / kThreads);
template <bool kBf16>
__device__ __forceinline__ void rowmax_planes_block(const float* __restrict__ A, int64_t rows, int64_t cols,
                                                    int64_t rows_pad, int64_t cols_pad, double* __restrict__ r,
                                                    int32_t* __restrict__ flag, const PlaneSpec& spec,
                                                    void* __restrict__ planes, int64_t t, int64_t bi,
                                                    float* wmax) {
    const bool real_row = t < rows;
    const float* s = A + (bi * rows + (real_row ? t : 0)) * cols;
    const bool vec_row = (cols & 3) == 0 && ((uintptr_t)s % 16) == 0;
    float v[kFusedChunks][8];
    float mx = 0.f;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < kFusedChunks; ++c) {
        const int64_t u = ((int64_t)c * kThreads + threadIdx.x) * 8;
        if (real_row && vec_row && u + 8 <= cols) {
            typedef float vec4 __attribute__((ext_vector_type(4)));
            const vec4 a0 = *(const vec4*)(s + u);
            const vec4 a1 = *(const vec4*)(s + u + 4);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[c][i] = a0[i];
                v[c][4 + i] = a1[i];
            }
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[c][i] = (real_row && u + i < cols) ? s[u + i] : 0.f;
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            bad |= bad_value(v[c][i]);
            mx = fmaxf(mx, v[c][i]);
        }
    }
    // the row's maximum (exact in FP32) over the workgroup
    for (int d = 32; d >= 1; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    mx = wmax[0];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) mx = fmaxf(mx, wmax[w]);
    const double sc = (double)mx;
    if (real_row && threadIdx.x == 0) r[bi * rows + t] = sc;
    if (bad) atomicOr(flag, 1);

    typedef typename std::conditional<kBf16, float, double>::type TC;
    const int64_t plane_elems = rows_pad * cols_pad;
    const bool zero_row = !real_row || sc == 0.0;
    const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
#pragma unroll
    for (int c = 0; c < kFusedChunks; ++c) {
        const int64_t u = ((int64_t)c * kThreads + threadIdx.x) * 8;
        if (u >= cols_pad) continue;
        TC x[8];
        if (!zero_row && sc >= DBL_MIN && u + 8 <= cols && (cols & 3) == 0) {
#pragma unroll
            for (int i = 0; i < 8; ++i) x[i] = (TC)((double)v[c][i] * inv);
        } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                double y = 0.0;
                if (!zero_row && u + i < cols) y = sc > 0.0 ? (double)v[c][i] / sc : 0.0;
                x[i] = (TC)y;
            }
        }
        write_power_chunk<TC, kBf16>(x, spec, planes, bi, plane_elems, t * cols_pad + u);
    }
}

// The row-max and plane pass of A with B's column maxima in the same
// launch: the column-max blocks are interleaved with the plane-row blocks
// (one every ratio + 1 while both last), so the two HBM-bound passes share
// the GPU instead of running one after the other.  c must be zero before
// the launch.
template <bool kBf16>
__global__ __launch_bounds__(kThreads) void mt_rowmax_planes_colmax_kernel(
    const float* __restrict__ A, int64_t rows, int64_t cols, int64_t rows_pad, int64_t cols_pad,
    double* __restrict__ r, int32_t* __restrict__ flag, PlaneSpec spec, void* __restrict__ planes,
    const float* __restrict__ B, int64_t kb, int64_t nb, double* __restrict__ c, int64_t na, int64_t nc,
    int64_t ratio, int64_t cgx, int64_t cgy) {
    __shared__ float wmax[kThreads / 64];
    const int64_t id = blockIdx.x;
    const int64_t span = nc * (ratio + 1);
    int64_t a_idx, c_idx = -1;
    if (id < span) {
        const int64_t g = id / (ratio + 1), pos = id - g * (ratio + 1);
        if (pos == ratio) c_idx = g;
        a_idx = g * ratio + pos;
    } else {
        a_idx = nc * ratio + (id - span);
    }
    if (c_idx >= 0) {
        colmax_block<float, false>(B, kb, nb, c, flag, nullptr, c_idx % cgx, (c_idx / cgx) % cgy, c_idx / (cgx * cgy));
        return;
    }
    if (a_idx < na)
        rowmax_planes_block<kBf16>(A, rows, cols, rows_pad, cols_pad, r, flag, spec, planes, a_idx % rows_pad,
                                   a_idx / rows_pad, wmax);
}

// X = exp(-s W) in FP64; +inf -> 0; diagonal -> 1.
template <typename TX>
__global__ __launch_bounds__(kThreads) void mt_apsp_transform_kernel(const float* __restrict__ W,
                                                                     int64_t n, double s,
                                                                     TX* __restrict__ X,
                                                                     int32_t* __restrict__ flag) {
    const int64_t total = n * n;
    bool bad = false;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const int64_t i = e / n, j = e - (e / n) * n;
        const float w = W[e];
        double x;
        if (i == j) {
            x = 1.0;
        } else {
            if (!(w >= 0.0f)) bad = true;  // negative or NaN
            x = exp(-s * (double)w);      // +inf -> 0
        }
        X[e] = (TX)x;
    }
    if (bad) atomicOr(flag, 1);
}

// D = -log(X) / s in FP64; X = 0 -> +inf.
// raw != 0: D = X (the (x, max) matrix itself, converted to D's type).
template <typename TX, typename TD>
__global__ __launch_bounds__(kThreads) void mt_apsp_to_dist_kernel(const TX* __restrict__ X,
                                                                   int64_t total, double s_inv,
                                                                   int raw, TD* __restrict__ D) {
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * kThreads) {
        const double x = (double)X[e];
        D[e] = raw ? (TD)x : (TD)(x > 0.0 ? -log(x) * s_inv + 0.0 : HUGE_VAL);
    }
}

// FP64 path, after the GEMM's selection: C = r_i c_j S^(1/p*) (the 1/p root of
// Sec. 1 with the restored row / column scale), optional clamp, APSP diagonal.
// With the r = 1 projection (Sec. 1: the terms modelled as copies of one
// value) the max is (S_{p*} / S_{p_lo})^(1/(p* - p_lo)), p_lo the family's
// next smaller p, whose ring result S2 the GEMM recorded; the plain root is
// kept where p* is the smallest p, none was stable, or S2 is 0.
template <typename TO>
__global__ __launch_bounds__(kThreads) void mt_select_root_f64_kernel(
    const double* __restrict__ S, const double* __restrict__ S2, const uint8_t* __restrict__ code,
    int64_t rows, int64_t m, int64_t n, const double* __restrict__ r, const double* __restrict__ c,
    RootSpec spec, TO* __restrict__ out, uint8_t* __restrict__ pstar_out) {
    for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t bi = row / m;
        const int64_t i = row - bi * m;
        const double ri = r ? r[row] : 1.0;
        for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n;
             j += (int64_t)gridDim.x * kThreads) {
            const int64_t e = row * n + j;
            const uint8_t q = code[e];
            const int qi = q == MT_PSTAR_NONE ? 0 : q;
            const int p = spec.p[qi];
            const double s = S[e];
            double root = p == 1 ? s : (s > 0.0 ? exp(log(s) / (double)p) : 0.0);
            if (spec.r1 && q != MT_PSTAR_NONE && q > 0) {
                const double s2 = S2[e];
                if (s2 > 0.0) root = exp(log(s / s2) / (double)(p - spec.p[q - 1]));
            }
            double v = ri * (c ? c[bi * n + j] : 1.0) * root * spec.corr[qi];
            if (spec.mode == EPI_APSP_X || spec.clamp) v = fmin(v, 1.0);
            if (spec.mode == EPI_APSP_X && i == j) v = 1.0;
            out[e] = (TO)v;
            if (pstar_out) pstar_out[e] = q;
        }
    }
}

// Selection and r = 2 projection from the S stack (Sec. 1): p* is the
// largest family p with S >= tau; with p* = 4q and S_q, S_2q, S_3q, S_4q all
// positive, the null vector of [[t1, t2, t3], [t2, t3, t4]] (t_k = S_kq /
// c^k, c = (S_4q / S_q)^(1/3), which scales the roots by c) is the cross
// product of its rows, g = (t2 t4 - t3^2, t2 t3 - t1 t4, t1 t3 - t2^2), and
// the estimate is the largest root x of g0 + g1 x + g2 x^2 (x = alpha^q / c)
// as alpha = (c x)^(1/q).  Numerical rank 1, complex or nonpositive roots, or
// a missing norm: the r = 1 projection with the next smaller family p; no
// such p or S_lo = 0: the plain root.  Rank 1: rho = sigma_2 / sigma_1 of
// the 2 x 3 matrix (from |g| = sigma_1 sigma_2 and the squared Frobenius
// norm sigma_1^2 + sigma_2^2) at most theta = eps / (q delta): the norms'
// relative rounding eps = (K + 4 p* + max |ln S|) 2^-53 (K terms, p*-fold
// products, the logarithms) moves the projected value by about
// eps / (q rho), and the projection is used where that stays below
// delta = 2.5e-6 (a quarter of the path's 1e-5).
constexpr double kR2Delta = 2.5e-6;

template <typename TO>
__global__ __launch_bounds__(kThreads) void mt_select_r2_kernel(const double* __restrict__ stack, int64_t stride,
                                                                int64_t rows, int64_t m, int64_t n,
                                                                const double* __restrict__ r,
                                                                const double* __restrict__ c, R2Spec spec,
                                                                TO* __restrict__ out, uint8_t* __restrict__ pstar_out) {
    for (int64_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const int64_t bi = row / m;
        const int64_t i = row - bi * m;
        const double ri = r ? r[row] : 1.0;
        for (int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x; j < n; j += (int64_t)gridDim.x * kThreads) {
            const int64_t e = row * n + j;
            int q = -1;
            for (int fi = spec.n - 1; fi >= 0; --fi)
                if (stack[(int64_t)spec.plane[fi] * stride + e] >= spec.tau) {
                    q = fi;
                    break;
                }
            const int qi = q < 0 ? 0 : q;
            const int p = spec.p[qi];
            const double s = stack[(int64_t)spec.plane[qi] * stride + e];
            double alpha = p == 1 ? s : (s > 0.0 ? exp(log(s) / (double)p) : 0.0);
            if (q > 0 && spec.lo[q] >= 0) {
                const double sl = stack[(int64_t)spec.lo[q] * stride + e];
                if (sl > 0.0) alpha = exp(log(s / sl) / (double)(p - spec.p[q - 1]));
            }
            if (q >= 0 && spec.q4[q][0] >= 0) {
                double lS[4];
                bool ok = true;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double v = stack[(int64_t)spec.q4[q][k] * stride + e];
                    ok &= v > 0.0;
                    lS[k] = v > 0.0 ? log(v) : 0.0;
                }
                if (ok) {
                    const double logc = (lS[3] - lS[0]) / 3.0;
                    double t[4];
#pragma unroll
                    for (int k = 0; k < 4; ++k) t[k] = exp(lS[k] - (k + 1) * logc);
                    const double g0 = t[1] * t[3] - t[2] * t[2];
                    const double g1 = t[1] * t[2] - t[0] * t[3];
                    const double g2 = t[0] * t[2] - t[1] * t[1];
                    const double gn = sqrt(g0 * g0 + g1 * g1 + g2 * g2);
                    const double rn = t[0] * t[0] + 2 * t[1] * t[1] + 2 * t[2] * t[2] + t[3] * t[3];
                    // y = sigma_1 sigma_2 / (sigma_1^2 + sigma_2^2) = rho / (1 + rho^2)
                    const double y = fmin(gn / rn, 0.5);
                    const double rho = 2.0 * y / (1.0 + sqrt(fmax(1.0 - 4.0 * y * y, 0.0)));
                    double lmax = 0.0;
#pragma unroll
                    for (int k = 0; k < 4; ++k) lmax = fmax(lmax, fabs(lS[k]));
                    const double theta =
                        (spec.k_inner + 4.0 * p + lmax) * 0x1p-53 / ((double)(p / 4) * kR2Delta);
                    const double disc = g1 * g1 - 4.0 * g2 * g0;
                    if (rho > theta && g2 != 0.0 && disc >= 0.0) {
                        const double sq = sqrt(disc);
                        const double x1 = (-g1 + sq) / (2.0 * g2), x2 = (-g1 - sq) / (2.0 * g2);
                        const double xm = x1 > x2 ? x1 : x2;
                        if (xm > 0.0) alpha = exp((log(xm) + logc) / (double)(p / 4));
                    }
                }
            }
            double v = ri * (c ? c[bi * n + j] : 1.0) * alpha;
            if (spec.mode == EPI_APSP_X || spec.clamp) v = fmin(v, 1.0);
            if (spec.mode == EPI_APSP_X && i == j) v = 1.0;
            out[e] = (TO)v;
            if (pstar_out) pstar_out[e] = q < 0 ? (uint8_t)MT_PSTAR_NONE : (uint8_t)q;
        }
    }
}

inline unsigned grid_for(int64_t items, int64_t per_block, int64_t cap = 65535 * 8) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_fill_u32(void* p, uint32_t value, int64_t words, hipStream_t st) {
    if (words <= 0) return hipSuccess;
    timing_before("mt_fill", st);
    hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(words, kThreads * 4, 4096)), dim3(kThreads), 0, st,
                       (uint32_t*)p, value, words);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_fill_zero_u32(void* p, int64_t words, hipStream_t st) { return launch_fill_u32(p, 0u, words, st); }

hipError_t launch_tail_sort(const EpiArgs& epi, int64_t rows, int64_t cap, hipStream_t st) {
    if (cap <= 0) return hipSuccess;
    hipError_t e = launch_fill_zero_u32(epi.tail_bucket, (epi.tail_buckets + 3) / 4 * 4, st);
    if (e != hipSuccess) return e;
    const dim3 grid(grid_for(cap, kThreads, 1024));
    timing_before("mt_tail_sort", st);
    hipLaunchKernelGGL(tail_hist_kernel, grid, dim3(kThreads), 0, st, epi.tail, epi.tail_count, rows,
                       epi.tail_shift, epi.tail_bucket);
    hipLaunchKernelGGL(tail_scan_kernel, dim3(1), dim3(kScanThreads), 0, st, epi.tail_bucket, epi.tail_buckets);
    hipLaunchKernelGGL(tail_scatter_kernel, grid, dim3(kThreads), 0, st, epi.tail, epi.tail_count, rows,
                       epi.tail_shift, epi.tail_bucket, epi.tail_sorted);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_rowmax(const void* A, int f64, int64_t rows, int64_t k, double* r, int32_t* flag,
                         hipStream_t st, const double* mul, int64_t rows_per_batch) {
    if (rows <= 0) return hipSuccess;
    const dim3 grid((unsigned)((rows + 3) / 4));
    timing_before("mt_rowmax", st);
#define MT_ROWMAX(T, M)                                                                        \
    hipLaunchKernelGGL((mt_rowmax_kernel<T, M>), grid, dim3(kThreads), 0, st, (const T*)A, rows, k, r, flag, \
                       mul, rows_per_batch)
    if (f64) {
        if (mul) MT_ROWMAX(double, true); else MT_ROWMAX(double, false);
    } else {
        if (mul) MT_ROWMAX(float, true); else MT_ROWMAX(float, false);
    }
#undef MT_ROWMAX
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_colmax(const void* B, int f64, int64_t b, int64_t k, int64_t n, double* c,
                         int32_t* flag, hipStream_t st, const double* mul) {
    hipError_t e = launch_fill_zero_u32(c, b * n * 2, st);
    if (e != hipSuccess || k <= 0) return e;
    const int64_t per_block = (int64_t)kThreads * (f64 ? 2 : 4);  // columns per block
    const dim3 grid((unsigned)((n + per_block - 1) / per_block), (unsigned)((k + 63) / 64), (unsigned)b);
    timing_before("mt_colmax", st);
#define MT_COLMAX(T, M) \
    hipLaunchKernelGGL((mt_colmax_kernel<T, M>), grid, dim3(kThreads), 0, st, (const T*)B, k, n, c, flag, mul)
    if (f64) {
        if (mul) MT_COLMAX(double, true); else MT_COLMAX(double, false);
    } else {
        if (mul) MT_COLMAX(float, true); else MT_COLMAX(float, false);
    }
#undef MT_COLMAX
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_balance(const double* a, const double* b, int64_t count, double* d, double* dinv,
                          hipStream_t st) {
    if (count <= 0) return hipSuccess;
    timing_before("mt_balance", st);
    hipLaunchKernelGGL(mt_balance_kernel, dim3(grid_for(count, kThreads, 1024)), dim3(kThreads), 0, st, a, b,
                       count, d, dinv);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_power_planes(const void* src, int src_f64, int transpose, int64_t b, int64_t rows,
                               int64_t cols, int64_t rows_pad, int64_t cols_pad,
                               const double* scale_rows, const double* scale_cols,
                               const PlaneSpec& spec, int bf16, void* planes, hipStream_t st,
                               const double* col_mul) {
    if (rows_pad <= 0 || cols_pad <= 0) return hipSuccess;
#define MT_PLANES(TS, BF, TR)                                                                    \
    hipLaunchKernelGGL((mt_power_planes_kernel<TS, BF, TR>),                                    \
                       dim3((unsigned)((cols_pad + PlaneTile<TS, TR>::U - 1) / PlaneTile<TS, TR>::U), \
                            (unsigned)((rows_pad + PlaneTile<TS, TR>::T - 1) / PlaneTile<TS, TR>::T), \
                            (unsigned)b),                                                       \
                       dim3(kThreads), 0, st, (const TS*)src, rows, cols, rows_pad, cols_pad,   \
                       scale_rows, scale_cols, col_mul, spec, planes)
    timing_before(bf16 ? "mt_power_planes_bf16" : "mt_power_planes_f64", st);
    if (src_f64) {
        if (bf16) {
            if (transpose) MT_PLANES(double, true, true); else MT_PLANES(double, true, false);
        } else {
            if (transpose) MT_PLANES(double, false, true); else MT_PLANES(double, false, false);
        }
    } else {
        if (bf16) {
            if (transpose) MT_PLANES(float, true, true); else MT_PLANES(float, true, false);
        } else {
            if (transpose) MT_PLANES(float, false, true); else MT_PLANES(float, false, false);
        }
    }
#undef MT_PLANES
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_planes_if(const int32_t* cond, const void* A, const void* B, int src_f64, int bf16, int64_t b,
                            int64_t m, int64_t n, int64_t k, int64_t mp, int64_t np, int64_t kp, const double* r,
                            const double* c, const double* a_mul, const double* b_mul, const PlaneSpec& spec,
                            void* a_planes, void* b_planes, hipStream_t st, const uint32_t* marks,
                            int64_t tile_bm) {
    if (b <= 0 || mp <= 0 || np <= 0 || kp <= 0) return hipSuccess;
    PlanesIfMarks mk;
    mk.marks = marks;
    mk.tile_bm = tile_bm;
    mk.tiles_m = marks ? mp / tile_bm : 0;
    mk.tiles_n = marks ? np / tile_bm : 0;
    // a marked plane row block lies in one tile row or column
    if (marks && (tile_bm <= 0 || mp % tile_bm || np % tile_bm || tile_bm % 64)) return hipErrorInvalidValue;
    auto operand = [&](const void* src, int64_t rows, int64_t rows_pad, const double* sc, const double* mul,
                       void* planes, int64_t tile_t, int64_t tile_u) {
        PlanesIfOperand o;
        o.src = src;
        o.rows = rows;
        o.cols = k;
        o.rows_pad = rows_pad;
        o.cols_pad = kp;
        o.scale_rows = sc;
        o.col_mul = mul;
        o.planes = planes;
        o.gx = (kp + tile_u - 1) / tile_u;
        o.gy = (rows_pad + tile_t - 1) / tile_t;
        o.blocks = o.gx * o.gy * b;
        return o;
    };
    timing_before("mt_planes_if", st);
    // an idle launch (cond clear) costs one short wave per workgroup: a
    // fixed grid of a few workgroups per CU, striding when the planes are due
    auto launch = [&](auto tag) {
        using TS = decltype(tag);
        const PlanesIfOperand oa =
            operand(A, m, mp, r, a_mul, a_planes, PlaneTile<TS, false>::T, PlaneTile<TS, false>::U);
        const PlanesIfOperand ob =
            operand(B, n, np, c, b_mul, b_planes, PlaneTile<TS, true>::T, PlaneTile<TS, true>::U);
        const int64_t total = oa.blocks + ob.blocks;
        const dim3 grid((unsigned)(total < 2048 ? total : 2048));
        if (bf16)
            hipLaunchKernelGGL((mt_planes_if_kernel<TS, true>), grid, dim3(kThreads), 0, st, cond, oa, ob, spec, mk);
        else
            hipLaunchKernelGGL((mt_planes_if_kernel<TS, false>), grid, dim3(kThreads), 0, st, cond, oa, ob, spec,
                               mk);
    };
    if (src_f64)
        launch(double{});
    else
        launch(float{});
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_rowmax_planes_colmax(const float* A, const float* B, int64_t b, int64_t rows, int64_t cols,
                                       int64_t rows_pad, int64_t cols_pad, int64_t nb, double* r, double* c,
                                       int32_t* flag, const PlaneSpec& spec, int bf16, void* planes,
                                       hipStream_t st) {
    if (rows_pad <= 0 || cols_pad <= 0 || b <= 0 || nb <= 0 || cols <= 0)
        return hipErrorInvalidValue;
    if (cols_pad > kFusedRowMaxK || cols > cols_pad) return hipErrorInvalidValue;
    hipError_t e = launch_fill_zero_u32(c, b * nb * 2, st);
    if (e != hipSuccess) return e;
    // B is b x cols x nb (its inner index runs over A's columns)
    const int64_t cgx = (nb + (int64_t)kThreads * 4 - 1) / ((int64_t)kThreads * 4);
    const int64_t cgy = (cols + 63) / 64;
    const int64_t na = rows_pad * b, nc = cgx * cgy * b;
    if (na < nc || na + nc > 0x7fffffff) return hipErrorInvalidValue;
    const int64_t ratio = na / nc;
    timing_before(bf16 ? "mt_power_planes_bf16" : "mt_power_planes_f64", st);
    if (bf16)
        hipLaunchKernelGGL(mt_rowmax_planes_colmax_kernel<true>, dim3((unsigned)(na + nc)), dim3(kThreads), 0, st,
                           A, rows, cols, rows_pad, cols_pad, r, flag, spec, planes, B, cols, nb, c, na, nc, ratio,
                           cgx, cgy);
    else
        hipLaunchKernelGGL(mt_rowmax_planes_colmax_kernel<false>, dim3((unsigned)(na + nc)), dim3(kThreads), 0, st,
                           A, rows, cols, rows_pad, cols_pad, r, flag, spec, planes, B, cols, nb, c, na, nc, ratio,
                           cgx, cgy);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_apsp_transform(const float* W, int64_t n, double s, void* X, int x_f64,
                                 int32_t* flag, hipStream_t st) {
    const dim3 grid(grid_for(n * n, kThreads * 8, 1 << 16));
    timing_before("mt_apsp_transform", st);
    if (x_f64)
        hipLaunchKernelGGL(mt_apsp_transform_kernel<double>, grid, dim3(kThreads), 0, st, W, n, s,
                           (double*)X, flag);
    else
        hipLaunchKernelGGL(mt_apsp_transform_kernel<float>, grid, dim3(kThreads), 0, st, W, n, s,
                           (float*)X, flag);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_apsp_to_dist(const void* X, int x_f64, int64_t n, double s, void* D, int d_f64,
                               int raw, hipStream_t st) {
    const dim3 grid(grid_for(n * n, kThreads * 8, 1 << 16));
    const double s_inv = 1.0 / s;
    timing_before("mt_apsp_to_dist", st);
    if (x_f64) {
        if (d_f64)
            hipLaunchKernelGGL((mt_apsp_to_dist_kernel<double, double>), grid, dim3(kThreads), 0, st,
                               (const double*)X, n * n, s_inv, raw, (double*)D);
        else
            hipLaunchKernelGGL((mt_apsp_to_dist_kernel<double, float>), grid, dim3(kThreads), 0, st,
                               (const double*)X, n * n, s_inv, raw, (float*)D);
    } else {
        if (d_f64)
            hipLaunchKernelGGL((mt_apsp_to_dist_kernel<float, double>), grid, dim3(kThreads), 0, st,
                               (const float*)X, n * n, s_inv, raw, (double*)D);
        else
            hipLaunchKernelGGL((mt_apsp_to_dist_kernel<float, float>), grid, dim3(kThreads), 0, st,
                               (const float*)X, n * n, s_inv, raw, (float*)D);
    }
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_select_root_f64(const double* S, const double* S2, const uint8_t* code, int64_t b,
                                  int64_t m, int64_t n, const double* r, const double* c,
                                  const RootSpec& spec, void* out, int out_f64, uint8_t* pstar_out,
                                  hipStream_t st) {
    const int64_t rows = b * m;
    if (rows <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)(rows < 65535 ? rows : 65535));
    timing_before("mt_select_root_f64", st);
    if (out_f64)
        hipLaunchKernelGGL(mt_select_root_f64_kernel<double>, grid, dim3(kThreads), 0, st, S, S2, code,
                           rows, m, n, r, c, spec, (double*)out, pstar_out);
    else
        hipLaunchKernelGGL(mt_select_root_f64_kernel<float>, grid, dim3(kThreads), 0, st, S, S2, code,
                           rows, m, n, r, c, spec, (float*)out, pstar_out);
    timing_after(st);
    return hipGetLastError();
}

hipError_t launch_select_r2_f64(const double* stack, int64_t stride, int64_t b, int64_t m, int64_t n,
                                const double* r, const double* c, const R2Spec& spec, void* out, int out_f64,
                                uint8_t* pstar_out, hipStream_t st) {
    const int64_t rows = b * m;
    if (rows <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + kThreads - 1) / kThreads), (unsigned)std::min<int64_t>(rows, 65535));
    timing_before("mt_select_r2", st);
    if (out_f64)
        hipLaunchKernelGGL(mt_select_r2_kernel<double>, grid, dim3(kThreads), 0, st, stack, stride, rows, m, n, r, c,
                           spec, (double*)out, pstar_out);
    else
        hipLaunchKernelGGL(mt_select_r2_kernel<float>, grid, dim3(kThreads), 0, st, stack, stride, rows, m, n, r, c,
                           spec, (float*)out, pstar_out);
    timing_after(st);
    return hipGetLastError();
}

}  // namespace mt
