// C ABI of libmaxtimes (include/maxtimes.h): argument checks, workspace
// layout, the launch sequence of the p-norm (max, x) estimate (Alg. 5 with
// the scaled ring call H' of Sec. 2.1) and of the APSP squaring loop (Sec. 2.2),
// and per-kernel event timing.  Host code only; kernels live in
// mt_elementwise.hip, mt_gemm_bf16.hip, mt_gemm_f64.hip and mt_backward.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "mt_internal.h"

namespace mt {

// ------------------------------------------------------------------ errors
namespace {
thread_local std::string g_last_error;

mt_status fail(mt_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

mt_status device_fail(hipError_t e, const char* what) {
    return fail(MT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define MT_TRY(call, what)                                 \
    do {                                                   \
        hipError_t _e = (call);                            \
        if (_e != hipSuccess) return device_fail(_e, what); \
    } while (0)

// ------------------------------------------------------------------ timing
struct TimedLaunch {
    const char* name;
    hipEvent_t start;
    hipEvent_t stop;
    int work_slot;  // index into g_work, -1 if the kernel counts no work
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_launches;
// Events are taken from a pool, filled when timing is switched on and
// refilled at reset, so that a timed launch costs the host two event records
// and no event creation (a host slower than the GPU would otherwise leave the
// GPU idle between an event and its kernel, and the idle time would count).
std::vector<hipEvent_t> g_event_pool;
constexpr size_t kEventPoolFill = 1024;
hipEvent_t take_event() {
    if (g_event_pool.empty()) {
        hipEvent_t e = nullptr;
        return hipEventCreate(&e) == hipSuccess ? e : nullptr;
    }
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
}
// Timing slots of timed launches (kTimingSlotWords counters per launch:
// executed work, first start and last end on the device clock), cleared at
// reset: a device array of the library, so that timing allocates nothing;
// g_work is its address on the device that was current at the first timed
// launch that counts work.
constexpr int kWorkSlots = 2048;
__device__ __align__(256) unsigned long long timing_work_counters[kWorkSlots * kTimingSlotWords];
unsigned long long* g_work = nullptr;
int g_work_used = 0;
// cleared slots: no work, start at the largest value (minimum taken), end 0
hipError_t clear_work_slots(int slots) {
    std::vector<unsigned long long> init((size_t)slots * kTimingSlotWords, 0ull);
    for (int i = 0; i < slots; ++i) init[(size_t)i * kTimingSlotWords + 1] = ~0ull;
    hipError_t e = hipMemcpy(g_work, init.data(), init.size() * sizeof(unsigned long long), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    return e;
}
}  // namespace

void timing_before(const char* name, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing) return;
    TimedLaunch t{name, take_event(), take_event(), -1};
    if (!t.start || !t.stop) return;
    (void)hipEventRecord(t.start, st);
    g_launches.push_back(t);
}

void timing_after(hipStream_t st) {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || g_launches.empty()) return;
    TimedLaunch& t = g_launches.back();
    if (t.stop) (void)hipEventRecord(t.stop, st);
}

unsigned long long* timing_work_slot() {
    std::lock_guard<std::mutex> lk(g_tmu);
    if (!g_timing || g_launches.empty() || g_work_used >= kWorkSlots) return nullptr;
    if (!g_work) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(timing_work_counters)) != hipSuccess) return nullptr;
        g_work = (unsigned long long*)p;
        if (clear_work_slots(kWorkSlots) != hipSuccess) {
            g_work = nullptr;
            return nullptr;
        }
    }
    g_launches.back().work_slot = g_work_used;
    return g_work + (size_t)kTimingSlotWords * g_work_used++;
}

namespace {

// ------------------------------------------------------------------ options
constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Family {
    int32_t n;
    int32_t p[MT_MAX_P];
    bool bf16;
    double tau;
    int32_t split_max_p;
    uint32_t flags;
    // r = 2 projection: the added norms 3p/4 (not in the family), ascending
    int32_t naux;
    int32_t paux[MT_MAX_P];
};

mt_status parse_options(const mt_options* opt, Family* f, bool xy = false) {
    if (!opt) return fail(MT_ERR_INVALID_ARG, "options pointer is NULL");
    if (!opt->p_family) return fail(MT_ERR_INVALID_ARG, "p_family is NULL");
    if (opt->n_p < 1 || opt->n_p > MT_MAX_P)
        return fail(MT_ERR_INVALID_ARG, "n_p = %d outside 1..%d", opt->n_p, MT_MAX_P);
    if (opt->path != MT_PATH_FP64 && opt->path != MT_PATH_BF16_SPLIT)
        return fail(MT_ERR_INVALID_ARG, "unknown path %d", opt->path);
    const uint32_t known = MT_FLAG_VALIDATE | MT_FLAG_NORM_CORRECT | MT_FLAG_CLAMP | MT_FLAG_RAW_OUTPUT |
                           MT_FLAG_PROJECT_R1 | MT_FLAG_PROJECT_R2 | MT_FLAG_XY_PAIRED | MT_FLAG_BALANCE;
    if (opt->flags & ~known) return fail(MT_ERR_INVALID_ARG, "unknown flag bits 0x%x", opt->flags & ~known);
    if ((opt->flags & MT_FLAG_XY_PAIRED) && !xy)
        return fail(MT_ERR_INVALID_ARG, "MT_FLAG_XY_PAIRED is for xy_topk_estimate only");
    if ((opt->flags & (MT_FLAG_PROJECT_R1 | MT_FLAG_PROJECT_R2)) && (opt->flags & MT_FLAG_NORM_CORRECT))
        return fail(MT_ERR_INVALID_ARG, "MT_FLAG_NORM_CORRECT applies to the plain root, not to a projection");
    if ((opt->flags & MT_FLAG_PROJECT_R1) && (opt->flags & MT_FLAG_PROJECT_R2))
        return fail(MT_ERR_INVALID_ARG, "MT_FLAG_PROJECT_R1 and MT_FLAG_PROJECT_R2 exclude each other");
    if ((opt->flags & MT_FLAG_PROJECT_R2) && opt->path != MT_PATH_FP64)
        return fail(MT_ERR_UNSUPPORTED, "MT_FLAG_PROJECT_R2 is implemented on the FP64 path only");
    if (!(opt->tau <= 0.0 || (opt->tau > 0.0 && std::isfinite(opt->tau))))
        return fail(MT_ERR_INVALID_ARG, "tau must be finite");
    f->n = opt->n_p;
    for (int q = 0; q < opt->n_p; ++q) {
        const int32_t p = opt->p_family[q];
        if (p < 1 || p > MT_MAX_POWER)
            return fail(MT_ERR_INVALID_ARG, "p_family[%d] = %d outside 1..%d", q, p, MT_MAX_POWER);
        if (q > 0 && p <= opt->p_family[q - 1])
            return fail(MT_ERR_INVALID_ARG, "p_family is not strictly ascending at index %d", q);
        f->p[q] = p;
    }
    f->bf16 = opt->path == MT_PATH_BF16_SPLIT;
    f->tau = opt->tau > 0.0 ? opt->tau : (f->bf16 ? MT_TAU_BF16_DEFAULT : MT_TAU_FP64_DEFAULT);
    f->split_max_p = opt->split_max_p < 0 ? 4 : opt->split_max_p;
    f->flags = opt->flags;
    f->naux = 0;
    if (f->flags & MT_FLAG_PROJECT_R2) {
        // 3p/4 for every p with p/4 and p/2 in the family, not in it itself
        auto in_family = [&](int32_t v) {
            for (int q = 0; q < f->n; ++q)
                if (f->p[q] == v) return true;
            return false;
        };
        for (int q = 0; q < f->n; ++q) {
            const int32_t p = f->p[q];
            if (p % 4 || !in_family(p / 4) || !in_family(p / 2) || in_family(3 * p / 4)) continue;
            if (f->n + f->naux >= MT_MAX_P)
                return fail(MT_ERR_UNSUPPORTED, "the family and the norms 3p/4 of MT_FLAG_PROJECT_R2 exceed %d powers",
                            MT_MAX_P);
            f->paux[f->naux++] = 3 * p / 4;  // ascending: p ascends
        }
    }
    return MT_OK;
}

// The powers whose planes and ring results a product needs, ascending: the
// family, plus the added norms of the r = 2 projection.
int all_powers(const Family& f, int32_t* out) {
    int a = 0, b = 0, n = 0;
    while (a < f.n || b < f.naux) {
        if (b >= f.naux || (a < f.n && f.p[a] < f.paux[b]))
            out[n++] = f.p[a++];
        else
            out[n++] = f.paux[b++];
    }
    return n;
}

// Planes of one operand: one per p (FP64), or hi (+ lo when split) per p (BF16).
PlaneSpec plane_spec(const Family& f) {
    PlaneSpec s;
    memset(&s, 0, sizeof s);
    int32_t pw[MT_MAX_P];
    s.n_p = all_powers(f, pw);
    int pl = 0;
    for (int q = 0; q < s.n_p; ++q) {
        s.p[q] = pw[q];
        s.split[q] = f.bf16 && pw[q] <= f.split_max_p;
        s.first_plane[q] = pl;
        pl += s.split[q] ? 2 : 1;
    }
    s.n_planes = pl;
    s.write_mask = 0xFFFFFFFFu;
    return s;
}

float round_up_to_float(double tau) {
    float f = (float)tau;
    if ((double)f < tau) f = nextafterf(f, INFINITY);
    return f;
}

// Largest p first; a split p runs (hi,hi), (hi,lo), (lo,hi).  The plan
// covers the powers of the plane spec: the family (pidx = family index), or
// with the r = 2 projection the family and its added norms (pidx = position
// among all of them, the plane of the S stack).
FamilyPlan family_plan(const Family& f, const PlaneSpec& ps, int64_t k) {
    FamilyPlan plan;
    memset(&plan, 0, sizeof plan);
    const int np = ps.n_p;
    const int32_t* P = ps.p;
    plan.n = np;
    plan.r1 = (f.flags & MT_FLAG_PROJECT_R1) ? 1 : 0;
    plan.tau = f.tau;
    plan.tau_f = round_up_to_float(f.tau);
    for (int e = 0; e < np; ++e) {
        const int q = np - 1 - e;
        PlanEntry& pe = plan.e[e];
        pe.pidx = q;
        pe.p = P[q];
        pe.inv_p = 1.0f / (float)P[q];
        pe.inv_dp = q > 0 ? 1.0f / (float)(P[q] - P[q - 1]) : 0.0f;
        pe.corr = (f.flags & MT_FLAG_NORM_CORRECT) && k > 0 ? (float)std::pow((double)k, -1.0 / P[q]) : 1.0f;
        // For terms in [0, 1] and a larger p' > p, S_p' <= S_p^(p'/p).  Below
        // rise_thr no larger p can be stable: the factor 2 under the power
        // covers the rounding of S_p', the factor 0.9 that of S_p (relative
        // errors of a few 2^-8 on the BF16 path, plus terms lost to underflow,
        // each below 2^-126 and together far below tau).
        if (e == 0) {
            pe.rise_thr = INFINITY;
            pe.rise_thr_f = INFINITY;
        } else {
            pe.rise_thr = 0.9 * std::pow(f.tau / 2.0, (double)P[q] / (double)P[q + 1]);
            float tf = (float)pe.rise_thr;
            if ((double)tf > pe.rise_thr) tf = nextafterf(tf, 0.0f);
            pe.rise_thr_f = tf;
        }
        const int hi = ps.first_plane[q];
        if (ps.split[q]) {
            pe.nseg = 3;
            pe.a_plane[0] = hi; pe.b_plane[0] = hi;
            pe.a_plane[1] = hi; pe.b_plane[1] = hi + 1;
            pe.a_plane[2] = hi + 1; pe.b_plane[2] = hi;
        } else {
            pe.nseg = 1;
            pe.a_plane[0] = hi;
            pe.b_plane[0] = hi;
        }
    }
    return plan;
}

// The r = 2 selection over the S stack (planes in the order of ps).
R2Spec r2_spec(const Family& f, const PlaneSpec& ps, int mode, int clamp, int64_t k) {
    R2Spec r;
    memset(&r, 0, sizeof r);
    auto plane_of = [&](int32_t v) {
        for (int t = 0; t < ps.n_p; ++t)
            if (ps.p[t] == v) return t;
        return -1;
    };
    r.n = f.n;
    for (int q = 0; q < f.n; ++q) {
        const int32_t p = f.p[q];
        r.p[q] = p;
        r.plane[q] = plane_of(p);
        r.lo[q] = q > 0 ? plane_of(f.p[q - 1]) : -1;
        const bool ok = p % 4 == 0 && plane_of(p / 4) >= 0 && plane_of(p / 2) >= 0 && plane_of(3 * p / 4) >= 0;
        for (int k = 0; k < 4; ++k) r.q4[q][k] = ok ? plane_of((k + 1) * (p / 4)) : -1;
    }
    r.tau = f.tau;
    r.mode = mode;
    r.clamp = clamp;
    r.k_inner = (double)k;
    return r;
}

RootSpec root_spec(const Family& f, int64_t k, int mode, int clamp) {
    RootSpec r;
    memset(&r, 0, sizeof r);
    for (int q = 0; q < f.n; ++q) {
        r.p[q] = f.p[q];
        r.corr[q] = (f.flags & MT_FLAG_NORM_CORRECT) && k > 0 ? std::pow((double)k, -1.0 / f.p[q]) : 1.0;
    }
    r.mode = mode;
    r.clamp = clamp;
    r.r1 = (f.flags & MT_FLAG_PROJECT_R1) ? 1 : 0;
    return r;
}

// ------------------------------------------------------------------ geometry
struct Geom {
    int64_t mp, np, kp;  // padded sizes of the planes
    int bm;              // FP64 tile (128 or 64); 256 for BF16
    size_t esize;        // plane element bytes
};

Geom product_geom(const Family& f, int64_t b, int64_t m, int64_t k, int64_t n) {
    Geom g;
    if (f.bf16) {
        g.bm = kBf16BM;
        g.kp = round_up(k, kBf16BK);
        g.esize = 2;
    } else {
        // 128-wide tiles when they give at least two workgroups per CU.
        const int64_t tiles128 = b * ((m + 127) / 128) * ((n + 127) / 128);
        g.bm = tiles128 >= 512 ? 128 : 64;
        g.kp = round_up(k, kF64BK);
        g.esize = 8;
    }
    g.mp = round_up(m, g.bm);
    g.np = round_up(n, g.bm);
    return g;
}

struct Layout {
    size_t hdr, r, c, bal, ap, bp, s, s2, code, tail, tail_sorted, tail_bucket, pilot, missed, x, total;
    int32_t tail_max;  // sparse-tail threshold the layout was sized for (0: no tail)
    int32_t tail_shift, tail_buckets;  // row buckets of the tail sort
};

// A tile with at most this many undecided entries hands them to the sparse
// tail (0 disables it).  512 of a 256 x 256 BF16 tile is 0.8 %.
std::atomic<int32_t> g_tail_max{512};
// Products with b m k n up to this many multiply-adds take the one-kernel
// FP64 path (mt_small.hip) when their options allow it; 0: never.
constexpr int64_t kSmallProductDefault = (int64_t)1 << 25;
std::atomic<int64_t> g_small_limit{kSmallProductDefault};

// Forward search start: a plan index, or kStartAuto (the pilot chooses).
constexpr int32_t kStartAuto = -1;
std::atomic<int32_t> g_start_entry{kStartAuto};

// Deferred planes of the smaller p (on by default).
std::atomic<int32_t> g_defer_planes{1};

// The pilot runs for products of at least this many output entries (below,
// its fixed cost is not worth it and the search starts at the largest p).
constexpr int64_t kPilotMinOutputs = (int64_t)1 << 22;
constexpr int32_t kPilotKParts = kMaxPilotKParts;

// The workspace of one product (plus an APSP X buffer when x_bytes > 0).
Layout product_layout(const Family& f, const PlaneSpec& ps, const Geom& g, int64_t b, int64_t m,
                      int64_t k, int64_t n, size_t x_bytes) {
    Layout L;
    size_t off = 0;
    L.hdr = off; off += align_up(sizeof(WsHeader));
    L.r = off;   off += align_up((size_t)(b * m) * 8);
    L.c = off;   off += align_up((size_t)(b * n) * 8);
    // inner-index balancing: column maxima of A, row maxima of B, d, 1 / d
    L.bal = off; off += (f.flags & MT_FLAG_BALANCE) ? 4 * align_up((size_t)(b * k) * 8) : 0;
    L.ap = off;  off += align_up((size_t)b * ps.n_planes * g.mp * g.kp * g.esize);
    L.bp = off;  off += align_up((size_t)b * ps.n_planes * g.np * g.kp * g.esize);
    L.s = L.s2 = L.code = 0;
    const bool r2 = (f.flags & MT_FLAG_PROJECT_R2) != 0;
    if (!f.bf16 && r2) {
        // the S stack: one plane per power of the plane spec
        L.s = off;    off += align_up((size_t)ps.n_p * (size_t)(b * m * n) * 8);
    } else if (!f.bf16) {
        L.s = off;    off += align_up((size_t)(b * m * n) * 8);
        if (f.flags & MT_FLAG_PROJECT_R1) {
            L.s2 = off; off += align_up((size_t)(b * m * n) * 8);
        }
        L.code = off; off += align_up((size_t)(b * m * n));
    }
    // sparse-tail list: at most tail_max entries per tile (none if the family
    // has a single p: nothing would be left to run; none for the r = 2
    // projection, which keeps every ring result)
    L.tail_max = f.n > 1 && !r2 ? g_tail_max.load() : 0;
    const int64_t tiles = b * (g.mp / g.bm) * (g.np / g.bm);
    const size_t list_bytes = align_up((size_t)tiles * (size_t)L.tail_max * sizeof(TailEntry));
    L.tail = off;
    off += list_bytes;
    // the list sorted by row bucket and state (two buckets per row bucket):
    // rows (over the batch) merged in powers of two until at most
    // kTailBuckets buckets remain
    L.tail_shift = 0;
    while (2 * (((b * m - 1) >> L.tail_shift) + 1) > kTailBuckets) ++L.tail_shift;
    L.tail_buckets = L.tail_max > 0 && b * m > 0 ? (int32_t)(2 * (((b * m - 1) >> L.tail_shift) + 1)) : 0;
    L.tail_sorted = off;
    off += L.tail_max > 0 ? list_bytes : 0;
    L.tail_bucket = off;
    off += align_up((size_t)(L.tail_buckets + 3) / 4 * 16);
    // pilot partial sums (float on the BF16 path, double on FP64)
    L.pilot = off;
    off += f.n > 1 ? align_up((size_t)kPilotKParts * f.n * kMaxPilotSide * kMaxPilotSide * (f.bf16 ? 4 : 8)) +
                         align_up(sizeof(PilotCounts))
                   : 0;
    // deferred planes: one word per output tile (with the tail)
    L.missed = off;
    off += L.tail_max > 0 ? align_up((size_t)tiles * 4) : 0;
    L.x = off;
    off += align_up(x_bytes);
    L.total = off;
    return L;
}

mt_status check_dims(int64_t b, int64_t m, int64_t k, int64_t n) {
    if (b < 0 || m < 0 || k < 0 || n < 0)
        return fail(MT_ERR_INVALID_ARG, "negative size (b=%lld m=%lld k=%lld n=%lld)", (long long)b,
                    (long long)m, (long long)k, (long long)n);
    const int64_t lim = (int64_t)1 << 24;
    if (m > lim || n > lim || k > lim || b > lim)
        return fail(MT_ERR_UNSUPPORTED, "a size exceeds 2^24");
    return MT_OK;
}

// The BF16 GEMM addresses a 256-row block of a plane with 32-bit byte
// offsets: the inner (contracted) dimension stays at or below 2^23.
mt_status check_bf16_inner(const Family& f, int64_t inner) {
    if (f.bf16 && inner > ((int64_t)1 << 23))
        return fail(MT_ERR_UNSUPPORTED, "the BF16 path contracts at most 2^23 terms per entry (got %lld)",
                    (long long)inner);
    return MT_OK;
}

mt_status check_ws(void* ws, size_t ws_bytes, size_t need) {
    if (ws_bytes < need)
        return fail(MT_ERR_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (need > 0 && !ws) return fail(MT_ERR_INVALID_ARG, "workspace is NULL");
    if (((uintptr_t)ws) % kAlign) return fail(MT_ERR_INVALID_ARG, "workspace is not 256-byte aligned");
    return MT_OK;
}

mt_status read_domain_flag(const uint8_t* ws, hipStream_t st) {
    int32_t flag = 0;
    MT_TRY(hipMemcpyAsync(&flag, ws, sizeof flag, hipMemcpyDeviceToHost, st), "domain flag copy");
    MT_TRY(hipStreamSynchronize(st), "domain flag sync");
    if (flag) return fail(MT_ERR_DOMAIN, "input has negative, NaN or infinite entries");
    return MT_OK;
}

// Backward workspace: adjoint planes of both gradient products and the
// power planes they multiply (every power split on the BF16 path).
struct BwdLayout {
    int64_t m_out, k_out, n_out;  // output rows / cols padded to the adjoint tile
    int64_t m_in, n_in;           // inner lengths padded to the K step
    int32_t g_planes;             // adjoint planes per batch item
    size_t hdr, r, c, bal, ex, xa, yb, pa, pb, total;
};

BwdLayout backward_layout(const Family& f, int64_t b, int64_t m, int64_t k, int64_t n) {
    BwdLayout L;
    const int64_t bm = f.bf16 ? kAdjBM : kAdjF64BM;
    const int64_t ks = f.bf16 ? kBf16BK : kF64BK;
    const size_t es = f.bf16 ? 2 : 8;
    L.m_out = round_up(m, bm);
    L.k_out = round_up(k, bm);
    L.n_out = round_up(n, bm);
    L.m_in = round_up(m, ks);
    L.n_in = round_up(n, ks);
    L.g_planes = f.bf16 ? 2 * f.n : f.n;
    const int64_t pw_planes = f.bf16 ? 2 * f.n : f.n;
    size_t off = 0;
    L.hdr = off; off += align_up(sizeof(WsHeader));
    L.r = off;   off += align_up((size_t)(b * m) * 8);
    L.c = off;   off += align_up((size_t)(b * n) * 8);
    // balanced forward: column maxima of A, row maxima of B, d, 1 / d
    L.bal = off; off += (f.flags & MT_FLAG_BALANCE) ? 4 * align_up((size_t)(b * k) * 8) : 0;
    L.ex = off;  off += align_up((size_t)(2 * b) * 4);
    L.xa = off;  off += align_up((size_t)b * L.g_planes * L.m_out * L.n_in * es);
    L.yb = off;  off += align_up((size_t)b * L.g_planes * L.n_out * L.m_in * es);
    L.pa = off;  off += align_up((size_t)b * pw_planes * L.k_out * L.n_in * es);
    L.pb = off;  off += align_up((size_t)b * pw_planes * L.k_out * L.m_in * es);
    L.total = off;
    return L;
}

// The product pipeline on already-validated arguments.  X-mode (APSP):
// A = B = X (n x n, r = c = 1 by construction), the output goes back to X.
mt_status run_product(const void* A, const void* B, int in_f64, int64_t b, int64_t m, int64_t k,
                      int64_t n, const Family& f, const PlaneSpec& ps, const Geom& g,
                      const Layout& L, uint8_t* ws, bool scale, int mode, int clamp, void* out,
                      int out_f64, uint8_t* pstar, hipStream_t st, bool fuse_rowmax = false) {
    double* r = scale ? (double*)(ws + L.r) : nullptr;
    double* c = scale ? (double*)(ws + L.c) : nullptr;
    void* ap = ws + L.ap;
    void* bp = ws + L.bp;
    // balanced inputs: A D and D^-1 B, d and 1 / d per inner index
    const bool bal = scale && (f.flags & MT_FLAG_BALANCE);
    const double* d = bal ? (const double*)(ws + L.bal + 2 * align_up((size_t)(b * k) * 8)) : nullptr;
    const double* dinv = bal ? (const double*)(ws + L.bal + 3 * align_up((size_t)(b * k) * 8)) : nullptr;
    const FamilyPlan plan = family_plan(f, ps, k);
    WsHeader* hdr = (WsHeader*)(ws + L.hdr);
    // The pilot chooses where the search starts (below: products large
    // enough, the tail on, no r = 1 projection).
    const int32_t s0 = g_start_entry.load();
    const bool pilot = !plan.r1 && s0 == kStartAuto && L.tail_max > 0 && f.n > 2 && k >= 256 &&
                       b * m * n >= kPilotMinOutputs;
    // Deferred planes (plain products the pilot steers): the planes of the
    // smaller p are written only once some entry needs them, which the
    // pilot's sample tells before the GEMM, or a tile or tail entry that
    // reaches them tells after it (those tiles then run again, after the
    // planes of their rows are written).  BF16 path: the two smallest p;
    // FP64 path, whose tau puts p* near the largest p: all but the three
    // largest.
    const bool defer = pilot && mode == EPI_PLAIN && !(f.flags & MT_FLAG_PROJECT_R2) && plan.n >= 5 &&
                       g_defer_planes.load() != 0;
    const int32_t n_eval = defer ? (f.bf16 ? plan.n - 2 : 3) : plan.n;
    PlaneSpec ps_now = ps, ps_late = ps;
    if (defer) {
        uint32_t late = 0;
        for (int q = 0; q < ps.n_p; ++q)
            for (int e = n_eval; e < plan.n; ++e)
                if (plan.e[e].a_plane[0] == ps.first_plane[q]) late |= 1u << q;
        ps_now.write_mask = ~late;
        ps_late.write_mask = late;
    }
    if (fuse_rowmax) {
        // r and the planes of A in one pass, with c taken by the same launch
        // (neither maximum was taken before)
        MT_TRY(launch_rowmax_planes_colmax((const float*)A, (const float*)B, b, m, k, g.mp, g.kp, n, r, c,
                                           (int32_t*)(ws + L.hdr), ps_now, f.bf16, ap, st),
               "row and column max, power planes (A)");
    } else {
        MT_TRY(launch_power_planes(A, in_f64, 0, b, m, k, g.mp, g.kp, r, nullptr, ps_now, f.bf16, ap, st, d),
               "power planes (A)");
    }
    MT_TRY(launch_power_planes(B, in_f64, 1, b, n, k, g.np, g.kp, c, nullptr, ps_now, f.bf16, bp, st, dinv),
           "power planes (B)");
    EpiArgs epi;
    memset(&epi, 0, sizeof epi);
    epi.r = r;
    epi.c = c;
    if (f.flags & MT_FLAG_PROJECT_R2) {
        // every ring result to the S stack, then selection and projection
        epi.mode = EPI_STORE_ALL;
        epi.out = ws + L.s;
        epi.out_f64 = 1;
        epi.stack_stride = b * m * n;
        MT_TRY(launch_pfamily_gemm_f64((const double*)ap, (const double*)bp, b, m, n, g.mp, g.np, g.kp,
                                       ps.n_planes, g.bm, plan, epi, st),
               "p-family GEMM (FP64, every ring result)");
        const R2Spec rs = r2_spec(f, ps, mode, clamp, k);
        MT_TRY(launch_select_r2_f64((const double*)(ws + L.s), b * m * n, b, m, n, r, c, rs, out, out_f64, pstar,
                                    st),
               "select and r = 2 projection");
        return MT_OK;
    }
    if (!plan.r1) {
        if (pilot) {
            PilotArgs pa;
            memset(&pa, 0, sizeof pa);
            pa.X = ap;
            pa.Y = bp;
            pa.x_plane_elems = g.mp * g.kp;
            pa.y_plane_elems = g.np * g.kp;
            pa.x_batch_elems = pa.x_plane_elems * ps.n_planes;
            pa.y_batch_elems = pa.y_plane_elems * ps.n_planes;
            pa.kp = g.kp;
            pa.rows = m;
            pa.cols = n;
            pa.b = b;
            pa.nr = (int32_t)std::min<int64_t>(kMaxPilotSide, m);
            pa.nc = (int32_t)std::min<int64_t>(kMaxPilotSide, n);
            pa.kparts = (int32_t)std::max<int64_t>(1, std::min<int64_t>(kPilotKParts, g.kp / 512));
            pa.tail_max = L.tail_max;
            pa.tile_entries = (int64_t)std::min<int64_t>(g.bm, m) * std::min<int64_t>(f.bf16 ? kBf16BN : g.bm, n);
            // one tail dot product (two plane rows of k_pad elements from
            // HBM) against one dense tile entry (2 BM BN k_pad flops at the
            // GEMM's rate), measured on MI355X: about 1/250
            pa.kappa = 1.0f / 250.0f;
            pa.part = ws + L.pilot;
            pa.counts = ws + L.pilot + align_up((size_t)kPilotKParts * f.n * kMaxPilotSide * kMaxPilotSide * (f.bf16 ? 4 : 8));
            pa.n_eval = n_eval;
            pa.low_need = defer ? &hdr->low_need : nullptr;
            pa.low_missed = defer ? &hdr->low_missed : nullptr;
            MT_TRY(launch_choose_start(pa, plan, &hdr->start, f.bf16 ? 0 : 1, st), "p search start (pilot)");
            if (defer)
                MT_TRY(launch_planes_if(&hdr->low_need, A, B, in_f64, f.bf16, b, m, n, k, g.mp, g.np, g.kp, r, c,
                                        d, dinv, ps_late, ap, bp, st),
                       "deferred planes (the pilot's sample needs them)");
        } else {
            const int32_t s1 = s0 < 0 ? 0 : (s0 < f.n ? s0 : f.n - 1);
            MT_TRY(launch_fill_u32(&hdr->start, (uint32_t)s1, 1, st), "p search start");
        }
        epi.start = &hdr->start;
    }
    if (L.tail_max > 0 && k > 0) {
        MT_TRY(launch_fill_zero_u32(&hdr->tail_count, 1, st), "clear tail count");
        epi.tail = (TailEntry*)(ws + L.tail);
        epi.tail_count = &hdr->tail_count;
        epi.tail_max = L.tail_max;
        epi.tail_sorted = (TailEntry*)(ws + L.tail_sorted);
        epi.tail_bucket = (int32_t*)(ws + L.tail_bucket);
        epi.tail_shift = L.tail_shift;
        epi.tail_buckets = L.tail_buckets;
    }
    if (f.bf16) {
        epi.mode = mode;
        epi.clamp = clamp;
        epi.out = out;
        epi.out_f64 = out_f64;
        epi.pstar = pstar;
        if (defer) {
            epi.low_need = &hdr->low_need;
            epi.low_missed = &hdr->low_missed;
            epi.missed_tile = (uint32_t*)(ws + L.missed);
            epi.n_eval = n_eval;
        }
        MT_TRY(launch_pfamily_gemm_bf16((const uint16_t*)ap, (const uint16_t*)bp, b, m, n, g.mp, g.np,
                                        g.kp, ps.n_planes, plan, epi, st),
               "p-family GEMM (BF16)");
        if (defer) {
            // tiles or tail entries that reached the deferred planes: write
            // them, then run those tiles again (each launch returns at once
            // when nothing was missed)
            MT_TRY(launch_planes_if(&hdr->low_missed, A, B, in_f64, f.bf16, b, m, n, k, g.mp, g.np, g.kp, r, c,
                                    d, dinv, ps_late, ap, bp, st, epi.missed_tile, g.bm),
                   "deferred planes (after a miss: the marked tiles' rows)");
            MT_TRY(launch_rerun_gemm_bf16((const uint16_t*)ap, (const uint16_t*)bp, b, m, n, g.mp, g.np, g.kp,
                                          ps.n_planes, plan, epi, st),
                   "p-family GEMM (BF16, tiles run again)");
        }
    } else {
        epi.mode = EPI_PLAIN;
        epi.out = ws + L.s;
        epi.out2 = (f.flags & MT_FLAG_PROJECT_R1) ? ws + L.s2 : nullptr;
        epi.out_f64 = 1;
        epi.pstar = ws + L.code;
        if (defer) {
            epi.low_need = &hdr->low_need;
            epi.low_missed = &hdr->low_missed;
            epi.missed_tile = (uint32_t*)(ws + L.missed);
            epi.n_eval = n_eval;
        }
        MT_TRY(launch_pfamily_gemm_f64((const double*)ap, (const double*)bp, b, m, n, g.mp, g.np, g.kp,
                                       ps.n_planes, g.bm, plan, epi, st),
               "p-family GEMM (FP64)");
        if (defer) {
            MT_TRY(launch_planes_if(&hdr->low_missed, A, B, in_f64, f.bf16, b, m, n, k, g.mp, g.np, g.kp, r, c,
                                    d, dinv, ps_late, ap, bp, st, epi.missed_tile, g.bm),
                   "deferred planes (after a miss: the marked tiles' rows)");
            MT_TRY(launch_rerun_gemm_f64((const double*)ap, (const double*)bp, b, m, n, g.mp, g.np, g.kp,
                                         ps.n_planes, g.bm, plan, epi, st),
                   "p-family GEMM (FP64, tiles run again)");
        }
        const RootSpec rsp = root_spec(f, k, mode, clamp);
        MT_TRY(launch_select_root_f64((const double*)(ws + L.s), (const double*)(ws + L.s2), ws + L.code, b, m,
                                      n, r, c, rsp, out, out_f64, pstar, st),
               "select root (FP64)");
    }
    return MT_OK;
}

}  // namespace
}  // namespace mt

using namespace mt;

extern "C" {

const char* maxtimes_version(void) { return "maxtimes-gfx950 0.1"; }

const char* maxtimes_status_string(mt_status s) {
    switch (s) {
        case MT_OK: return "ok";
        case MT_ERR_INVALID_ARG: return "invalid argument";
        case MT_ERR_DOMAIN: return "input outside the domain (negative, NaN or infinite)";
        case MT_ERR_WORKSPACE: return "workspace too small";
        case MT_ERR_DEVICE: return "device or launch failure";
        case MT_ERR_UNSUPPORTED: return "unsupported argument combination";
    }
    return "unknown status";
}

const char* maxtimes_last_error(void) { return g_last_error.c_str(); }

mt_status maxtimes_workspace_size(int64_t b, int64_t m, int64_t k, int64_t n, const mt_options* opt,
                                  size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if ((s = check_dims(b, m, k, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, k)) != MT_OK) return s;
    const PlaneSpec ps = plane_spec(f);
    const Geom g = product_geom(f, b, m, k, n);
    *bytes = product_layout(f, ps, g, b, m, k, n, 0).total;
    return MT_OK;
}

mt_status maxtimes_workspace_map(int64_t b, int64_t m, int64_t k, int64_t n, const mt_options* opt,
                                 mt_workspace_map* map) {
    g_last_error.clear();
    if (!map) return fail(MT_ERR_INVALID_ARG, "map pointer is NULL");
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if ((s = check_dims(b, m, k, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, k)) != MT_OK) return s;
    const PlaneSpec ps = plane_spec(f);
    const Geom g = product_geom(f, b, m, k, n);
    const Layout L = product_layout(f, ps, g, b, m, k, n, 0);
    memset(map, 0, sizeof *map);
    map->r_offset = L.r;
    map->c_offset = L.c;
    map->a_planes_offset = L.ap;
    map->b_planes_offset = L.bp;
    map->m_pad = g.mp;
    map->n_pad = g.np;
    map->k_pad = g.kp;
    map->n_planes = ps.n_planes;
    map->elem_bytes = (int32_t)g.esize;
    map->n_powers = ps.n_p;
    for (int q = 0; q < ps.n_p; ++q) {
        map->power[q] = ps.p[q];
        map->first_plane[q] = ps.first_plane[q];
        map->split[q] = ps.split[q];
    }
    return MT_OK;
}

}  // extern "C"

namespace mt {
namespace {

// ------------------------------------------------------------------ static scratch
// The workspace of maxtimes_estimate_noalloc: a device array of the library.
// Every GPU the library runs on holds its own copy, at its own address, until
// the process ends.  In host code the array's name is not a device address:
// host code uses only the address hipGetSymbolAddress gives for the current
// device, kept per device.
constexpr size_t kScratchBytes = MT_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

mt_status scratch_of_current_device(void** out) {
    int dev = 0;
    MT_TRY(hipGetDevice(&dev), "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(MT_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        MT_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "address of the static scratch");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return MT_OK;
}

// maxtimes_estimate on a caller workspace, or (workspace == nullptr and
// use_scratch) on the static scratch of the current device.
mt_status estimate_impl(const void* A, const void* B, mt_dtype dtype, int64_t b, int64_t m, int64_t k, int64_t n,
                        const mt_options* opt, void* C, uint8_t* p_star, void* workspace, size_t ws_bytes,
                        void* stream, bool use_scratch) {
    g_last_error.clear();
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if (f.flags & MT_FLAG_RAW_OUTPUT) return fail(MT_ERR_INVALID_ARG, "MT_FLAG_RAW_OUTPUT is for apsp_estimate");
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if ((s = check_dims(b, m, k, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, k)) != MT_OK) return s;
    if (b == 0 || m == 0 || n == 0) return MT_OK;
    if (!C) return fail(MT_ERR_INVALID_ARG, "C is NULL");
    if (k > 0 && (!A || !B)) return fail(MT_ERR_INVALID_ARG, "A or B is NULL");
    const PlaneSpec ps = plane_spec(f);
    const Geom g = product_geom(f, b, m, k, n);
    const Layout L = product_layout(f, ps, g, b, m, k, n, 0);
    if (use_scratch) {
        if (L.total > kScratchBytes)
            return fail(MT_ERR_WORKSPACE,
                        "this product needs %zu bytes of workspace; the static scratch of "
                        "maxtimes_estimate_noalloc holds %zu (call maxtimes_estimate with a workspace)",
                        L.total, kScratchBytes);
        if ((s = scratch_of_current_device(&workspace)) != MT_OK) return s;
        ws_bytes = kScratchBytes;
    }
    if ((s = check_ws(workspace, ws_bytes, L.total)) != MT_OK) return s;

    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)workspace;
    const int f64 = dtype == MT_F64;
    // small FP64-path products without projections, balancing or the
    // domain check: one kernel (maxima, powers, ring products, selection)
    const uint32_t small_ok = MT_FLAG_CLAMP | MT_FLAG_NORM_CORRECT;
    if (!f.bf16 && k > 0 && !(f.flags & ~small_ok) && b <= 65535 && (m + 31) / 32 <= 65535 &&
        (double)b * m * k * n <= (double)g_small_limit.load()) {
        SmallSpec sp;
        memset(&sp, 0, sizeof sp);
        const RootSpec rsp = root_spec(f, k, EPI_PLAIN, (f.flags & MT_FLAG_CLAMP) ? 1 : 0);
        sp.n = f.n;
        for (int q = 0; q < f.n; ++q) {
            sp.p[q] = f.p[q];
            sp.corr[q] = rsp.corr[q];
        }
        sp.tau = f.tau;
        sp.clamp = rsp.clamp;
        MT_TRY(launch_small_product_f64(A, B, f64, b, m, k, n, sp, C, f64, p_star, st), "small product (FP64)");
        return MT_OK;
    }
    int32_t* flag = (int32_t*)(ws + L.hdr);
    // everything the kernels expect at zero is cleared by kernels of the
    // call itself (the header: domain flag, tail count, p* histogram), so a
    // workspace that holds an earlier call's contents is fine
    MT_TRY(launch_fill_zero_u32(ws + L.hdr, sizeof(WsHeader) / 4, st), "clear header");
    bool fuse_rowmax = false;
    if ((f.flags & MT_FLAG_BALANCE) && k > 0) {
        // inner-index balancing: a_k = max_i A_ik, b_k = max_j B_kj,
        // d_k = sqrt(b_k / a_k); then r_i = max_k A_ik d_k, c_j = max_k B_kj / d_k
        const size_t sec = align_up((size_t)(b * k) * 8);
        double* amax = (double*)(ws + L.bal);
        double* bmax = (double*)(ws + L.bal + sec);
        double* d = (double*)(ws + L.bal + 2 * sec);
        double* dinv = (double*)(ws + L.bal + 3 * sec);
        MT_TRY(launch_colmax(A, f64, b, m, k, amax, flag, st), "column max of A (balancing)");
        MT_TRY(launch_rowmax(B, f64, b * k, n, bmax, flag, st), "row max of B (balancing)");
        MT_TRY(launch_balance(amax, bmax, b * k, d, dinv, st), "balancing factors");
        MT_TRY(launch_rowmax(A, f64, b * m, k, (double*)(ws + L.r), flag, st, d, m), "row max");
        MT_TRY(launch_colmax(B, f64, b, k, n, (double*)(ws + L.c), flag, st, dinv), "column max");
    } else {
        // FP32 rows that fit one workgroup take their maxima in the plane
        // pass of A, and B's column maxima run in the same launch (unless the
        // domain check must come before the planes)
        fuse_rowmax = !f64 && !(f.flags & MT_FLAG_VALIDATE) && g.kp <= kFusedRowMaxK && b <= 65535 && k > 0 &&
                      n > 0 && g.mp * b >= ((n + 1023) / 1024) * ((k + 63) / 64) * b;
        if (!fuse_rowmax) {
            MT_TRY(launch_rowmax(A, f64, b * m, k, (double*)(ws + L.r), flag, st), "row max");
            MT_TRY(launch_colmax(B, f64, b, k, n, (double*)(ws + L.c), flag, st), "column max");
        }
    }
    if (f.flags & MT_FLAG_VALIDATE) {
        if ((s = read_domain_flag(ws + L.hdr, st)) != MT_OK) return s;
    }
    return run_product(A, B, f64, b, m, k, n, f, ps, g, L, ws, true, EPI_PLAIN,
                       (f.flags & MT_FLAG_CLAMP) ? 1 : 0, C, f64, p_star, st, fuse_rowmax);
}

}  // namespace
}  // namespace mt

extern "C" {

mt_status maxtimes_estimate(const void* A, const void* B, mt_dtype dtype, int64_t b, int64_t m,
                            int64_t k, int64_t n, const mt_options* opt, void* C, uint8_t* p_star,
                            void* workspace, size_t ws_bytes, void* stream) {
    return estimate_impl(A, B, dtype, b, m, k, n, opt, C, p_star, workspace, ws_bytes, stream, false);
}

mt_status maxtimes_estimate_noalloc(const void* A, const void* B, mt_dtype dtype, int64_t b, int64_t m, int64_t k,
                                    int64_t n, const mt_options* opt, void* C, uint8_t* p_star, void* stream) {
    return estimate_impl(A, B, dtype, b, m, k, n, opt, C, p_star, nullptr, 0, stream, true);
}

mt_status apsp_workspace_size(int64_t n, const mt_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if ((s = check_dims(1, n, n, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, n)) != MT_OK) return s;
    if (f.flags & MT_FLAG_BALANCE) return fail(MT_ERR_INVALID_ARG, "MT_FLAG_BALANCE is for maxtimes_estimate");
    const PlaneSpec ps = plane_spec(f);
    const Geom g = product_geom(f, 1, n, n, n);
    *bytes = product_layout(f, ps, g, 1, n, n, n, (size_t)(n * n) * (f.bf16 ? 4 : 8)).total;
    return MT_OK;
}

mt_status apsp_estimate(const float* W, int64_t n, double s_scale, int32_t n_squarings,
                        const mt_options* opt, void* D, mt_dtype d_dtype, uint8_t* p_star_last,
                        void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if (f.flags & MT_FLAG_NORM_CORRECT) return fail(MT_ERR_UNSUPPORTED, "MT_FLAG_NORM_CORRECT is not defined for APSP");
    if (f.flags & MT_FLAG_BALANCE)
        return fail(MT_ERR_INVALID_ARG,
                    "MT_FLAG_BALANCE is for maxtimes_estimate (an APSP operand has row and column maxima 1)");
    if (d_dtype != MT_F32 && d_dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)d_dtype);
    if ((s = check_dims(1, n, n, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, n)) != MT_OK) return s;
    if (!(s_scale > 0.0) || !std::isfinite(s_scale)) return fail(MT_ERR_INVALID_ARG, "s must be finite and > 0");
    if (n == 0) return MT_OK;
    if (!W || !D) return fail(MT_ERR_INVALID_ARG, "W or D is NULL");
    int T = n_squarings;
    if (T < 0) {
        T = 0;
        while (((int64_t)1 << T) < n) ++T;
    }
    if (T > 64) return fail(MT_ERR_INVALID_ARG, "n_squarings = %d is too large", T);
    const PlaneSpec ps = plane_spec(f);
    const Geom g = product_geom(f, 1, n, n, n);
    const int x_f64 = f.bf16 ? 0 : 1;
    const Layout L = product_layout(f, ps, g, 1, n, n, n, (size_t)(n * n) * (x_f64 ? 8 : 4));
    if ((s = check_ws(workspace, ws_bytes, L.total)) != MT_OK) return s;

    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)workspace;
    void* X = ws + L.x;
    int32_t* flag = (int32_t*)(ws + L.hdr);
    MT_TRY(launch_fill_zero_u32(ws + L.hdr, sizeof(WsHeader) / 4, st), "clear header");
    MT_TRY(launch_apsp_transform(W, n, s_scale, X, x_f64, flag, st), "exp transform");
    if (f.flags & MT_FLAG_VALIDATE) {
        if ((s = read_domain_flag(ws + L.hdr, st)) != MT_OK) return s;
    }
    // X has X_ii = 1 and X <= 1 after the transform and after every squaring,
    // so its row and column maxima are 1: the scaled call needs no scaling.
    for (int t = 0; t < T; ++t) {
        s = run_product(X, X, x_f64, 1, n, n, n, f, ps, g, L, ws, false, EPI_APSP_X, 1, X, x_f64,
                        t == T - 1 ? p_star_last : nullptr, st);
        if (s != MT_OK) return s;
    }
    MT_TRY(launch_apsp_to_dist(X, x_f64, n, s_scale, D, d_dtype == MT_F64,
                               (f.flags & MT_FLAG_RAW_OUTPUT) ? 1 : 0, st),
           "log transform");
    return MT_OK;
}

mt_status maxtimes_backward_workspace_size(int64_t b, int64_t m, int64_t k, int64_t n,
                                           const mt_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if ((s = check_dims(b, m, k, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, m > n ? m : n)) != MT_OK) return s;
    *bytes = backward_layout(f, b, m, k, n).total;
    return MT_OK;
}

mt_status maxtimes_estimate_backward(const void* A, const void* B, const void* G, const void* C,
                                     const uint8_t* p_star, mt_dtype dtype, int64_t b, int64_t m,
                                     int64_t k, int64_t n, const mt_options* opt, void* dA, void* dB,
                                     void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    Family f;
    mt_status s = parse_options(opt, &f);
    if (s != MT_OK) return s;
    if (f.flags & (MT_FLAG_NORM_CORRECT | MT_FLAG_CLAMP | MT_FLAG_RAW_OUTPUT | MT_FLAG_PROJECT_R1 | MT_FLAG_PROJECT_R2))
        return fail(MT_ERR_UNSUPPORTED,
                    "the backward supports the plain estimate only (no norm correction, clamp or projection)");
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if ((s = check_dims(b, m, k, n)) != MT_OK) return s;
    if ((s = check_bf16_inner(f, m > n ? m : n)) != MT_OK) return s;
    if (!dA && !dB) return MT_OK;
    if (b == 0 || k == 0) return MT_OK;  // nothing to write (dA, dB are empty)
    if (m > 0 && n > 0 && (!A || !B || !G || !C || !p_star))
        return fail(MT_ERR_INVALID_ARG, "A, B, G, C and p_star must be non-NULL");
    const BwdLayout L = backward_layout(f, b, m, k, n);
    if ((s = check_ws(workspace, ws_bytes, L.total)) != MT_OK) return s;

    hipStream_t st = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)workspace;
    const int f64 = dtype == MT_F64;
    const size_t esz = f64 ? 8 : 4;
    if (m == 0 || n == 0) {
        // C is empty: both gradients are zero
        if (dA) MT_TRY(launch_fill_zero_u32(dA, b * m * k * esz / 4, st), "zero dA");
        if (dB) MT_TRY(launch_fill_zero_u32(dB, b * k * n * esz / 4, st), "zero dB");
        return MT_OK;
    }
    int32_t* flag = (int32_t*)(ws + L.hdr);
    int32_t* hist = ((WsHeader*)(ws + L.hdr))->hist;
    double* r = (double*)(ws + L.r);
    double* c = (double*)(ws + L.c);
    MT_TRY(launch_fill_zero_u32(ws + L.hdr, sizeof(WsHeader) / 4, st), "clear header");
    // A balanced forward (MT_FLAG_BALANCE) is differentiated on the balanced
    // pair (A D, D^-1 B), whose scaled quantities stay in range, and taken
    // back by the chain rule (columns of dA times d_k, rows of dB over d_k);
    // with p* given, C does not depend on d
    const bool bal = (f.flags & MT_FLAG_BALANCE) != 0;
    const size_t bsec = align_up((size_t)(b * k) * 8);
    double* dfac = bal ? (double*)(ws + L.bal + 2 * bsec) : nullptr;
    double* dinv = bal ? (double*)(ws + L.bal + 3 * bsec) : nullptr;
    if (bal) {
        double* amax = (double*)(ws + L.bal);
        double* bmax = (double*)(ws + L.bal + bsec);
        MT_TRY(launch_colmax(A, f64, b, m, k, amax, flag, st), "column max of A (balancing)");
        MT_TRY(launch_rowmax(B, f64, b * k, n, bmax, flag, st), "row max of B (balancing)");
        MT_TRY(launch_balance(amax, bmax, b * k, dfac, dinv, st), "balancing factors");
        MT_TRY(launch_rowmax(A, f64, b * m, k, r, flag, st, dfac, m), "row max");
        MT_TRY(launch_colmax(B, f64, b, k, n, c, flag, st, dinv), "column max");
    } else {
        MT_TRY(launch_rowmax(A, f64, b * m, k, r, flag, st), "row max");
        MT_TRY(launch_colmax(B, f64, b, k, n, c, flag, st), "column max");
    }
    MT_TRY(launch_pstar_hist(p_star, b * m * n, f.n, hist, st), "p* histogram");

    AdjPrepSpec sp;
    memset(&sp, 0, sizeof sp);
    sp.n_p = f.n;
    for (int q = 0; q < f.n; ++q) sp.p[q] = f.p[q];
    sp.planes = L.g_planes;
    sp.xa_rows_pad = L.m_out;
    sp.xa_cols_pad = L.n_in;
    sp.yb_rows_pad = L.n_out;
    sp.yb_cols_pad = L.m_in;
    // BF16 planes carry r_i and c_j divided by a power of two per batch item
    // (their largest value then fits in (0, 1]); the adjoint GEMMs scale back
    int32_t* ex = f.bf16 ? (int32_t*)(ws + L.ex) : nullptr;
    if (ex) MT_TRY(launch_scale_exp(r, c, b, m, n, ex, st), "scale exponents");
    MT_TRY(launch_adjoint_prep(G, C, p_star, f64, r, c, ex, b, m, n, sp, hist, f.bf16, ws + L.xa, ws + L.yb, st),
           "adjoint planes");

    // every power split into hi + lo on the BF16 path (G has mixed signs)
    PlaneSpec ps;
    memset(&ps, 0, sizeof ps);
    ps.n_p = f.n;
    for (int q = 0; q < f.n; ++q) {
        ps.p[q] = f.p[q];
        ps.split[q] = f.bf16 ? 1 : 0;
        ps.first_plane[q] = f.bf16 ? 2 * q : q;
    }
    ps.n_planes = f.bf16 ? 2 * f.n : f.n;
    ps.write_mask = 0xFFFFFFFFu;
    FamilyPlan plan;
    memset(&plan, 0, sizeof plan);
    plan.n = f.n;
    plan.tau = f.tau;
    plan.tau_f = round_up_to_float(f.tau);
    for (int e = 0; e < f.n; ++e) {
        PlanEntry& pe = plan.e[e];
        pe.pidx = e;
        pe.p = f.p[e];
        pe.inv_p = 1.0f / (float)f.p[e];
        pe.corr = 1.0f;
        if (f.bf16) {
            const int h = 2 * e;
            pe.nseg = 3;
            pe.a_plane[0] = h; pe.b_plane[0] = h;
            pe.a_plane[1] = h; pe.b_plane[1] = h + 1;
            pe.a_plane[2] = h + 1; pe.b_plane[2] = h;
        } else {
            pe.nseg = 1;
            pe.a_plane[0] = e;
            pe.b_plane[0] = e;
        }
    }
    if (dA) {
        // dA (m x k) = sum_p A'^(p-1) .* (Gt_p B'^p^T): X = Gt planes (rows m, inner n),
        // Y = B'^p planes (rows k, inner n; B row-major is already K-contiguous)
        MT_TRY(launch_power_planes(B, f64, 0, b, k, n, L.k_out, L.n_in, dfac, c, ps, f.bf16, ws + L.pa, st),
               "power planes (B, adjoint)");
        AdjArgs aa;
        memset(&aa, 0, sizeof aa);
        aa.M = A;
        aa.m_f64 = f64;
        aa.scale_rows = r;
        aa.scale_cols = dinv;   // balanced: A' = A d / r
        aa.out_col_mul = dfac;  // dL/dA = d_k dL/d(A D)
        aa.hist = hist;
        aa.out = dA;
        aa.out_f64 = f64;
        aa.post_exp = ex ? ex + b : nullptr;  // the Gt planes carry c_j / 2^ex
        if (f.bf16)
            MT_TRY(launch_adjoint_gemm_bf16((const uint16_t*)(ws + L.xa), (const uint16_t*)(ws + L.pa), b, m, k,
                                            L.m_out, L.k_out, L.n_in, L.g_planes, ps.n_planes, plan, aa, st),
                   "adjoint GEMM (dA)");
        else
            MT_TRY(launch_adjoint_gemm_f64((const double*)(ws + L.xa), (const double*)(ws + L.pa), b, m, k,
                                           L.m_out, L.k_out, L.n_in, L.g_planes, ps.n_planes, plan, aa, st),
                   "adjoint GEMM (dA)");
    }
    if (dB) {
        // dB (k x n) = sum_p B'^(p-1) .* (A'^p^T Gt'_p): X = A'^p transposed (rows k,
        // inner m), Y = Gt' planes transposed (rows n, inner m)
        MT_TRY(launch_power_planes(A, f64, 1, b, k, m, L.k_out, L.m_in, dinv, r, ps, f.bf16, ws + L.pb, st),
               "power planes (A, adjoint)");
        AdjArgs ab;
        memset(&ab, 0, sizeof ab);
        ab.M = B;
        ab.m_f64 = f64;
        ab.scale_cols = c;
        ab.scale_rows = dfac;   // balanced: B' = B / (d c)
        ab.out_row_mul = dinv;  // dL/dB = dL/d(D^-1 B) / d_k
        ab.hist = hist;
        ab.out = dB;
        ab.out_f64 = f64;
        ab.post_exp = ex;  // the Gt' planes carry r_i / 2^ex
        if (f.bf16)
            MT_TRY(launch_adjoint_gemm_bf16((const uint16_t*)(ws + L.pb), (const uint16_t*)(ws + L.yb), b, k, n,
                                            L.k_out, L.n_out, L.m_in, ps.n_planes, L.g_planes, plan, ab, st),
                   "adjoint GEMM (dB)");
        else
            MT_TRY(launch_adjoint_gemm_f64((const double*)(ws + L.pb), (const double*)(ws + L.yb), b, k, n,
                                           L.k_out, L.n_out, L.m_in, ps.n_planes, L.g_planes, plan, ab, st),
                   "adjoint GEMM (dB)");
    }
    return MT_OK;
}

mt_status maxtimes_exact(const void* A, const void* B, mt_dtype dtype, int64_t b, int64_t m,
                         int64_t k, int64_t n, void* E, void* stream) {
    g_last_error.clear();
    mt_status s = check_dims(b, m, k, n);
    if (s != MT_OK) return s;
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (b == 0 || m == 0 || n == 0) return MT_OK;
    if (!E) return fail(MT_ERR_INVALID_ARG, "E is NULL");
    if (k > 0 && (!A || !B)) return fail(MT_ERR_INVALID_ARG, "A or B is NULL");
    if (b > 65535 || m > ((int64_t)65535 * 64)) return fail(MT_ERR_UNSUPPORTED, "b or m too large for the exact kernel");
    MT_TRY(launch_exact_maxtimes(A, B, dtype == MT_F64, b, m, k, n, E, (hipStream_t)stream), "exact product");
    return MT_OK;
}

// Workspace of maxconv_estimate: empty up to n + m - 1 = kMaxConvN, the
// long-vector buffers above.
struct MaxconvLayout {
    size_t tw, rxy, inv, s_sel, code, buf0, buf1, total;
};
MaxconvLayout maxconv_layout(int64_t b, int64_t n, int64_t m) {
    MaxconvLayout L{};
    const int64_t len = n + m - 1;
    if (len <= kMaxConvN) return L;
    const int64_t N = (int64_t)1 << maxconv_log_size(n, m);
    size_t off = 0;
    L.tw = off;
    off += (size_t)round_up((N / 8 + 1) * 16, kAlign);
    L.rxy = off;
    off += (size_t)round_up(b * 8, kAlign);
    L.inv = off;
    off += (size_t)round_up(2 * b * 8, kAlign);
    L.s_sel = off;
    off += (size_t)round_up(b * len * 8, kAlign);
    L.code = off;
    off += (size_t)round_up(b * len, kAlign);
    L.buf0 = off;
    off += (size_t)round_up(b * N * 16, kAlign);
    L.buf1 = off;
    off += (size_t)round_up(b * N * 16, kAlign);
    L.total = off;
    return L;
}

mt_status maxconv_check(int64_t b, int64_t n, int64_t m, const mt_options* opt, Family* f) {
    mt_status s = parse_options(opt, f);
    if (s != MT_OK) return s;
    if (f->bf16) return fail(MT_ERR_UNSUPPORTED, "the max-convolution runs on the FP64 path only");
    if (f->flags) return fail(MT_ERR_UNSUPPORTED, "the max-convolution takes no flags");
    if (b < 0 || n < 0 || m < 0)
        return fail(MT_ERR_INVALID_ARG, "negative size (b=%lld n=%lld m=%lld)", (long long)b, (long long)n,
                    (long long)m);
    if (b == 0 || n == 0 || m == 0) return MT_OK;
    if (n + m - 1 > kLongConvN)
        return fail(MT_ERR_UNSUPPORTED, "n + m - 1 = %lld exceeds %d", (long long)(n + m - 1), kLongConvN);
    if (b >= ((int64_t)1 << 31)) return fail(MT_ERR_UNSUPPORTED, "b must be below 2^31");
    return MT_OK;
}

mt_status maxconv_workspace_size(int64_t b, int64_t n, int64_t m, const mt_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    Family f;
    mt_status s = maxconv_check(b, n, m, opt, &f);
    if (s != MT_OK) return s;
    *bytes = (b == 0 || n == 0 || m == 0) ? 0 : maxconv_layout(b, n, m).total;
    return MT_OK;
}

mt_status maxconv_estimate(const void* x, const void* y, mt_dtype dtype, int64_t b, int64_t n, int64_t m,
                           const mt_options* opt, void* z, uint8_t* p_star, void* workspace, size_t ws_bytes,
                           void* stream) {
    g_last_error.clear();
    Family f;
    mt_status s = maxconv_check(b, n, m, opt, &f);
    if (s != MT_OK) return s;
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (b == 0 || n == 0 || m == 0) return MT_OK;
    if (!x || !y || !z) return fail(MT_ERR_INVALID_ARG, "x, y or z is NULL");
    const MaxconvLayout L = maxconv_layout(b, n, m);
    s = check_ws(workspace, ws_bytes, L.total);
    if (s != MT_OK) return s;
    MaxconvSpec spec{};
    spec.n = f.n;
    for (int q = 0; q < f.n; ++q) spec.p[q] = f.p[q];
    spec.tau = opt->tau > 0.0 ? opt->tau : MT_TAU_FFT_DEFAULT;
    uint8_t* ws = (uint8_t*)workspace;
    MaxconvWorkspace w{};
    if (L.total) {
        w = MaxconvWorkspace{(double2*)(ws + L.tw), (double*)(ws + L.rxy), (double*)(ws + L.inv),
                             (double*)(ws + L.s_sel), ws + L.code, (double2*)(ws + L.buf0),
                             (double2*)(ws + L.buf1)};
    }
    MT_TRY(launch_maxconv(x, y, dtype == MT_F64, b, n, m, spec, z, p_star, w, (hipStream_t)stream),
           "max-convolution");
    return MT_OK;
}

mt_status maxconv_exact(const void* x, const void* y, mt_dtype dtype, int64_t b, int64_t n, int64_t m,
                        void* z, void* stream) {
    g_last_error.clear();
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (b < 0 || n < 0 || m < 0)
        return fail(MT_ERR_INVALID_ARG, "negative size (b=%lld n=%lld m=%lld)", (long long)b, (long long)n,
                    (long long)m);
    if (b == 0 || n == 0 || m == 0) return MT_OK;
    const int64_t lim = (int64_t)1 << 24;
    if (n > lim || m > lim || b > ((int64_t)1 << 38) / (n + m - 1))
        return fail(MT_ERR_UNSUPPORTED, "n or m above 2^24, or b (n + m - 1) above 2^38");
    if (!x || !y || !z) return fail(MT_ERR_INVALID_ARG, "x, y or z is NULL");
    MT_TRY(launch_maxconv_exact(x, y, dtype == MT_F64, b, n, m, z, (hipStream_t)stream), "exact max-convolution");
    return MT_OK;
}

// Workspace of xy_topk_estimate: the ring results of both runs, then the
// second run's values and both runs' diagonals.
struct XyLayout {
    size_t sigma, psi, values1, diag0, diag1, tw, mxy, buf0, buf1, cand_m, cand_psi, cand_cols, total;
};
XyLayout xy_layout(int64_t n, int32_t k, int n_p) {
    XyLayout L{};
    const int64_t len = 2 * n - 1;
    size_t off = 0;
    L.sigma = off;
    off += (size_t)round_up(2 * (int64_t)n_p * len * 8, kAlign);
    L.psi = off;
    off += (size_t)round_up(2 * len * 8, kAlign);
    L.values1 = off;
    off += (size_t)round_up((int64_t)k * 8, kAlign);
    L.diag0 = off;
    off += (size_t)round_up((int64_t)k * 4, kAlign);
    L.diag1 = off;
    off += (size_t)round_up((int64_t)k * 4, kAlign);
    L.tw = L.mxy = L.buf0 = L.buf1 = 0;
    if (len > kMaxConvN) {
        const int logN = maxconv_log_size(n, n);
        const int64_t N = (int64_t)1 << logN;
        L.tw = off;
        off += (size_t)round_up((N / 8 + 1) * 16, kAlign);
        L.mxy = off;
        off += kAlign;
        L.buf0 = off;
        off += (size_t)round_up(2 * (int64_t)n_p * N * 16, kAlign);
        L.buf1 = off;
        off += (size_t)round_up(2 * (int64_t)n_p * N * 16, kAlign);
    }
    L.cand_m = L.cand_psi = L.cand_cols = 0;
    if (k > 0 && k <= kPairedMaxK) {
        const int64_t K = k < len ? k : len;
        L.cand_m = off;
        off += (size_t)round_up(2 * K * 4, kAlign);
        L.cand_psi = off;
        off += (size_t)round_up(2 * K * 8, kAlign);
        L.cand_cols = off;
        off += (size_t)round_up(2 * (int64_t)n_p * K * 8, kAlign);
    }
    L.total = off;
    return L;
}

mt_status xy_check(int64_t n, int32_t k, const mt_options* opt, Family* f) {
    mt_status s = parse_options(opt, f, true);
    if (s != MT_OK) return s;
    if (f->bf16) return fail(MT_ERR_UNSUPPORTED, "the x + y top k runs on the FP64 path only");
    if (f->flags & ~MT_FLAG_XY_PAIRED)
        return fail(MT_ERR_UNSUPPORTED, "the x + y top k takes no flag but MT_FLAG_XY_PAIRED");
    if (n < 1 || k < 0) return fail(MT_ERR_INVALID_ARG, "need n >= 1 and k >= 0 (n=%lld k=%d)", (long long)n, k);
    if ((f->flags & MT_FLAG_XY_PAIRED) && k > kPairedMaxK)
        return fail(MT_ERR_UNSUPPORTED, "the paired queue takes k <= %d (k=%d)", kPairedMaxK, k);
    if (2 * n - 1 > kLongConvN)
        return fail(MT_ERR_UNSUPPORTED, "2n - 1 = %lld exceeds %d", (long long)(2 * n - 1), kLongConvN);
    if (k > (1 << 24)) return fail(MT_ERR_UNSUPPORTED, "k above 2^24");
    return MT_OK;
}

mt_status xy_topk_workspace_size(int64_t n, int32_t k, const mt_options* opt, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    Family f;
    mt_status s = xy_check(n, k, opt, &f);
    if (s != MT_OK) return s;
    *bytes = xy_layout(n, k, f.n).total;
    return MT_OK;
}

mt_status xy_topk_estimate(const void* x, const void* y, mt_dtype dtype, int64_t n, int32_t k,
                           const mt_options* opt, double* values, int32_t* diag, int32_t* i_idx,
                           int32_t* j_idx, void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    Family f;
    mt_status s = xy_check(n, k, opt, &f);
    if (s != MT_OK) return s;
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (!x || !y) return fail(MT_ERR_INVALID_ARG, "x or y is NULL");
    if (k > 0 && !values) return fail(MT_ERR_INVALID_ARG, "values is NULL");
    const bool paired = (f.flags & MT_FLAG_XY_PAIRED) != 0;
    const XyLayout L = xy_layout(n, k, f.n);
    s = check_ws(workspace, ws_bytes, L.total);
    if (s != MT_OK) return s;
    MaxconvSpec spec{};
    spec.n = f.n;
    for (int q = 0; q < f.n; ++q) spec.p[q] = f.p[q];
    spec.tau = opt->tau > 0.0 ? opt->tau : MT_TAU_FFT_DEFAULT;
    uint8_t* ws = (uint8_t*)workspace;
    XyWorkspace w{(double*)(ws + L.sigma), (double*)(ws + L.psi), (double*)(ws + L.values1),
                  (int32_t*)(ws + L.diag0), (int32_t*)(ws + L.diag1),
                  L.tw ? (double2*)(ws + L.tw) : nullptr, L.mxy ? (double*)(ws + L.mxy) : nullptr,
                  L.buf0 ? (double2*)(ws + L.buf0) : nullptr, L.buf1 ? (double2*)(ws + L.buf1) : nullptr,
                  L.cand_m ? (int32_t*)(ws + L.cand_m) : nullptr, L.cand_psi ? (double*)(ws + L.cand_psi) : nullptr,
                  L.cand_cols ? (double*)(ws + L.cand_cols) : nullptr};
    MT_TRY(launch_xy_topk(x, y, dtype == MT_F64, n, k, spec, paired, values, diag, i_idx, j_idx, w,
                          (hipStream_t)stream),
           "x + y top k");
    return MT_OK;
}

mt_status apsp_exact_rows_workspace_size(int64_t n, int32_t n_src, size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    if (n < 0 || n_src < 0) return fail(MT_ERR_INVALID_ARG, "negative size (n=%lld n_src=%d)", (long long)n, n_src);
    if (n > ((int64_t)1 << 24) || n_src > 65535 * 64)
        return fail(MT_ERR_UNSUPPORTED, "n above 2^24 or n_src above 65535 x 64");
    *bytes = exact_rows_workspace(n, n_src);
    return MT_OK;
}

mt_status apsp_exact_rows(const float* W, int64_t n, const int32_t* sources, int32_t n_src, double* D,
                          int64_t* rounds, void* workspace, size_t ws_bytes, void* stream) {
    g_last_error.clear();
    size_t need = 0;
    mt_status s = apsp_exact_rows_workspace_size(n, n_src, &need);
    if (s != MT_OK) return s;
    if (n == 0 || n_src == 0) {
        if (rounds) *rounds = 0;
        return MT_OK;
    }
    if (!W || !sources || !D) return fail(MT_ERR_INVALID_ARG, "W, sources or D is NULL");
    if ((s = check_ws(workspace, ws_bytes, need)) != MT_OK) return s;
    int64_t r = 0;
    int32_t bad = 0;
    MT_TRY(launch_exact_rows(W, n, sources, n_src, D, (uint8_t*)workspace, (hipStream_t)stream, &r, &bad),
           "exact rows (Bellman-Ford)");
    if (bad) return fail(MT_ERR_INVALID_ARG, "a source index is outside 0..%lld", (long long)(n - 1));
    if (rounds) *rounds = r;
    return MT_OK;
}

mt_status apsp_affine_workspace_size(size_t* bytes) {
    g_last_error.clear();
    if (!bytes) return fail(MT_ERR_INVALID_ARG, "bytes pointer is NULL");
    *bytes = affine_workspace();
    return MT_OK;
}

mt_status apsp_affine_correct(void* D, mt_dtype dtype, int64_t n, const int32_t* sources, int32_t n_src,
                              const double* exact, double* ab, int32_t apply, void* workspace, size_t ws_bytes,
                              void* stream) {
    g_last_error.clear();
    if (dtype != MT_F32 && dtype != MT_F64) return fail(MT_ERR_INVALID_ARG, "unknown dtype %d", (int)dtype);
    if (n < 0 || n_src < 0) return fail(MT_ERR_INVALID_ARG, "negative size (n=%lld n_src=%d)", (long long)n, n_src);
    if (n > ((int64_t)1 << 24)) return fail(MT_ERR_UNSUPPORTED, "n above 2^24");
    if (!ab) return fail(MT_ERR_INVALID_ARG, "ab is NULL");
    if (n > 0 && (!D || (n_src > 0 && (!sources || !exact))))
        return fail(MT_ERR_INVALID_ARG, "D, sources or exact is NULL");
    mt_status s = check_ws(workspace, ws_bytes, affine_workspace());
    if (s != MT_OK) return s;
    MT_TRY(launch_affine_correct(D, dtype == MT_F64, n, sources, n_src, exact, ab, (uint8_t*)workspace,
                                 apply != 0 && n > 0, (hipStream_t)stream),
           "affine correction");
    return MT_OK;
}

mt_status maxtimes_set_tail_threshold(int32_t max_entries) {
    g_last_error.clear();
    if (max_entries < 0 || max_entries > 65536)
        return fail(MT_ERR_INVALID_ARG, "tail threshold %d outside 0..65536", max_entries);
    g_tail_max.store(max_entries);
    return MT_OK;
}

int32_t maxtimes_tail_threshold(void) { return g_tail_max.load(); }

mt_status maxtimes_set_search_start(int32_t entry) {
    g_last_error.clear();
    if (entry < -1 || entry >= MT_MAX_P)
        return fail(MT_ERR_INVALID_ARG, "search start %d outside -1..%d", entry, MT_MAX_P - 1);
    g_start_entry.store(entry);
    return MT_OK;
}

int32_t maxtimes_search_start(void) { return g_start_entry.load(); }

mt_status maxtimes_set_deferred_planes(int32_t on) {
    g_last_error.clear();
    if (on != 0 && on != 1) return fail(MT_ERR_INVALID_ARG, "deferred planes switch %d is not 0 or 1", on);
    g_defer_planes.store(on);
    return MT_OK;
}

int32_t maxtimes_deferred_planes(void) { return g_defer_planes.load(); }

mt_status maxtimes_set_small_product_limit(int64_t max_work) {
    g_last_error.clear();
    if (max_work < 0) return fail(MT_ERR_INVALID_ARG, "small-product limit %lld is negative", (long long)max_work);
    g_small_limit.store(max_work);
    return MT_OK;
}

int64_t maxtimes_small_product_limit(void) { return g_small_limit.load(); }

mt_status maxtimes_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    while (g_timing && g_event_pool.size() < kEventPoolFill) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) break;
        g_event_pool.push_back(e);
    }
    if (g_timing && !g_work) {
        // the timing slots' address and their first clearing (a synchronous
        // copy) here, not inside the first timed launch that counts work,
        // whose pair of events would otherwise hold that copy and the wait
        // for everything queued before it
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(timing_work_counters)) == hipSuccess) {
            g_work = (unsigned long long*)p;
            if (clear_work_slots(kWorkSlots) != hipSuccess) g_work = nullptr;
        }
    }
    return MT_OK;
}

mt_status maxtimes_timing_reset(void) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_tmu);
    for (auto& t : g_launches) {
        if (t.stop) (void)hipEventSynchronize(t.stop);
        if (t.start) g_event_pool.push_back(t.start);
        if (t.stop) g_event_pool.push_back(t.stop);
    }
    g_launches.clear();
    if (g_work && g_work_used > 0) {
        hipError_t e = clear_work_slots(g_work_used);
        if (e != hipSuccess) return device_fail(e, "clearing the work counters");
    }
    g_work_used = 0;
    return MT_OK;
}

mt_status maxtimes_timing_read(const char* prefix, double* total_ms, int64_t* launches) {
    g_last_error.clear();
    if (!prefix || !total_ms || !launches) return fail(MT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    double ms = 0.0;
    int64_t cnt = 0;
    const size_t pl = strlen(prefix);
    for (auto& t : g_launches) {
        if (strncmp(t.name, prefix, pl) != 0 || !t.stop) continue;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e != hipSuccess) return device_fail(e, "event sync");
        float x = 0.f;
        e = hipEventElapsedTime(&x, t.start, t.stop);
        if (e != hipSuccess) return device_fail(e, "event elapsed");
        ms += x;
        ++cnt;
    }
    *total_ms = ms;
    *launches = cnt;
    return MT_OK;
}

mt_status maxtimes_timing_work(const char* prefix, double* flops) {
    g_last_error.clear();
    if (!prefix || !flops) return fail(MT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    *flops = 0.0;
    if (!g_work || g_work_used == 0) return MT_OK;
    const size_t pl = strlen(prefix);
    for (auto& t : g_launches) {
        if (strncmp(t.name, prefix, pl) != 0 || !t.stop) continue;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e != hipSuccess) return device_fail(e, "event sync");
    }
    std::vector<unsigned long long> w((size_t)g_work_used * kTimingSlotWords);
    hipError_t e = hipMemcpy(w.data(), g_work, w.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "reading the work counters");
    double sum = 0.0;
    for (auto& t : g_launches)
        if (t.work_slot >= 0 && strncmp(t.name, prefix, pl) == 0)
            sum += (double)w[(size_t)t.work_slot * kTimingSlotWords];
    *flops = sum;
    return MT_OK;
}

mt_status maxtimes_timing_span(const char* prefix, double* total_ms, int64_t* launches) {
    g_last_error.clear();
    if (!prefix || !total_ms || !launches) return fail(MT_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_tmu);
    *total_ms = 0.0;
    *launches = 0;
    if (!g_work || g_work_used == 0) return MT_OK;
    const size_t pl = strlen(prefix);
    for (auto& t : g_launches) {
        if (strncmp(t.name, prefix, pl) != 0 || !t.stop) continue;
        hipError_t e = hipEventSynchronize(t.stop);
        if (e != hipSuccess) return device_fail(e, "event sync");
    }
    int dev = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e != hipSuccess) return device_fail(e, "reading the device clock rate");
    if (khz <= 0) return fail(MT_ERR_UNSUPPORTED, "the device reports no real-time clock rate");
    std::vector<unsigned long long> w((size_t)g_work_used * kTimingSlotWords);
    e = hipMemcpy(w.data(), g_work, w.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return device_fail(e, "reading the timing slots");
    double ticks = 0.0;
    int64_t cnt = 0;
    for (auto& t : g_launches) {
        if (t.work_slot < 0 || strncmp(t.name, prefix, pl) != 0) continue;
        const unsigned long long t0 = w[(size_t)t.work_slot * kTimingSlotWords + 1];
        const unsigned long long t1 = w[(size_t)t.work_slot * kTimingSlotWords + 2];
        if (t1 < t0) continue;  // the kernel records no span
        ticks += (double)(t1 - t0);
        ++cnt;
    }
    *total_ms = ticks / (double)khz;
    *launches = cnt;
    return MT_OK;
}

}  // extern "C"
