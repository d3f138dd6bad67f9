// C ABI of the PEOs search library (declarations and contracts: include/peos.h).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/peos.h"
#include "k_edge_build.hpp"
#include "k_query_table.hpp"
#include "k_search.hpp"
#include "k_descend.hpp"

struct peos_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    int device;
};

// launch-plan overrides of one index (0 = automatic); they change speed only
struct PeosTuning {
    int hash_cap = 0, listcap = 0, slots = 0, waves = 0;
    bool no_long = false;  // never choose the long-vector variant
};
constexpr int kNumClassTunings = 8;  // ef classes of a split batch

struct peos_index {
    const int32_t* perm;     // dimension permutation of the test, or null
    const float* sdirs;      // 64 x d SimHash vectors (PEOS_FLAG_SIMHASH), or null
    int64_t sig_off;         // SimHash signatures within a record
    const float* base;
    const uint16_t* base16;  // bfloat16 traversal copy inside index_mem, or null
    const int32_t* graph;
    const float* dirs_a;
    const float* dirs_b;
    uint8_t* rec;
    int64_t n;
    int32_t d, R, L, m, metric, flags, entry;
    int64_t node_stride, codes_off, scal_off, bf16_off;
    int device;
    int num_cu;          // compute units of the device
    int64_t lds_per_cu;  // LDS bytes per compute unit
    // launch plan overrides: for every call, and per ef class of a split batch
    std::mutex* tune_mu = nullptr;
    PeosTuning tune;
    PeosTuning class_tune[kNumClassTunings];
    // upper layers for the entry descent (peos_set_upper_layers), or null
    const int32_t* up_node = nullptr;
    const int32_t* up_adj = nullptr;
    const int32_t* up_down = nullptr;
    int32_t up_ru = 0, up_top = 0;
};

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess) return fail(PEOS_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kMaxSlots = 4096;      // resident search waves at most
constexpr int kMaxEf = 4096;
// the search kernel's static LDS: its copy of the arguments and the
// leader's posted gather (waves per query)
constexpr int64_t kStaticLds = 272;

int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct Layout {
    int64_t stride, codes_off, scal_off, sig_off;
};

constexpr int kFlagsAll = PEOS_FLAG_BF16_BASE | PEOS_FLAG_FP16 | PEOS_FLAG_COMPACT;  // kernel variants
constexpr int kFlagsKnown = kFlagsAll | PEOS_FLAG_SIMHASH;
static_assert(PEOS_FLAG_COMPACT == peos::kFlagCompact, "flag values of the kernel variants");

// record of a node: codes [R][round_up(L+1, 4)] bytes | pad to 16 | scalars
// [R][4] floats (halves with PEOS_FLAG_FP16) | with PEOS_FLAG_SIMHASH, pad to
// 16 and [R] 64-bit sign signatures | pad to 128.  With
// PEOS_FLAG_BF16_BASE the n x d bfloat16 copy follows the records.
// code bytes per edge of the full records: room for the codes of the
// search kernel's subspace bound (8, 16 or 32) plus the residual code, so a
// lane loads its edge's codes with a fixed number of dword loads
int64_t code_bytes_of(int L) { return round_up((L <= 8 ? 8 : (L <= 16 ? 16 : 32)) + 1, 4); }

Layout layout_of(int R, int L, int flags)
{
    Layout l;
    if (flags & PEOS_FLAG_COMPACT) {
        // node header (16 bytes) | 4 code bytes per edge | 2 scalar bytes per edge
        l.codes_off = 16;
        l.scal_off = 16 + 4LL * R;
        l.sig_off = 0;
        l.stride = round_up(l.scal_off + 2LL * R, 128);
        return l;
    }
    l.codes_off = 0;
    l.scal_off = round_up((int64_t)R * code_bytes_of(L), 16);
    const int64_t end = l.scal_off + ((flags & PEOS_FLAG_FP16) ? 8LL : 16LL) * R;
    l.sig_off = (flags & PEOS_FLAG_SIMHASH) ? round_up(end, 16) : 0;
    l.stride = round_up((flags & PEOS_FLAG_SIMHASH) ? l.sig_off + 8LL * R : end, 128);
    return l;
}

int check_shape(int64_t n, int32_t d, int32_t R, int32_t L, int32_t m)
{
    if (n < 1 || n > 0x7fffffffLL) return fail(PEOS_EINVAL, "n=%lld out of range [1, 2^31)", (long long)n);
    if (d < 4 || d % 4) return fail(PEOS_EINVAL, "d=%d must be a positive multiple of 4", d);
    if (R < 1 || R > 64) return fail(PEOS_EINVAL, "R=%d must be in [1, 64]", R);
    if (L < 1 || L > 32 || d % L) return fail(PEOS_EINVAL, "L=%d must divide d=%d and be <= 32", L, d);
    if ((d / L) % 4) return fail(PEOS_EINVAL, "d/L=%d must be a multiple of 4", d / L);
    if (m < 16 || m % 16 || 2 * m > 256) return fail(PEOS_EINVAL, "m=%d must be 16, 32, .. 128", m);
    return PEOS_OK;
}

// the current device, checked to be a gfx950 once, with its compute-unit
// count and LDS per compute unit (the launch plans are sized from these)
struct DeviceInfo {
    int checked = 0;  // 1 gfx950, -1 other
    int num_cu = 0;
    int64_t lds_per_cu = 0;
};

int check_device(int* dev, DeviceInfo* info = nullptr)
{
    HIP_TRY(hipGetDevice(dev));
    static std::mutex mu;
    static DeviceInfo devs[64];
    std::lock_guard<std::mutex> g(mu);
    if (*dev < 0 || *dev >= 64) return fail(PEOS_EDEVICE, "device index %d", *dev);
    DeviceInfo& di = devs[*dev];
    if (di.checked == 0) {
        hipDeviceProp_t p;
        HIP_TRY(hipGetDeviceProperties(&p, *dev));
        di.checked = (std::strncmp(p.gcnArchName, "gfx950", 6) == 0) ? 1 : -1;
        di.num_cu = p.multiProcessorCount;
        di.lds_per_cu = (int64_t)p.maxSharedMemoryPerMultiProcessor;
        if (di.num_cu < 1 || di.lds_per_cu < 64 * 1024) di.checked = -1;
    }
    if (di.checked < 0) return fail(PEOS_EDEVICE, "device %d is not a gfx950 (CUs %d, LDS/CU %lld)", *dev, di.num_cu, (long long)di.lds_per_cu);
    if (info) *info = di;
    return PEOS_OK;
}

// Standard normal quantile: Acklam's rational approximation (2003) refined
// by one Halley step on the erfc form of the CDF (full double precision).
double norm_ppf(double p)
{
    static const double a[] = {-3.969683028665376e+01, 2.209460984245205e+02, -2.759285104469687e+02,
                               1.383577518672690e+02, -3.066479806614716e+01, 2.506628277459239e+00};
    static const double b[] = {-5.447609879822406e+01, 1.615858368580409e+02, -1.556989798598866e+02,
                               6.680131188771972e+01, -1.328068155288572e+01};
    static const double c[] = {-7.784894002430293e-03, -3.223964580411365e-01, -2.400758277161838e+00,
                               -2.549732539343734e+00, 4.374664141464968e+00, 2.938163982698783e+00};
    static const double dd[] = {7.784695709041462e-03, 3.224671290700398e-01, 2.445134137142996e+00,
                                3.754408661907416e+00};
    const double plow = 0.02425, phigh = 1 - plow;
    double x;
    if (p < plow) {
        double q = std::sqrt(-2 * std::log(p));
        x = (((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
            ((((dd[0] * q + dd[1]) * q + dd[2]) * q + dd[3]) * q + 1);
    } else if (p <= phigh) {
        double q = p - 0.5, r = q * q;
        x = (((((a[0] * r + a[1]) * r + a[2]) * r + a[3]) * r + a[4]) * r + a[5]) * q /
            (((((b[0] * r + b[1]) * r + b[2]) * r + b[3]) * r + b[4]) * r + 1);
    } else {
        double q = std::sqrt(-2 * std::log(1 - p));
        x = -(((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
            ((((dd[0] * q + dd[1]) * q + dd[2]) * q + dd[3]) * q + 1);
    }
    const double e = 0.5 * std::erfc(-x / std::sqrt(2.0)) - p;
    const double u = e * std::sqrt(2 * M_PI) * std::exp(x * x / 2);
    return x - u / (1 + x * u / 2);
}

static_assert(kNumClassTunings == peos::kMaxClasses, "one tuning per ef class");

// The quantile table of the compact form (Sec. 4.3 reads the quantile from a
// table): entry b = T(b / bins) of step (6) with w_reg = 1, w_res = 0,
// evaluated in double precision on the host and rounded down to single (the
// smallest T of its bin, since T grows with A, so the table never raises the
// threshold).
void compact_lut(int L, double eta, double c_eps, float* lut)
{
    for (int b = 0; b < peos::kCompactLutBins; ++b) {
        const double A = (double)b / peos::kCompactLutBins;
        const double t = A * eta + c_eps * std::sqrt(1.0 - (double)L * A * A / (double)(L + 1));
        float f = (float)t;
        if ((double)f > t) f = std::nextafter(f, -INFINITY);
        lut[b] = f;
    }
}

// the index's overrides for a launch of ef class cls (-1: no class split)
PeosTuning tuning_of(const peos_index* ix, int cls)
{
    std::lock_guard<std::mutex> g(*ix->tune_mu);
    PeosTuning t = ix->tune;
    if (cls >= 0 && cls < kNumClassTunings) {
        const PeosTuning& c = ix->class_tune[cls];
        if (c.hash_cap > 0) t.hash_cap = c.hash_cap;
        if (c.slots > 0) t.slots = c.slots;
        if (c.waves > 0) t.waves = c.waves;
    }
    return t;
}

// The search kernels may use up to 64 KB of LDS; raise the limit once per
// device (not a stream operation, so it also holds for captured launches).
int ensure_kernel_attrs(int dev)
{
    static std::mutex mu;
    static bool done[64] = {false};
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64) return fail(PEOS_EDEVICE, "device index %d", dev);
    if (!done[dev]) {
#define PEOS_FNS(ML, RG)                                                                      \
    (const void*)peos::k_search<ML, 0, RG>, (const void*)peos::k_search<ML, 1, RG>,          \
        (const void*)peos::k_search<ML, 2, RG>, (const void*)peos::k_search<ML, 3, RG>
#define PEOS_FNS_LONG(ML)                                                                     \
    (const void*)peos::k_search<ML, 16, false>, (const void*)peos::k_search<ML, 17, false>,   \
        (const void*)peos::k_search<ML, 18, false>, (const void*)peos::k_search<ML, 19, false>
        const void* fns[] = {PEOS_FNS(8, false),  PEOS_FNS(16, false), PEOS_FNS(32, false),
                             PEOS_FNS(8, true),   PEOS_FNS(16, true),  PEOS_FNS(32, true),
                             (const void*)peos::k_search<8, 8, false>,
                             (const void*)peos::k_search<8, 9, false>,
                             (const void*)peos::k_search<8, 8, true>,
                             (const void*)peos::k_search<8, 9, true>,
                             PEOS_FNS_LONG(16), PEOS_FNS_LONG(32)};
#undef PEOS_FNS_LONG
#undef PEOS_FNS
        for (const void* f : fns)
            HIP_TRY(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024));
        HIP_TRY(hipFuncSetAttribute((const void*)peos::k_query_table,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, 64 * 1024));
        done[dev] = true;
    }
    return PEOS_OK;
}

// words of one visited bitmap: n bits, a whole number of 16-byte blocks (so
// a slot's bitmap is cleared with 16-byte stores)
// per-slot spill region: the visited bitmap (n bits in whole 16-byte
// blocks), then, from n = 2^19 on, a list of 4,096 ids that lets a spilled
// query clear just the words it set (below that a whole clear is cheap)
int64_t spill_bitmap_words_of(const peos_index* ix) { return round_up((ix->n + 31) / 32, 4); }
int64_t spill_list_cap_of(const peos_index* ix) { return spill_bitmap_words_of(ix) >= 16384 ? 4096 : 0; }
int64_t spill_words_of(const peos_index* ix) { return spill_bitmap_words_of(ix) + spill_list_cap_of(ix); }

struct SearchPlan {
    bool list_in_lds;  // a list capacity was forced: keep the list in LDS
    bool regl;         // the list lives in registers (no LDS list)
    bool long_rows;    // the low-occupancy variant for long vectors
    int waves;         // wavefronts per query (workgroup size / 64)
    int listcap, listslack, hcap, visit_limit, slots;
    int64_t lds;
    int64_t spill_words;
};

// per_query: k or ef given per query (then queries may have ef below efmax)
// resident waves per CU that the search kernel's registers allow (four SIMDs)
constexpr int64_t kSearchWavesPerCu = 4 * PEOS_SEARCH_WAVES_PER_EU;

SearchPlan plan_search(const peos_index* ix, int64_t nq, int efmax, int pool, bool per_query,
                       int cls = -1)
{
    SearchPlan p;
    const PeosTuning t = tuning_of(ix, cls);
    const int64_t lds_cu = ix->lds_per_cu;
    const int64_t ncu = ix->num_cu;
    const int lmin = pool < 0 ? -pool * efmax : (pool > efmax ? pool : efmax);
    // unbounded queue: room for 16 ef entries (the list of the printed Alg. 1
    // stays well below that in practice), at most 2048
    int lc = pool != 0 ? lmin : (16 * efmax > 256 ? 16 * efmax : 256);
    if (pool == 0 && lc > 2048) lc = lmin > 2048 ? lmin : 2048;
    if (t.listcap > 0) lc = t.listcap > lmin ? t.listcap : lmin;
    p.list_in_lds = t.listcap > 0;
    lc = (int)round_up(lc, 64);
    if (lc > kMaxEf * 2) lc = kMaxEf * 2;
    p.listcap = lc;
    // list entries first (the visited hash is sized below)
    p.listslack = (pool > 0 && pool <= efmax && !per_query) ? 0 : 64;
    // the list in registers when every query's capacity is its own ef
    // (<= 64): pool = 1 with per-query lists, or pool <= ef with one list
    // size; it then takes no LDS (the output reuses the visited hash)
    p.regl = efmax <= 64 && pool > 0 && (per_query ? pool == 1 : pool <= efmax) &&
             !p.list_in_lds;
    // the table row width of the kernel instantiation: MAXL + 1
    const int64_t tw = (ix->L <= 8 ? 8 : (ix->L <= 16 ? 16 : 32)) + 1;
    const int64_t fixed = 4LL * ix->d + 8LL * tw * ix->m +
                          (p.regl ? 0 : 8LL * (lc + p.listslack)) + 4LL * 2 * 64;
    // visited hash.  A query that fills 7/8 of it moves to the HBM bitmap,
    // where every visited test is a memory round trip on its chain.  With a
    // bounded list: 20 slots per list entry (on the 1M SIFT-like graph a
    // quarter to two fifths of the queries then spill at ef = 72 to 128, and
    // that beats a hash large enough to keep them all, which costs resident
    // waves: 26 slots per entry searched 5-9% slower), but no more than lets
    // the batch's queries share the CUs (ceil(nq / CUs) of them, at most 11
    // per CU: a small batch at a large ef keeps every query resident), and at
    // least what fits the LDS share of the 16 waves per CU the kernel's
    // registers allow; 1024 to 8192.  The unbounded queue (pool = 0) visits
    // several times more nodes per list entry: 32 slots per entry, from 2048,
    // and for lists up to 64 the 16-wave fit.
    const int64_t fit = (lds_cu / kSearchWavesPerCu - kStaticLds - fixed) / 4;
    int hc;
    if (pool != 0) {
        int64_t q_cu = (nq + ncu - 1) / ncu;
        q_cu = q_cu < 1 ? 1 : (q_cu > 11 ? 11 : q_cu);
        const int64_t share = (lds_cu / q_cu - kStaticLds - fixed) / 4;
        int64_t want = 20LL * efmax;
        if (want > share) want = share;
        hc = (int)(want > fit ? want : fit);
    } else {
        hc = 2048;
        while (hc < 32 * efmax && hc < 8192) hc *= 2;
        if (hc == 2048 && fit < hc) hc = (int)fit;
    }
    hc = hc < 1024 ? 1024 : (hc > 8192 ? 8192 : hc);
    if (t.hash_cap > 0) hc = t.hash_cap;
    hc &= ~3;  // whole buckets of four slots
    if (p.regl && hc < 2 * 64) hc = 2 * 64;  // the output staging of the register list
    p.hcap = hc;
    p.visit_limit = (7 * hc) / 8;
    // survivor ids and distances | qv | table | list (lc + slack; none in
    // registers) | hash.
    // A merge writes up to one wave of survivors past the capacity; that
    // room (slack) is needed only when entries past ef are kept (pool above
    // ef, or the unbounded queue); when the capacity is ef they are dropped.
    p.lds = fixed + 4LL * hc;
    int64_t per_cu = lds_cu / (p.lds + kStaticLds);
    if (per_cu < 1) per_cu = 1;
    if (per_cu > kSearchWavesPerCu) per_cu = kSearchWavesPerCu;
    // long vectors (d > 512, L > 8, list in LDS): when the LDS or the batch
    // allows at most 8 waves per CU anyway, the variant with the registers
    // of two waves per SIMD keeps twice the rows in flight
    p.long_rows = ix->d > 512 && ix->L > 8 && !(ix->flags & PEOS_FLAG_COMPACT) && !p.regl &&
                  (per_cu <= 8 || nq <= 8 * ncu) && !t.no_long;
    if (p.long_rows && per_cu > 8) per_cu = 8;
    // waves per query: the registers allow 16 waves per CU (8 with the
    // long-vector variant); when the batch leaves room, give each query 2 or
    // 4 waves (its rows gathered by all of them) as long as every query of
    // the batch is still resident at once
    const int64_t wpc = p.long_rows ? 8 : kSearchWavesPerCu;
    int waves = 1;
    if (t.waves > 0) {
        waves = t.waves;
    } else {
        for (int cand = peos::kMaxWavesPerQuery; cand > 1; cand >>= 1) {
            const int64_t q_cu = per_cu < wpc / cand ? per_cu : wpc / cand;
            if (nq <= q_cu * ncu) {
                waves = cand;
                break;
            }
        }
    }
    p.waves = waves;
    if (per_cu > wpc / waves) per_cu = wpc / waves;
    if (per_cu < 1) per_cu = 1;
    int64_t slots = per_cu * ncu;
    if (slots > kMaxSlots) slots = kMaxSlots;
    if (t.slots > 0) slots = t.slots;
    if (slots > nq) slots = nq;
    p.slots = (int)(slots > 0 ? slots : 1);
    p.spill_words = spill_words_of(ix);
    return p;
}

// workspace: work counters (one per ef class) and class ranges | quantile
// table of the compact form | tables | norms | query order of the class split
// | entries of the descent | one visited bitmap per resident workgroup (last,
// so that the offsets before it do not depend on the number of workgroups)
struct WsLayout {
    int64_t counter_off, ranges_off, lut_off, tables_off, qnorm_off, qperm_off, entries_off,
        spill_off, slots, total;
};

// slots: visited bitmaps to hold (resident workgroups of the launch); 0 =
// as many as a launch of nq queries may have
WsLayout ws_layout(const peos_index* ix, int64_t nq, int64_t spill_words, int64_t slots = 0)
{
    WsLayout w;
    if (slots <= 0) slots = nq < kMaxSlots ? nq : kMaxSlots;
    if (slots < 1) slots = 1;
    w.counter_off = 0;
    w.ranges_off = 64;
    w.lut_off = 256;
    w.tables_off = round_up(w.lut_off + 4 * peos::kCompactLutBins, 256);
    w.qnorm_off = round_up(w.tables_off + nq * (int64_t)(ix->L + 1) * ix->m * 4, 256);
    w.qperm_off = round_up(w.qnorm_off + nq * 4, 256);
    w.entries_off = round_up(w.qperm_off + nq * 4, 256);
    w.spill_off = round_up(w.entries_off + nq * 4, 256);
    w.slots = slots;
    w.total = round_up(w.spill_off + slots * spill_words * 4, 256);
    return w;
}

// number of ef classes a batch with list sizes up to efmax is split into
int num_classes(int efmax)
{
    int c = 1;
    while (c < peos::kMaxClasses && efmax > (32 << (c - 1))) ++c;
    return c;
}

}  // namespace

namespace peos {

// Calibration: random 512-byte rows gathered the way the search gathers
// survivor rows (8 lanes per row, 4 float4 loads each, two groups of 8 rows
// in flight per wave), `iters` rounds per wave, row indices from a
// multiplicative hash of (wave, round, slot) reduced to [0, n_rows).
__global__ __launch_bounds__(64) void k_probe_gather(const float4* rows, int64_t n_rows, int iters,
                                                     float* sink)
{
    const int lane = lane_id();
    const int grp = lane >> 3, sub = lane & 7;
    float acc = 0.f;
    for (int it = 0; it < iters; ++it) {
        float4 v[2][4];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const uint64_t key = ((uint64_t)blockIdx.x * 131071u + (uint64_t)it * 8191u +
                                  (uint64_t)(h * 8 + grp)) * 0x9E3779B97F4A7C15ull;
            const int64_t r = (int64_t)((key >> 17) % (uint64_t)n_rows);
            const float4* row = rows + r * 32;
#pragma unroll
            for (int k = 0; k < 4; ++k) v[h][k] = row[sub + 8 * k];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int k = 0; k < 4; ++k) acc += v[h][k].x + v[h][k].y + v[h][k].z + v[h][k].w;
    }
    acc = wave_sum(acc);
    if (lane == 0) sink[blockIdx.x] = acc;
}

}  // namespace peos

extern "C" {

const char* peos_last_error(void) { return g_err; }

int peos_set_long_rows(peos_index* ix, int32_t enable)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (enable != 0 && enable != 1) return fail(PEOS_EINVAL, "enable=%d", enable);
    std::lock_guard<std::mutex> g(*ix->tune_mu);
    ix->tune.no_long = enable == 0;
    return PEOS_OK;
}

static int check_waves(int32_t waves)
{
    if (waves != 0 && waves != 1 && waves != 2 && waves != 4)
        return fail(PEOS_EINVAL, "waves=%d not in {0, 1, 2, 4}", waves);
    return PEOS_OK;
}

int peos_set_search_tuning(peos_index* ix, int32_t hash_cap, int32_t listcap, int32_t slots,
                           int32_t waves)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (hash_cap != 0 && (hash_cap < 64 || hash_cap > 16384))
        return fail(PEOS_EINVAL, "hash_cap=%d not in [64, 16384]", hash_cap);
    if (listcap < 0 || listcap > 2 * kMaxEf) return fail(PEOS_EINVAL, "listcap=%d", listcap);
    if (slots < 0 || slots > kMaxSlots) return fail(PEOS_EINVAL, "slots=%d", slots);
    int rc = check_waves(waves);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(*ix->tune_mu);
    ix->tune.hash_cap = hash_cap;
    ix->tune.listcap = listcap;
    ix->tune.slots = slots;
    ix->tune.waves = waves;
    return PEOS_OK;
}

int peos_set_class_tuning(peos_index* ix, int32_t cls, int32_t hash_cap, int32_t slots,
                          int32_t waves)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (cls < 0 || cls >= peos::kMaxClasses) return fail(PEOS_EINVAL, "class %d not in [0, %d)", cls, peos::kMaxClasses);
    if (hash_cap != 0 && (hash_cap < 64 || hash_cap > 16384))
        return fail(PEOS_EINVAL, "hash_cap=%d not in [64, 16384]", hash_cap);
    if (slots < 0 || slots > kMaxSlots) return fail(PEOS_EINVAL, "slots=%d", slots);
    int rc = check_waves(waves);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(*ix->tune_mu);
    ix->class_tune[cls].hash_cap = hash_cap;
    ix->class_tune[cls].slots = slots;
    ix->class_tune[cls].waves = waves;
    return PEOS_OK;
}

const char* peos_strerror(int code)
{
    switch (code) {
    case PEOS_OK: return "ok";
    case PEOS_EINVAL: return "invalid argument";
    case PEOS_ENOSPACE: return "buffer too small";
    case PEOS_EHIP: return "HIP runtime error";
    case PEOS_EGRAPH: return "invalid graph (id out of range, self loop or repeated neighbour)";
    case PEOS_EDEVICE: return "no gfx950 device";
    case PEOS_EBUSY: return "request queue full";
    default: return "unknown error";
    }
}

int peos_index_bytes(int64_t n, int32_t d, int32_t R, int32_t L, int32_t m, int32_t flags,
                     size_t* index_bytes, size_t* build_ws_bytes)
{
    if (!index_bytes || !build_ws_bytes) return fail(PEOS_EINVAL, "null output pointer");
    if (flags & ~kFlagsKnown) return fail(PEOS_EINVAL, "flags=%d not supported", flags);
    if ((flags & PEOS_FLAG_COMPACT) && L > 4)
        return fail(PEOS_EINVAL, "PEOS_FLAG_COMPACT needs L <= 4 (L=%d)", L);
    if ((flags & PEOS_FLAG_COMPACT) && (flags & (PEOS_FLAG_FP16 | PEOS_FLAG_SIMHASH)))
        return fail(PEOS_EINVAL, "PEOS_FLAG_COMPACT does not combine with PEOS_FLAG_FP16 or PEOS_FLAG_SIMHASH");
    int rc = check_shape(n, d, R, L, m);
    if (rc) return rc;
    Layout l = layout_of(R, L, flags);
    int64_t bytes = n * l.stride;
    if (flags & PEOS_FLAG_BF16_BASE) bytes = round_up(bytes, 256) + n * (int64_t)d * 2;
    *index_bytes = (size_t)bytes;
    *build_ws_bytes = 256;
    return PEOS_OK;
}

int peos_build_tables(const float* base, int64_t n, int32_t d, const int32_t* graph, int32_t R,
                      int32_t entry, int32_t L, int32_t m, const float* dirs_a,
                      const float* dirs_b, int32_t metric, int32_t flags, void* index_mem,
                      size_t index_bytes, void* ws, size_t ws_bytes, void* stream,
                      peos_index** out)
{
    return peos_build_tables_ex(base, n, d, graph, R, entry, L, m, dirs_a, dirs_b, metric, flags,
                                nullptr, index_mem, index_bytes, ws, ws_bytes, stream, out);
}

int peos_build_tables_ex(const float* base, int64_t n, int32_t d, const int32_t* graph, int32_t R,
                         int32_t entry, int32_t L, int32_t m, const float* dirs_a,
                         const float* dirs_b, int32_t metric, int32_t flags,
                         const peos_build_options* opt, void* index_mem, size_t index_bytes,
                         void* ws, size_t ws_bytes, void* stream, peos_index** out)
{
    const int32_t* perm = opt ? opt->perm : nullptr;
    const float* sdirs = opt ? opt->simhash_dirs : nullptr;
    if ((flags & PEOS_FLAG_SIMHASH) && !sdirs) return fail(PEOS_EINVAL, "PEOS_FLAG_SIMHASH needs simhash_dirs");
    if ((flags & PEOS_FLAG_SIMHASH) && perm) return fail(PEOS_EINVAL, "a dimension permutation does not combine with PEOS_FLAG_SIMHASH");
    if (!out) return fail(PEOS_EINVAL, "null output handle");
    *out = nullptr;
    size_t need = 0, need_ws = 0;
    int rc = peos_index_bytes(n, d, R, L, m, flags, &need, &need_ws);
    if (rc) return rc;
    if (!base || !graph || !dirs_a || !dirs_b || !index_mem || !ws)
        return fail(PEOS_EINVAL, "null device pointer");
    if (((uintptr_t)base & 15u) != 0 || ((uintptr_t)index_mem & 15u) != 0 ||
        ((uintptr_t)dirs_a & 15u) != 0 || ((uintptr_t)dirs_b & 15u) != 0)
        return fail(PEOS_EINVAL, "base, dirs_a, dirs_b and index_mem must be 16-byte aligned");
    if (entry < 0 || entry >= n) return fail(PEOS_EINVAL, "entry=%d out of range", entry);
    if (metric != PEOS_METRIC_L2 && metric != PEOS_METRIC_ANGULAR && metric != PEOS_METRIC_IP)
        return fail(PEOS_EINVAL, "metric=%d", metric);
    if (index_bytes < need) return fail(PEOS_ENOSPACE, "index_bytes %zu < %zu", index_bytes, need);
    if (ws_bytes < need_ws) return fail(PEOS_ENOSPACE, "ws_bytes %zu < %zu", ws_bytes, need_ws);
    int dev;
    DeviceInfo di;
    rc = check_device(&dev, &di);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    Layout l = layout_of(R, L, flags);
    int32_t* err = (int32_t*)ws;
    hipLaunchKernelGGL(peos::k_zero_u32, dim3(1), dim3(64), 0, s, (uint32_t*)err, 1);
    peos::EdgeBuildArgs a;
    a.base = base;
    a.graph = graph;
    a.dirs_a = dirs_a;
    a.dirs_b = dirs_b;
    a.rec = (uint8_t*)index_mem;
    a.err = err;
    a.n = n;
    a.node_stride = l.stride;
    a.codes_off = l.codes_off;
    a.scal_off = l.scal_off;
    a.d = d;
    a.R = R;
    a.L = L;
    a.m = m;
    a.metric = metric;
    a.half_scalars = (flags & PEOS_FLAG_FP16) ? 1 : 0;
    a.perm = perm;
    a.sdirs = (flags & PEOS_FLAG_SIMHASH) ? sdirs : nullptr;
    a.sig_off = l.sig_off;
    a.compact = (flags & PEOS_FLAG_COMPACT) ? 1 : 0;
    size_t lds = sizeof(float) * (size_t)(5 * d + 4 * L) + sizeof(int32_t) * (size_t)R * 4;
    hipLaunchKernelGGL(peos::k_edge_build, dim3((unsigned)n), dim3(64), lds, s, a);
    HIP_TRY(hipGetLastError());
    const int64_t bf16_off = (flags & PEOS_FLAG_BF16_BASE) ? round_up(n * l.stride, 256) : 0;
    if (flags & PEOS_FLAG_BF16_BASE) {
        hipLaunchKernelGGL(peos::k_to_bf16, dim3(4096), dim3(256), 0, s, base,
                           (uint16_t*)((uint8_t*)index_mem + bf16_off), n * (int64_t)d);
        HIP_TRY(hipGetLastError());
    }
    int32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(PEOS_EGRAPH, "graph has an id out of range, a self loop or a repeated neighbour");
    peos_index* ix = new (std::nothrow) peos_index;
    if (!ix) return fail(PEOS_EINVAL, "out of host memory");
    ix->tune_mu = new (std::nothrow) std::mutex;
    if (!ix->tune_mu) {
        delete ix;
        return fail(PEOS_EINVAL, "out of host memory");
    }
    ix->perm = perm;
    ix->sdirs = (flags & PEOS_FLAG_SIMHASH) ? sdirs : nullptr;
    ix->sig_off = l.sig_off;
    ix->base = base;
    ix->base16 = (flags & PEOS_FLAG_BF16_BASE) ? (const uint16_t*)((uint8_t*)index_mem + bf16_off) : nullptr;
    ix->bf16_off = bf16_off;
    ix->graph = graph;
    ix->dirs_a = dirs_a;
    ix->dirs_b = dirs_b;
    ix->rec = (uint8_t*)index_mem;
    ix->n = n;
    ix->d = d;
    ix->R = R;
    ix->L = L;
    ix->m = m;
    ix->metric = metric;
    ix->flags = flags;
    ix->entry = entry;
    ix->node_stride = l.stride;
    ix->codes_off = l.codes_off;
    ix->scal_off = l.scal_off;
    ix->device = dev;
    ix->num_cu = di.num_cu;
    ix->lds_per_cu = di.lds_per_cu;
    *out = ix;
    return PEOS_OK;
}

int peos_index_layout(const peos_index* ix, peos_layout* out)
{
    if (!ix || !out) return fail(PEOS_EINVAL, "null pointer");
    out->n = ix->n;
    out->d = ix->d;
    out->R = ix->R;
    out->L = ix->L;
    out->m = ix->m;
    out->metric = ix->metric;
    out->flags = ix->flags;
    out->entry = ix->entry;
    out->node_stride = ix->node_stride;
    out->codes_offset = ix->codes_off;
    out->scalars_offset = ix->scal_off;
    const bool compact = (ix->flags & PEOS_FLAG_COMPACT) != 0;
    out->code_bytes = compact ? 4 : code_bytes_of(ix->L);
    out->scalar_bytes = compact ? 2 : ((ix->flags & PEOS_FLAG_FP16) ? 8 : 16);
    out->bf16_offset = ix->bf16_off;
    out->simhash_offset = ix->sig_off;
    return PEOS_OK;
}

void peos_free(peos_index* ix)
{
    if (!ix) return;
    delete ix->tune_mu;
    delete ix;
}

int peos_set_upper_layers(peos_index* ix, const peos_upper_layers* up)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (!up) {
        ix->up_node = ix->up_adj = ix->up_down = nullptr;
        return PEOS_OK;
    }
    if (up->levels < 1 || up->levels > 32 || up->R < 1 || up->R > 64 || up->rows < 1 ||
        up->rows > 0x7fffffffLL || !up->layer_start || !up->node || !up->adj || !up->down)
        return fail(PEOS_EINVAL, "levels=%d R=%d rows=%lld", up->levels, up->R, (long long)up->rows);
    const int64_t* ls = up->layer_start;
    if (ls[0] != 0 || ls[up->levels] != up->rows)
        return fail(PEOS_EINVAL, "layer_start must run from 0 to rows");
    for (int l = 0; l < up->levels; ++l)
        if (ls[l + 1] <= ls[l]) return fail(PEOS_EINVAL, "layer %d is empty", l + 1);
    if (up->top < ls[up->levels - 1] || up->top >= up->rows)
        return fail(PEOS_EINVAL, "top=%lld is not a row of the top layer", (long long)up->top);
    const int64_t rows = up->rows;
    std::vector<int32_t> node((size_t)rows), down((size_t)rows), adj((size_t)rows * up->R);
    HIP_TRY(hipMemcpy(node.data(), up->node, node.size() * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(down.data(), up->down, down.size() * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(adj.data(), up->adj, adj.size() * 4, hipMemcpyDeviceToHost));
    for (int l = 0; l < up->levels; ++l) {
        for (int64_t r = ls[l]; r < ls[l + 1]; ++r) {
            if (node[r] < 0 || node[r] >= ix->n)
                return fail(PEOS_EINVAL, "row %lld: node %d out of range", (long long)r, node[r]);
            for (int j = 0; j < up->R; ++j) {
                const int32_t nb = adj[(size_t)r * up->R + j];
                if (nb == -1) continue;
                if (nb < ls[l] || nb >= ls[l + 1] || nb == r)
                    return fail(PEOS_EINVAL, "row %lld: neighbour row %d outside its layer", (long long)r, nb);
            }
            const int32_t dn = down[r];
            if (l == 0 ? dn != -1 : (dn < ls[l - 1] || dn >= ls[l] || node[dn] != node[r]))
                return fail(PEOS_EINVAL, "row %lld: down=%d is not the same node one layer below", (long long)r, dn);
        }
    }
    ix->up_node = up->node;
    ix->up_adj = up->adj;
    ix->up_down = up->down;
    ix->up_ru = up->R;
    ix->up_top = (int32_t)up->top;
    return PEOS_OK;
}

int peos_query_tables(const peos_index* ix, const float* queries, int64_t nq, float* tables,
                      float* qnorms, void* stream)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (nq < 0) return fail(PEOS_EINVAL, "nq=%lld", (long long)nq);
    if (nq == 0) return PEOS_OK;
    if (!queries || !tables || !qnorms) return fail(PEOS_EINVAL, "null device pointer");
    if (((uintptr_t)queries & 15u) != 0) return fail(PEOS_EINVAL, "queries must be 16-byte aligned");
    peos::QueryTableArgs a;
    a.queries = queries;
    a.dirs_a = ix->dirs_a;
    a.dirs_b = ix->dirs_b;
    a.tables = tables;
    a.qnorms = qnorms;
    a.nq = nq;
    a.d = ix->d;
    a.L = ix->L;
    a.m = ix->m;
    a.half_out = (ix->flags & PEOS_FLAG_FP16) ? 1 : 0;
    a.perm = ix->perm;
    const int64_t blocks = (nq + 15) / 16;
    const size_t tile = sizeof(float) * 16 * (size_t)(ix->d + 4);
    a.staged = tile <= 64 * 1024 ? 1 : 0;
    // staged rows; with m = 16 the parts of the full-space tile reuse them
    // (at least 4 waves x 64 lanes x 4 floats)
    const size_t parts = ix->m == 16 ? sizeof(float) * 4 * 64 * peos::kTableWaves : 0;
    const size_t lds = a.staged ? std::max(tile, parts) : 0;
    int rc = ensure_kernel_attrs(ix->device);
    if (rc) return rc;
    hipLaunchKernelGGL(peos::k_query_table, dim3((unsigned)blocks), dim3(64 * peos::kTableWaves),
                       lds, (hipStream_t)stream, a);
    HIP_TRY(hipGetLastError());
    return PEOS_OK;
}

int peos_search_ws_bytes(const peos_index* ix, int64_t nq, int32_t efmax, int32_t pool,
                         size_t* ws_bytes)
{
    if (!ix || !ws_bytes) return fail(PEOS_EINVAL, "null pointer");
    if (nq < 0 || efmax < 1 || efmax > kMaxEf || pool < -16 || pool > 2 * kMaxEf)
        return fail(PEOS_EINVAL, "nq=%lld efmax=%d pool=%d", (long long)nq, efmax, pool);
    WsLayout w = ws_layout(ix, nq, spill_words_of(ix));
    *ws_bytes = (size_t)w.total;
    return PEOS_OK;
}

// one launch of the search kernel for the queries of qrange (all queries
// when qperm is null), planned for list sizes up to efmax
static int launch_search(const peos_index* ix, const peos::SearchArgs& base_args, int64_t nq,
                         int efmax, int pool, bool per_query, int cls, const uint32_t* counter,
                         int slots_cap, hipStream_t s)
{
    SearchPlan plan = plan_search(ix, nq, efmax, pool, per_query, cls);
    // the list in registers when every query's capacity is its own ef
    // (<= 64): pool = 1 with per-query lists, or pool <= ef with one list size
    const bool regl = plan.regl;
    if (slots_cap > 0 && plan.slots > slots_cap) plan.slots = slots_cap;
    if (plan.lds + kStaticLds > 64 * 1024) return fail(PEOS_EINVAL, "list/visited capacity needs %lld bytes of LDS", (long long)plan.lds);
    peos::SearchArgs a = base_args;
    a.counter = const_cast<uint32_t*>(counter);
    a.spill_words = (int32_t)plan.spill_words;
    a.spill_bitmap_words = (int32_t)spill_bitmap_words_of(ix);
    a.spill_list_cap = (int32_t)spill_list_cap_of(ix);
    a.listcap = plan.listcap;
    a.listslack = plan.listslack;
    a.hcap = plan.hcap;
    a.visit_limit = plan.visit_limit;
    const dim3 grid((unsigned)plan.slots);
    const dim3 block((unsigned)(64 * plan.waves));
    static_assert(sizeof(peos::SearchArgs) + 16 <= kStaticLds, "argument copy must fit its LDS share");
    const size_t lds = (size_t)plan.lds;
#define PEOS_LAUNCH2(ML, RG)                                                                      \
    switch (ix->flags & kFlagsAll) {                                                              \
    case 0: hipLaunchKernelGGL((peos::k_search<ML, 0, RG>), grid, block, lds, s, a); break;     \
    case 1: hipLaunchKernelGGL((peos::k_search<ML, 1, RG>), grid, block, lds, s, a); break;     \
    case 2: hipLaunchKernelGGL((peos::k_search<ML, 2, RG>), grid, block, lds, s, a); break;     \
    default: hipLaunchKernelGGL((peos::k_search<ML, 3, RG>), grid, block, lds, s, a); break;    \
    }
#define PEOS_LAUNCH_LONG(ML)                                                                      \
    switch (ix->flags & kFlagsAll) {                                                              \
    case 0: hipLaunchKernelGGL((peos::k_search<ML, 16, false>), grid, block, lds, s, a); break; \
    case 1: hipLaunchKernelGGL((peos::k_search<ML, 17, false>), grid, block, lds, s, a); break; \
    case 2: hipLaunchKernelGGL((peos::k_search<ML, 18, false>), grid, block, lds, s, a); break; \
    default: hipLaunchKernelGGL((peos::k_search<ML, 19, false>), grid, block, lds, s, a); break;\
    }
#define PEOS_LAUNCH(ML)                                                                           \
    if (regl) { PEOS_LAUNCH2(ML, true) } else { PEOS_LAUNCH2(ML, false) }
    static_assert(peos::kVariantLong == 16, "long-vector variants are FLAGS + 16");
    // compact records (L <= 4): their own variants of the L <= 8 kernel
    if (ix->flags & PEOS_FLAG_COMPACT) {
        const bool bf = (ix->flags & PEOS_FLAG_BF16_BASE) != 0;
        if (regl && bf) hipLaunchKernelGGL((peos::k_search<8, 9, true>), grid, block, lds, s, a);
        else if (regl) hipLaunchKernelGGL((peos::k_search<8, 8, true>), grid, block, lds, s, a);
        else if (bf) hipLaunchKernelGGL((peos::k_search<8, 9, false>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((peos::k_search<8, 8, false>), grid, block, lds, s, a);
    } else if (ix->L <= 8) { PEOS_LAUNCH(8) }
    else if (plan.long_rows && ix->L <= 16) { PEOS_LAUNCH_LONG(16) }
    else if (plan.long_rows) { PEOS_LAUNCH_LONG(32) }
    else if (ix->L <= 16) { PEOS_LAUNCH(16) }
    else { PEOS_LAUNCH(32) }
#undef PEOS_LAUNCH
#undef PEOS_LAUNCH2
#undef PEOS_LAUNCH_LONG
    HIP_TRY(hipGetLastError());
    return PEOS_OK;
}

static int search_impl(const peos_index* ix, const float* queries, const float* tables,
                       const float* qnorms, int64_t nq, const int32_t* k, const int32_t* ef,
                       int32_t k_all, int32_t ef_all, int32_t kstride, int32_t pool, float eps,
                       int32_t mode, int64_t* ids, float* dists, int32_t* stats, void* ws,
                       size_t ws_bytes, hipStream_t s, int slots_cap = 0, int64_t ws_slots = 0)
{
    const int efmax = ef_all > k_all ? ef_all : k_all;
    WsLayout w = ws_layout(ix, nq, spill_words_of(ix), ws_slots);
    // a launch never has more resident workgroups than visited bitmaps
    if (slots_cap <= 0 || slots_cap > w.slots) slots_cap = (int)w.slots;
    if ((int64_t)ws_bytes < w.total) return fail(PEOS_ENOSPACE, "ws_bytes %zu < %lld", ws_bytes, (long long)w.total);
    int rc = ensure_kernel_attrs(ix->device);
    if (rc) return rc;
    peos::SearchArgs a;
    a.base = ix->base;
    a.base16 = ix->base16;
    a.graph = ix->graph;
    a.rec = ix->rec;
    a.node_stride = (int32_t)ix->node_stride;
    a.codes_off = (int32_t)ix->codes_off;
    a.scal_off = (int32_t)ix->scal_off;
    a.sig_off = (int32_t)ix->sig_off;
    a.aux = ix->sdirs;
    a.queries = queries;
    a.tables = tables;
    a.qnorms = qnorms;
    a.kq = k;
    a.efq = ef;
    a.qperm = nullptr;
    a.qrange = nullptr;
    a.ids = ids;
    a.dists = dists;
    a.stats = stats;
    a.entries = nullptr;
    a.counter = nullptr;
    a.spill = (uint32_t*)((char*)ws + w.spill_off);
    a.spill_words = 0;
    a.spill_bitmap_words = 0;
    a.spill_list_cap = 0;
    a.n = (int32_t)ix->n;
    a.nq = (int32_t)nq;
    a.k_all = k_all;
    a.ef_all = ef_all;
    a.kstride = kstride;
    a.d = ix->d;
    a.R = ix->R;
    a.L = ix->L;
    a.m = ix->m;
    a.metric = ix->metric;
    a.mode = mode;
    a.entry = ix->entry;
    const double eta = std::sqrt(2.0 * ix->L * std::log((double)ix->m));
    a.eta = (float)eta;
    a.c_eps = (float)norm_ppf((double)eps);
    a.hoeff = mode == PEOS_MODE_SIMHASH ? (float)std::sqrt(64.0 * std::log(1.0 / (double)eps) / 2.0) : 0.f;
    a.kappa = (float)((double)ix->L / (double)(ix->L + 1));
    a.pool = pool;
    uint32_t* counters = (uint32_t*)((char*)ws + w.counter_off);
    const bool per_query = k != nullptr || ef != nullptr;
    const int nclass = ef ? num_classes(efmax) : 1;
    hipLaunchKernelGGL(peos::k_zero_u32, dim3(1), dim3(64), 0, s, counters, peos::kMaxClasses);
    if (ix->up_node) {
        // entry descent through the upper layers: one wave per query
        peos::DescendArgs da;
        da.base = ix->base;
        da.base16 = ix->base16;
        da.queries = queries;
        da.qnorms = qnorms;
        da.node = ix->up_node;
        da.adj = ix->up_adj;
        da.down = ix->up_down;
        da.entries = (int32_t*)((char*)ws + w.entries_off);
        da.stats = stats;
        da.nq = (int32_t)nq;
        da.d = ix->d;
        da.ru = ix->up_ru;
        da.top = ix->up_top;
        da.metric = ix->metric;
        da.max_steps = 1 << 16;
        const unsigned blocks = (unsigned)(nq < 16384 ? nq : 16384);
        const size_t lds = sizeof(float) * (size_t)ix->d + 3 * 64 * sizeof(float);
        if (ix->base16)
            hipLaunchKernelGGL(peos::k_descend<true>, dim3(blocks), dim3(64), lds, s, da);
        else
            hipLaunchKernelGGL(peos::k_descend<false>, dim3(blocks), dim3(64), lds, s, da);
        HIP_TRY(hipGetLastError());
        a.entries = da.entries;
    }
    if ((ix->flags & PEOS_FLAG_COMPACT) && mode == PEOS_MODE_PEOS) {
        float* lut = (float*)((char*)ws + w.lut_off);
        peos::CompactLut t;
        compact_lut(ix->L, eta, norm_ppf((double)eps), t.v);
        hipLaunchKernelGGL(peos::k_store_lut, dim3(1), dim3(peos::kCompactLutBins), 0, s, t, lut);
        HIP_TRY(hipGetLastError());
        a.aux = lut;
    }
    if (nclass == 1) return launch_search(ix, a, nq, efmax, pool, per_query, -1, counters, slots_cap, s);
    // per-query list sizes: one launch per ef class, each with the LDS plan
    // of its own largest list (small lists are not held to the largest one's
    // visited-hash and list capacity), largest class first
    uint32_t* ranges = (uint32_t*)((char*)ws + w.ranges_off);
    int32_t* qperm = (int32_t*)((char*)ws + w.qperm_off);
    hipLaunchKernelGGL(peos::k_classify, dim3(1), dim3(1024), 0, s, k, ef, k_all, ef_all, nq, nclass,
                       qperm, ranges);
    HIP_TRY(hipGetLastError());
    a.qperm = qperm;
    for (int c = nclass - 1; c >= 0; --c) {
        a.qrange = ranges + 2 * c;
        const int ef_c = c == nclass - 1 ? efmax : (32 << c);
        rc = launch_search(ix, a, nq, ef_c, pool, true, c, counters + c, slots_cap, s);
        if (rc) return rc;
    }
    return PEOS_OK;
}

static int check_search_args(const peos_index* ix, const float* queries, int64_t nq, int32_t k_all,
                             int32_t ef_all, int32_t kstride, int32_t pool, float eps, int32_t mode,
                             const int64_t* ids, const float* dists, const void* ws)
{
    if (!ix) return fail(PEOS_EINVAL, "null index");
    if (nq < 0 || nq > 0x7fffffffLL) return fail(PEOS_EINVAL, "nq=%lld", (long long)nq);
    if (k_all < 1 || kstride < k_all) return fail(PEOS_EINVAL, "k_all=%d kstride=%d", k_all, kstride);
    if (ef_all < 1 || ef_all > kMaxEf || k_all > kMaxEf) return fail(PEOS_EINVAL, "ef_all=%d (max %d)", ef_all, kMaxEf);
    if (pool < -16 || pool > 2 * kMaxEf) return fail(PEOS_EINVAL, "pool=%d", pool);
    if (pool < 0 && -pool * ef_all > 2 * kMaxEf) return fail(PEOS_EINVAL, "pool=%d x ef=%d above %d", pool, ef_all, 2 * kMaxEf);
    if (mode != PEOS_MODE_PEOS && mode != PEOS_MODE_EXHAUSTIVE && mode != PEOS_MODE_SIMHASH) return fail(PEOS_EINVAL, "mode=%d", mode);
    if (mode != PEOS_MODE_EXHAUSTIVE && !(eps > 0.f && eps <= 0.5f)) return fail(PEOS_EINVAL, "eps=%g not in (0, 0.5]", (double)eps);
    if (mode == PEOS_MODE_SIMHASH && !(ix->flags & PEOS_FLAG_SIMHASH)) return fail(PEOS_EINVAL, "PEOS_MODE_SIMHASH needs an index built with PEOS_FLAG_SIMHASH");
    if (nq > 0 && (!queries || !ids || !dists || !ws)) return fail(PEOS_EINVAL, "null device pointer");
    if (((uintptr_t)queries & 15u) != 0) return fail(PEOS_EINVAL, "queries must be 16-byte aligned");
    return PEOS_OK;
}

int peos_search_tables(const peos_index* ix, const float* queries, const float* tables,
                       const float* qnorms, int64_t nq, const int32_t* k, const int32_t* ef,
                       int32_t k_all, int32_t ef_all, int32_t kstride, int32_t pool, float eps,
                       int32_t mode, int64_t* ids, float* dists, int32_t* stats, void* ws,
                       size_t ws_bytes, void* stream)
{
    int rc = check_search_args(ix, queries, nq, k_all, ef_all, kstride, pool, eps, mode, ids, dists, ws);
    if (rc) return rc;
    if (nq == 0) return PEOS_OK;
    if (!tables || !qnorms) return fail(PEOS_EINVAL, "null table pointer");
    return search_impl(ix, queries, tables, qnorms, nq, k, ef, k_all, ef_all, kstride, pool, eps,
                       mode, ids, dists, stats, ws, ws_bytes, (hipStream_t)stream);
}

int peos_search(const peos_index* ix, const float* queries, int64_t nq, const int32_t* k,
                const int32_t* ef, int32_t k_all, int32_t ef_all, int32_t kstride, int32_t pool,
                float eps, int32_t mode, int64_t* ids, float* dists, int32_t* stats, void* ws,
                size_t ws_bytes, void* stream)
{
    int rc = check_search_args(ix, queries, nq, k_all, ef_all, kstride, pool, eps, mode, ids, dists, ws);
    if (rc) return rc;
    if (nq == 0) return PEOS_OK;
    WsLayout w = ws_layout(ix, nq, spill_words_of(ix));
    if ((int64_t)ws_bytes < w.total) return fail(PEOS_ENOSPACE, "ws_bytes %zu < %lld", ws_bytes, (long long)w.total);
    float* tables = (float*)((char*)ws + w.tables_off);
    float* qnorms = (float*)((char*)ws + w.qnorm_off);
    rc = peos_query_tables(ix, queries, nq, tables, qnorms, stream);
    if (rc) return rc;
    return search_impl(ix, queries, tables, qnorms, nq, k, ef, k_all, ef_all, kstride, pool, eps,
                       mode, ids, dists, stats, ws, ws_bytes, (hipStream_t)stream);
}

constexpr int kEnergyBlocks = 2048;

}  // extern "C"

// Scratch of peos_search_static: a file-scope device array, one copy per
// device the library runs on (held until the process ends).  Host code never
// uses its name as an address: the device address of each device's copy is
// looked up once, with that device current, and kept (scratch_address).
static constexpr size_t kScratchBytes = size_t(PEOS_STATIC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

int scratch_address(int dev, void** out)
{
    static std::mutex mu;
    static void* addr[64] = {nullptr};
    std::lock_guard<std::mutex> g(mu);
    if (dev < 0 || dev >= 64) return fail(PEOS_EDEVICE, "device index %d", dev);
    if (!addr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(PEOS_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return PEOS_OK;
}

}  // namespace

extern "C" {

int peos_search_static(const peos_index* ix, const float* queries, int64_t nq, const int32_t* k,
                       const int32_t* ef, int32_t k_all, int32_t ef_all, int32_t kstride,
                       int32_t pool, float eps, int32_t mode, int64_t* ids, float* dists,
                       int32_t* stats, void* stream)
{
    // the workspace check of check_search_args is met by the scratch array
    int rc = check_search_args(ix, queries, nq, k_all, ef_all, kstride, pool, eps, mode, ids,
                               dists, (const void*)1);
    if (rc) return rc;
    if (nq == 0) return PEOS_OK;
    int dev;
    rc = check_device(&dev);
    if (rc) return rc;
    if (dev != ix->device) return fail(PEOS_EINVAL, "current device %d is not the index's %d", dev, ix->device);
    void* ws = nullptr;
    rc = scratch_address(dev, &ws);
    if (rc) return rc;
    // as many visited bitmaps (resident workgroups) as the scratch holds
    // after the per-query part, up to what the batch can use
    const int64_t sw = spill_words_of(ix);
    const WsLayout w1 = ws_layout(ix, nq, sw, 1);
    if ((size_t)w1.total > kScratchBytes)
        return fail(PEOS_ENOSPACE, "nq=%lld with n=%lld needs %lld scratch bytes, %zu available",
                    (long long)nq, (long long)ix->n, (long long)w1.total, kScratchBytes);
    int64_t slots = ((int64_t)kScratchBytes - w1.spill_off) / (sw * 4);
    const int64_t most = nq < kMaxSlots ? nq : kMaxSlots;
    if (slots > most) slots = most;
    const WsLayout w = ws_layout(ix, nq, sw, slots);
    float* tables = (float*)((char*)ws + w.tables_off);
    float* qnorms = (float*)((char*)ws + w.qnorm_off);
    rc = peos_query_tables(ix, queries, nq, tables, qnorms, stream);
    if (rc) return rc;
    return search_impl(ix, queries, tables, qnorms, nq, k, ef, k_all, ef_all, kstride, pool, eps,
                       mode, ids, dists, stats, ws, kScratchBytes, (hipStream_t)stream, 0, slots);
}

int peos_probe_gather(const float* rows, int64_t n_rows, int32_t waves, int32_t iters,
                      float* sink, void* stream)
{
    if (!rows || !sink) return fail(PEOS_EINVAL, "null pointer");
    if (n_rows < 1 || waves < 1 || iters < 1) return fail(PEOS_EINVAL, "n_rows=%lld waves=%d iters=%d", (long long)n_rows, waves, iters);
    if (((uintptr_t)rows & 15u) != 0) return fail(PEOS_EINVAL, "rows must be 16-byte aligned");
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipLaunchKernelGGL(peos::k_probe_gather, dim3((unsigned)waves), dim3(64), 0, (hipStream_t)stream,
                       reinterpret_cast<const float4*>(rows), n_rows, iters, sink);
    HIP_TRY(hipGetLastError());
    return PEOS_OK;
}

int peos_dimension_permutation_ws_bytes(int32_t d, size_t* ws_bytes)
{
    if (!ws_bytes || d < 1) return fail(PEOS_EINVAL, "bad arguments");
    *ws_bytes = (size_t)kEnergyBlocks * (size_t)d * sizeof(float);
    return PEOS_OK;
}

int peos_dimension_permutation(const float* base, int64_t n, int32_t d, const int32_t* graph,
                               int32_t R, int32_t L, int32_t* perm, void* ws, size_t ws_bytes,
                               void* stream)
{
    if (!base || !graph || !perm || !ws) return fail(PEOS_EINVAL, "null pointer");
    if (n < 1 || d < 1 || R < 1 || L < 1 || d % L) return fail(PEOS_EINVAL, "n=%lld d=%d R=%d L=%d", (long long)n, d, R, L);
    size_t need = 0;
    peos_dimension_permutation_ws_bytes(d, &need);
    if (ws_bytes < need) return fail(PEOS_ENOSPACE, "ws_bytes %zu < %zu", ws_bytes, need);
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int blocks = (int)(n < kEnergyBlocks ? n : kEnergyBlocks);
    hipLaunchKernelGGL(peos::k_edge_energy, dim3(blocks), dim3(256), 0, s, base, graph, n, d, R,
                       (float*)ws);
    HIP_TRY(hipGetLastError());
    std::vector<float> part((size_t)blocks * d);
    HIP_TRY(hipMemcpyAsync(part.data(), ws, part.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // per-dimension energy (the common 1/|E| factor changes no decision)
    std::vector<double> avg((size_t)d, 0.0);
    for (int b = 0; b < blocks; ++b)
        for (int j = 0; j < d; ++j) avg[j] += (double)part[(size_t)b * d + j];
    // ascending energy, ties by index; d/L rounds of L, each dimension to
    // the subspace with the largest running sum not yet served this round
    std::vector<int> order((size_t)d);
    for (int j = 0; j < d; ++j) order[j] = j;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return avg[x] < avg[y]; });
    const int dp = d / L;
    std::vector<double> sum((size_t)L, 0.0);
    std::vector<int> fill((size_t)L, 0);
    for (int round = 0; round < dp; ++round) {
        std::vector<char> served((size_t)L, 0);
        for (int j = 0; j < L; ++j) {
            const int dim = order[(size_t)round * L + j];
            int best = -1;
            for (int i = 0; i < L; ++i)
                if (!served[i] && (best < 0 || sum[i] > sum[best])) best = i;
            served[best] = 1;
            sum[best] += avg[dim];
            perm[(size_t)best * dp + fill[best]++] = dim;
        }
    }
    return PEOS_OK;
}

int peos_graph_create(const peos_index* ix, const float* queries, int64_t nq, const int32_t* k,
                      const int32_t* ef, int32_t k_all, int32_t ef_all, int32_t kstride,
                      int32_t pool, float eps, int32_t mode, int64_t* ids, float* dists,
                      int32_t* stats, void* ws, size_t ws_bytes, peos_graph** out)
{
    if (!out) return fail(PEOS_EINVAL, "null output handle");
    *out = nullptr;
    int rc = check_search_args(ix, queries, nq, k_all, ef_all, kstride, pool, eps, mode, ids, dists, ws);
    if (rc) return rc;
    if (nq == 0) return fail(PEOS_EINVAL, "nq = 0: nothing to capture");
    WsLayout w = ws_layout(ix, nq, spill_words_of(ix));
    if ((int64_t)ws_bytes < w.total) return fail(PEOS_ENOSPACE, "ws_bytes %zu < %lld", ws_bytes, (long long)w.total);
    rc = ensure_kernel_attrs(ix->device);
    if (rc) return rc;
    hipStream_t cs;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = peos_search(ix, queries, nq, k, ef, k_all, ef_all, kstride, pool, eps, mode, ids, dists,
                         stats, ws, ws_bytes, cs);
        e = hipStreamEndCapture(cs, &g);
    }
    (void)hipStreamDestroy(cs);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(PEOS_EHIP, "stream capture: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(PEOS_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    peos_graph* pg = new (std::nothrow) peos_graph;
    if (!pg) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(PEOS_EINVAL, "out of host memory");
    }
    pg->graph = g;
    pg->exec = x;
    pg->device = ix->device;
    *out = pg;
    return PEOS_OK;
}

int peos_graph_launch(peos_graph* g, void* stream)
{
    if (!g) return fail(PEOS_EINVAL, "null graph");
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return PEOS_OK;
}

void peos_graph_destroy(peos_graph* g)
{
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"

#include "peos_serve.hpp"
