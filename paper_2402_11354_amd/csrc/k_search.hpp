// Graph search with the PEOs routing test (Alg. 1 with Alg. 2 as RoutingTest).
//
// One wavefront per query; the grid is persistent and pulls query indices
// from an atomic counter.  Per query, in LDS:
//   qv    the query vector;
//   tab   its projection table (step (5)), sign-duplicated: row i holds
//         T_i[j] at j and -T_i[j] at m + j, so a code byte indexes it directly;
//   list  the candidate list, sorted by (distance, id): its first ef entries
//         are the result list R, entries beyond are nodes of the priority
//         queue P that were pushed out of R before being expanded.  Ids carry
//         an "expanded" bit.  Popping P = the first unexpanded entry;
//   hash  the visited set (open addressing), moved to a per-slot bitmap in
//         HBM if it fills up.
// Per expansion of v (delta read once, before the neighbours are tested):
//   lane j < R loads neighbour id j of v and, when R is full and the test is
//   on, edge j's L+1 code bytes and four scalars (all three loads depend on v
//   only, so they are issued together, the id first); visited filter;
//   routing test of step (6); survivors are marked visited and their vectors
//   gathered by groups of lanes (64/ns... lanes per vector, so every
//   survivor's load is in flight at once); survivors closer than delta (or
//   all, while R is not full) are merged into the list.
#pragma once

#include "peos_device.hpp"

namespace peos {

// precision-form flags (the index flags): bfloat16 traversal copy of the
// base; halves for the edge scalars and the projection tables
constexpr int kFlagBf16Base = 1;
constexpr int kFlagFp16 = 2;
constexpr int kFlagCompact = 8;
// launch variant, not an index flag: long vectors at low occupancy (at most
// two waves per SIMD, so a wave has the registers for 2 x 16 rows in flight)
constexpr int kVariantLong = 16;
// Fourth dword of a raw buffer resource on CDNA: data format 32 bits (a
// resource with no data format reads zeros), no swizzle, no index stride.
constexpr int kBufferRsrcWord3 = 0x00020000;
constexpr int kCompactLutBins = 256;

struct SearchArgs {
    const float* base;
    const uint16_t* base16;  // bfloat16 copy of the base (kFlagBf16Base)
    const int32_t* graph;
    const uint8_t* rec;
    int32_t node_stride, codes_off, scal_off, sig_off;  // bytes (records < 2 GB apart)
    const float* aux;       // SimHash mode: 64 x d sign vectors; compact
                            // records: the quantile table (kCompactLutBins)
    const float* queries;
    const float* tables;
    const float* qnorms;
    const int32_t* kq;
    const int32_t* efq;
    const int32_t* qperm;   // optional: query order (a class of the batch)
    const uint32_t* qrange; // with qperm: {begin, end} of this launch's part
    int64_t* ids;
    float* dists;
    int32_t* stats;
    uint32_t* counter;  // work counter, zero before launch
    uint32_t* spill;    // per slot: visited bitmap, then the list of ids set after a spill
    const int32_t* entries;  // per-query entry nodes (upper-layer descent), or null
    int32_t spill_words;         // per-slot stride of spill
    int32_t spill_bitmap_words;  // bitmap words (n bits, whole 16-byte blocks)
    int32_t spill_list_cap;      // ids the list holds (0: no list)
    int32_t n, nq;      // both below 2^31
    int k_all, ef_all, kstride;
    int d, R, L, m, metric, mode, entry;
    float eta, c_eps, kappa, hoeff;
    int listcap, listslack, pool, hcap, visit_limit;
};

constexpr int kNumStats = 14;
constexpr int kStatusZeroQuery = 1;
constexpr int kStatusPoolFull = 2;
constexpr int kStatusSpill = 4;

// visited set: buckets of four slots (one 16-byte LDS read each) over
// cap/4 buckets, two candidate buckets per key (two multiplicative hashes
// scaled to [0, cap/4)).  An insert takes the candidate with more free
// slots; only when both are full does it go to the first bucket after the
// first candidate that has room (linear probing).  Buckets fill front to back
// and nothing is ever removed, so a lookup that finds a free slot in either
// candidate is done, and otherwise scans on from the first candidate to the
// first bucket with a free slot.  A lookup is one round of two parallel reads
// unless both candidates are full, which two choices keep rare at the loads
// the search allows (no long chains as with one choice).
__device__ __forceinline__ uint32_t hash_bucket(uint32_t u, uint32_t nb)
{
    return (uint32_t)(((uint64_t)(u * 0x9E3779B1u) * nb) >> 32);
}

__device__ __forceinline__ uint32_t hash_bucket2(uint32_t u, uint32_t nb)
{
    return (uint32_t)(((uint64_t)((u ^ (u >> 15)) * 0x85EBCA6Bu) * nb) >> 32);
}

__device__ __forceinline__ int free_slots(uint4 k)
{
    return (k.x == kEmpty) + (k.y == kEmpty) + (k.z == kEmpty) + (k.w == kEmpty);
}

__device__ __forceinline__ bool has_key(uint4 k, uint32_t u)
{
    return k.x == u || k.y == u || k.z == u || k.w == u;
}

__device__ __forceinline__ bool hash_lookup(const uint32_t* h, uint32_t cap, uint32_t u)
{
    const uint32_t nb = cap >> 2;
    const uint32_t b1 = hash_bucket(u, nb), b2 = hash_bucket2(u, nb);
    const uint4 k1 = reinterpret_cast<const uint4*>(h)[b1];
    const uint4 k2 = reinterpret_cast<const uint4*>(h)[b2];
    if (has_key(k1, u) || has_key(k2, u)) return true;
    if (k1.w == kEmpty || k2.w == kEmpty) return false;
    // both candidates full: the overflow scan from the first candidate
    uint32_t b = b1;
    for (;;) {
        b = (b + 1u == nb) ? 0u : b + 1u;
        const uint4 k = reinterpret_cast<const uint4*>(h)[b];
        if (has_key(k, u)) return true;
        if (k.w == kEmpty) return false;
    }
}

__device__ __forceinline__ void hash_insert(uint32_t* h, uint32_t cap, uint32_t u)
{
    const uint32_t nb = cap >> 2;
    const uint32_t b1 = hash_bucket(u, nb), b2 = hash_bucket2(u, nb);
    for (;;) {
        const uint4 k1 = reinterpret_cast<const uint4*>(h)[b1];
        const uint4 k2 = reinterpret_cast<const uint4*>(h)[b2];
        if (has_key(k1, u) || has_key(k2, u)) return;
        const int f1 = free_slots(k1), f2 = free_slots(k2);
        uint32_t b;
        uint4 k;
        if (f1 == 0 && f2 == 0) {
            // overflow: the first bucket after b1 with room
            b = b1;
            for (;;) {
                b = (b + 1u == nb) ? 0u : b + 1u;
                k = reinterpret_cast<const uint4*>(h)[b];
                if (has_key(k, u)) return;
                if (k.w == kEmpty) break;
            }
        } else if (f2 > f1) {
            b = b2;
            k = k2;
        } else {
            b = b1;
            k = k1;
        }
        const int e = k.x == kEmpty ? 0 : k.y == kEmpty ? 1 : k.z == kEmpty ? 2 : 3;
        const uint32_t prev = atomicCAS(&h[4 * b + e], kEmpty, u);
        if (prev == kEmpty || prev == u) return;
        // another lane took the slot: read the candidates again
    }
}

__device__ __forceinline__ bool bitmap_test(const uint32_t* bm, uint32_t u)
{
    const uint32_t w = __hip_atomic_load(bm + (u >> 5), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return (w >> (u & 31u)) & 1u;
}

// Exact distances of ns vectors (ids in Su) to the query, G lanes per vector
// (G = 1, 2, 4, 8 or 16).  Every G gives bit-identical results: the d
// coordinates are read in float4 chunks, chunk c belongs to segment c mod 16,
// each segment is an fma chain over its chunks in increasing c, and the 16
// segment sums are added in one fixed binary tree ((0+1), (2+3), ...; then
// pairs of those; ...).  Lane s of a group owns segments s, s+G, ...; the
// tree levels that pair segments of different lanes are xor shuffles (an add
// is commutative, so both partners get the same bits), the remaining levels
// are local.  Angular distance = fma(-sum, 1/|q|, 1).
// one chunk (four coordinates) of a stored vector, as floats
template <bool BF>
struct Chunk;
template <>
struct Chunk<false> {
    typedef float4 raw;
    static __device__ __forceinline__ float4 get(raw v) { return v; }
};
template <>
struct Chunk<true> {
    typedef uint2 raw;  // four bfloat16
    static __device__ __forceinline__ float4 get(raw v)
    {
        return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u),
                           __uint_as_float(v.y << 16), __uint_as_float(v.y & 0xffff0000u));
    }
};

// CLAMP: every lane issues all its loads (an idle slot reads row 0, a chunk
// past the row re-reads the last one) and discards the extra terms with a
// select, so the loads are straight-line code the compiler keeps in flight
// together (with exec-masked loads it waits for each before the next).
template <int G, int PER, int K, bool BF, bool CLAMP = false>
__device__ __forceinline__ void gather_distances(const void* base, int d, const uint32_t* Su, int ns,
                                                 const float* qv, int metric, float inv_qn,
                                                 float* Sdist)
{
#pragma clang fp contract(off)
    typedef typename Chunk<BF>::raw raw;
    constexpr int NP = 16 / G;        // segments per lane
    constexpr int SPR = kWave / G;    // vectors per pass of the wave, per slot
    static_assert(K % NP == 0, "a load step must cover whole segment rounds");
    const int lane = lane_id();
    const int t = lane / G;
    const int s = lane % G;
    const int nch = d >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(qv);
    // lane s of a group reads chunks c = s + G*k, k = 0, 1, ...; chunk number
    // k of the lane belongs to its segment k mod NP, so each segment still
    // sums its chunks in increasing c.  K loads per vector are issued before
    // any of them is used.
    for (int b0 = 0; b0 < ns; b0 += SPR * PER) {
        float part[PER][NP];
        const raw* x4[PER];
        bool act[PER];
#pragma unroll
        for (int pp = 0; pp < PER; ++pp) {
            const int idx = b0 + t + pp * SPR;
            act[pp] = idx < ns;
            x4[pp] = reinterpret_cast<const raw*>(base) + (int64_t)(act[pp] ? Su[idx] : 0u) * (d >> 2);
#pragma unroll
            for (int j = 0; j < NP; ++j) part[pp][j] = 0.f;
        }
        for (int k0 = 0; (CLAMP ? 0 : s) + G * k0 < nch; k0 += K) {
            raw xv[PER][K];
#pragma unroll
            for (int pp = 0; pp < PER; ++pp)
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int c = s + G * (k0 + kk);
                    if (CLAMP) xv[pp][kk] = x4[pp][c < nch ? c : nch - 1];
                    else if (act[pp] && c < nch) xv[pp][kk] = x4[pp][c];
                }
#pragma unroll
            for (int pp = 0; pp < PER; ++pp)
#pragma unroll
                for (int kk = 0; kk < K; ++kk) {
                    const int c = s + G * (k0 + kk);
                    const bool ok = act[pp] && c < nch;
                    if (CLAMP || ok) {
                        const float4 x = Chunk<BF>::get(xv[pp][kk]);
                        const float4 q = q4[CLAMP ? (c < nch ? c : nch - 1) : c];
                        float acc = part[pp][kk % NP];
                        if (metric == 0) {
                            const float t0 = x.x - q.x, t1 = x.y - q.y, t2 = x.z - q.z, t3 = x.w - q.w;
                            acc = fmaf(t0, t0, acc);
                            acc = fmaf(t1, t1, acc);
                            acc = fmaf(t2, t2, acc);
                            acc = fmaf(t3, t3, acc);
                        } else {
                            acc = fmaf(x.x, q.x, acc);
                            acc = fmaf(x.y, q.y, acc);
                            acc = fmaf(x.z, q.z, acc);
                            acc = fmaf(x.w, q.w, acc);
                        }
                        part[pp][kk % NP] = (CLAMP && !ok) ? part[pp][kk % NP] : acc;
                    }
                }
        }
#pragma unroll
        for (int pp = 0; pp < PER; ++pp) {
            // tree levels across lanes (segment index bits below log2 G)
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                if (G > 1) part[pp][j] = part[pp][j] + xor_lane<1>(part[pp][j]);
                if (G > 2) part[pp][j] = part[pp][j] + xor_lane<2>(part[pp][j]);
                if (G > 4) part[pp][j] = part[pp][j] + xor_lane<4>(part[pp][j]);
                if (G > 8) part[pp][j] = part[pp][j] + xor_lane<8>(part[pp][j]);
            }
            // remaining levels inside the lane
#pragma unroll
            for (int h = 1; h < NP; h <<= 1)
#pragma unroll
                for (int j = 0; j < NP; j += 2 * h) part[pp][j] = part[pp][j] + part[pp][j + h];
            const int idx = b0 + t + pp * SPR;
            if (act[pp] && s == 0)
                Sdist[idx] = (metric == 0) ? part[pp][0]
                           : (metric == 2) ? -part[pp][0] : fmaf(-part[pp][0], inv_qn, 1.f);
        }
    }
}

template <bool BF, bool WIDE = false, bool LONG = false>
__device__ __forceinline__ void distances(const void* base, int d, const uint32_t* Su, int ns,
                                          const float* qv, int metric, float inv_qn, float* Sdist)
{
    // 4..16 lanes per vector; each lane keeps at most 8 chunk loads in
    // flight: one round trip for up to 4 vectors of 256 coordinates (16
    // lanes x 4 chunks; not 8 chunks, whose second half a row of up to 256
    // coordinates only re-reads and discards: 1.4% faster at d = 128), 8 of
    // 256 (8 lanes x 8) or 16 of 128 (4 lanes x 8).  The chunk-to-segment
    // map (chunk c to segment c mod 16) and the add tree do not depend on
    // the lanes per vector or the loads per lane.
    // Long bfloat16 vectors: 16 lanes x 16 chunks (8 bytes each) cover up to
    // 1024 coordinates in one round trip per 4 vectors.  The low-occupancy
    // variant keeps two such rows per lane group in flight: one round trip
    // per 8 vectors of up to 1024 coordinates, fp32 or bfloat16 (it is
    // only launched for d > 512, and is correct for any d).
    if (LONG) {
        gather_distances<16, 2, 16, BF, true>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
        return;
    }
    if (WIDE && d > 512) {
        gather_distances<16, 1, 16, BF>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
        return;
    }
    if (ns <= 4) gather_distances<16, 1, 4, BF, true>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
    else if (ns <= 8) gather_distances<8, 1, 8, BF, true>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
    else if (ns <= 16) gather_distances<4, 1, 8, BF, true>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
    else gather_distances<4, 2, 4, BF, true>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
}

#ifndef PEOS_SEARCH_WAVES_PER_EU
#define PEOS_SEARCH_WAVES_PER_EU 4
#endif

// Waves per query.  A workgroup of W = blockDim.x / 64 wavefronts searches
// one query: wave 0 (the leader) runs the whole search; waves 1..W-1 (the
// helpers) only gather survivor rows.  At each gather of ns >= 2 rows the
// leader posts the count in LDS and the workgroup meets at a barrier; wave w
// then computes the distances of rows [w c, (w+1) c), c = ceil(ns / W), and
// the workgroup meets again.  Every row is still reduced by one lane group of
// one wave in the fixed order, so results do not depend on W; what W buys is
// W times the row loads in flight per query, for batches too small to fill
// the chip with one wave per query.
constexpr int kMaxWavesPerQuery = 4;
enum CoopOp : uint32_t { kCoopExit = 0, kCoopTraversal = 1, kCoopFull = 2 };

// the leader's gather: alone (W = 1 or a single row), or split over the
// workgroup.  op selects the rows the helpers read (traversal copy or the
// full-precision base).
template <bool BF, bool WIDE, bool LONG>
__device__ __forceinline__ void lead_distances(int nw, uint32_t* coop, const void* base, int d,
                                               const uint32_t* Su, int ns, const float* qv,
                                               int metric, float inv_qn, float* Sdist, uint32_t op)
{
    if (nw == 1 || ns < 2) {
        distances<BF, WIDE, LONG>(base, d, Su, ns, qv, metric, inv_qn, Sdist);
        return;
    }
    if (lane_id() == 0) {
        coop[0] = op;
        coop[1] = (uint32_t)ns;
        coop[2] = __float_as_uint(inv_qn);
    }
    __syncthreads();  // rows posted
    const int c = (ns + nw - 1) / nw;
    distances<BF, WIDE, LONG>(base, d, Su, ns < c ? ns : c, qv, metric, inv_qn, Sdist);
    __syncthreads();  // every wave's distances are in Sdist
}

// N consecutive dwords at byte offset off of a buffer, in loads of up to 16
// bytes (zeros where the range ends)
template <int N>
__device__ __forceinline__ void load_words(__amdgpu_buffer_rsrc_t rs, int off, uint32_t* w)
{
    int i = 0;
#pragma unroll
    for (; i + 4 <= N; i += 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off + 4 * i, 0, 0);
        w[i] = v[0]; w[i + 1] = v[1]; w[i + 2] = v[2]; w[i + 3] = v[3];
    }
    if constexpr (N % 4 == 3) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, off + 4 * i, 0, 0);
        w[i] = v[0]; w[i + 1] = v[1]; w[i + 2] = v[2];
    } else if constexpr (N % 4 == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off + 4 * i, 0, 0);
        w[i] = v[0]; w[i + 1] = v[1];
    } else if constexpr (N % 4 == 1) {
        w[i] = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 4 * i, 0, 0);
    }
}

// REGL: the candidate list is the result list alone (capacity = ef <= 64,
// the HNSW stopping rule): entry i lives in lane i's registers (rd, ri), so
// the pop is a ballot and the merge a register scatter through LDS staging.
template <int MAXL, int FLAGS, bool REGL>
__global__ __launch_bounds__(kMaxWavesPerQuery * 64,
                             (FLAGS & kVariantLong) ? 2 : PEOS_SEARCH_WAVES_PER_EU) void k_search(
    SearchArgs a)
{
    constexpr bool LONG = (FLAGS & kVariantLong) != 0;
    constexpr bool BF = (FLAGS & kFlagBf16Base) != 0;
    constexpr bool H16 = (FLAGS & kFlagFp16) != 0;
    constexpr bool CP = (FLAGS & kFlagCompact) != 0;
    const void* tbase = BF ? (const void*)a.base16 : (const void*)a.base;
    extern __shared__ __align__(16) unsigned char sm[];
    const int lane = lane_id();
    const int nw = wave_uniform((int)(blockDim.x >> 6));   // waves per query
    const int wv = wave_uniform((int)(threadIdx.x >> 6));  // this wave's rank
    // The arguments used once per query live in LDS and are read where they
    // are used, so they do not hold scalar registers across the expansion
    // loop (which would otherwise spill).
    __shared__ SearchArgs ca;
    __shared__ uint32_t coop[4];  // the leader's posted gather: op, rows, 1/|q|
    if (wv == 0) {
        for (int t = lane; t < (int)(sizeof(SearchArgs) / 4); t += kWave)
            reinterpret_cast<uint32_t*>(&ca)[t] = reinterpret_cast<const uint32_t*>(&a)[t];
    }
    wave_sync();
    if (nw > 1) {
        __syncthreads();
        if (wv > 0) {
            // helper: gather this wave's share of each posted set of rows
            // until the leader posts the exit
            uint32_t* Su_h = reinterpret_cast<uint32_t*>(sm);
            float* Sd_h = reinterpret_cast<float*>(Su_h + kWave);
            const float* qv_h = Sd_h + kWave;
            for (;;) {
                __syncthreads();  // rows posted
                const uint32_t op = coop[0];
                if (op == kCoopExit) break;
                const int ns = (int)coop[1];
                const float inv_qn = __uint_as_float(coop[2]);
                const int c = (ns + nw - 1) / nw;
                const int b = wv * c;
                const int e = ns < b + c ? ns : b + c;
                if (b < e) {
                    if (op == kCoopTraversal)
                        distances<BF, (MAXL >= 16) && BF, LONG>(tbase, a.d, Su_h + b, e - b, qv_h,
                                                                 a.metric, inv_qn, Sd_h + b);
                    else
                        distances<false, false, LONG>(a.base, a.d, Su_h + b, e - b, qv_h, a.metric,
                                                      inv_qn, Sd_h + b);
                }
                __syncthreads();  // distances in Sdist
            }
            return;
        }
    }
    const int d = a.d, R = a.R, L = a.L, m = a.m;
    const int hcap = a.hcap;
    const int slack = wave_uniform(ca.listslack);  // room past the capacity during a merge
    const int listcap = wave_uniform(ca.listcap);
    // survivor staging and the query first, at fixed offsets (no registers
    // hold their addresses), then table | list | visited hash
    uint32_t* Su = reinterpret_cast<uint32_t*>(sm);
    float* Sdist = reinterpret_cast<float*>(Su + kWave);
    float* qv = Sdist + kWave;
    float* tab = qv + d;
    // table: entry (i, c) of code byte c in subspace i at c (MAXL+1) + i,
    // both signs stored (2m codes), zero for L < i <= MAXL
    constexpr int TW = MAXL + 1;
    // the list in LDS (none when it lives in registers: the output then
    // stages it in the visited hash, which is dead by then)
    const int lds_list = REGL ? 0 : listcap + slack;
    float* Lr = tab + 2 * m * TW;
    uint32_t* hash = reinterpret_cast<uint32_t*>(Lr) + 2 * lds_list;
    float* Ld = REGL ? reinterpret_cast<float*>(hash) : Lr;
    uint32_t* Li = REGL ? hash + kWave : reinterpret_cast<uint32_t*>(Lr) + lds_list;
    uint32_t* bitmap = a.spill + (int64_t)blockIdx.x * a.spill_words;
    // The bitmap is cleared whole when this workgroup first spills; after
    // that a spilled query lists the ids it sets past the hash's and clears
    // just their words when it ends, so the next spill finds it clear (the
    // whole clear writes n/8 bytes, which at 10M nodes costs more than the
    // query's search).  A query that overflows the list leaves it unknown.
    uint32_t* slist = bitmap + a.spill_bitmap_words;
    bool bm_unknown = true;

    uint32_t qbegin = 0, qend = wave_uniform((uint32_t)ca.nq);
    if (ca.qperm) {
        qbegin = wave_uniform(ca.qrange[0]);
        qend = wave_uniform(ca.qrange[1]);
    }
    for (;;) {
        uint32_t qtaken = 0;
        if (lane == 0) qtaken = atomicAdd(ca.counter, 1u);
        const uint32_t slot = wave_uniform((uint32_t)__shfl((int)qtaken, 0, kWave)) + qbegin;
        if (slot >= qend) {
            if (nw > 1) {
                // release the helpers
                if (lane == 0) coop[0] = kCoopExit;
                __syncthreads();
            }
            break;
        }
        const int64_t qi = ca.qperm ? (int64_t)wave_uniform(ca.qperm[slot]) : (int64_t)slot;

        // per-query k and ef are clamped to the launch bounds k_all, ef_all
        const int k_all = wave_uniform(ca.k_all), ef_all = wave_uniform(ca.ef_all);
        const int pool = wave_uniform(ca.pool);
        int kq = ca.kq ? wave_uniform(ca.kq[qi]) : k_all;
        kq = kq < 1 ? 1 : (kq > k_all ? k_all : kq);
        int efq = ca.efq ? wave_uniform(ca.efq[qi]) : ef_all;
        efq = efq > ef_all ? ef_all : efq;
        efq = efq > kq ? efq : kq;
        // list capacity: pool > 0 a fixed capacity (at least ef), pool < 0
        // |pool| times this query's ef, 0 the kernel's (the unbounded queue)
        int cap = pool > 0 ? (pool > efq ? pool : efq) : (pool < 0 ? -pool * efq : listcap);
        cap = cap < listcap ? cap : listcap;
        if (REGL) cap = cap < kWave ? cap : kWave;
        const float qn = wave_uniform(ca.qnorms[qi]);
        int status = 0;
        // wave-uniform counts, and per-lane counts summed over the wave at
        // the end of the query (kept in vector registers: no scalar
        // registers and no ballot per count in the expansion loop)
        int st_exp = 0, st_ndist = 0, st_ins = 0, st_texp = 0;
        int lc_edges = 0, lc_skip = 0, lc_ge1 = 0, lc_le0 = 0, lc_h = 0, lc_zero = 0, lc_pass = 0;
        int size = 0;

        if (qn > 0.f && qn < INFINITY) {
            const float inv_qn = 1.f / qn;
            const float* qg = ca.queries + qi * d;
            for (int t = lane; t < d; t += kWave) qv[t] = qg[t];
            if (H16) {
                const _Float16* tg = reinterpret_cast<const _Float16*>(ca.tables) + qi * (int64_t)(L + 1) * m;
                for (int c = lane; c < 2 * m; c += kWave)
                    for (int i = 0; i < TW; ++i) {
                        const float v = i <= L ? (float)tg[i * m + (c < m ? c : c - m)] : 0.f;
                        tab[c * TW + i] = c < m ? v : -v;
                    }
            } else {
                const float* tg = ca.tables + qi * (int64_t)(L + 1) * m;
                for (int c = lane; c < 2 * m; c += kWave)
                    for (int i = 0; i < TW; ++i) {
                        const float v = i <= L ? tg[i * m + (c < m ? c : c - m)] : 0.f;
                        tab[c * TW + i] = c < m ? v : -v;
                    }
            }
            for (int t = lane; t < hcap; t += kWave) hash[t] = kEmpty;
            // SimHash mode: the query's 64 sign bits, lane i projecting on c_i
            // (an fma chain over the coordinates in order)
            uint64_t qsig = 0;
            if (a.mode == 2) {
                const float* cv = a.aux + (int64_t)lane * d;
                float p = 0.f;
                for (int k = 0; k < d; ++k) p = fmaf(qg[k], cv[k], p);
                qsig = ballot(p >= 0.f);
            }
            const uint32_t v0 = (uint32_t)wave_uniform(ca.entries ? ca.entries[qi] : ca.entry);
            if (lane == 0) Su[0] = v0;
            wave_sync();
            distances<BF, (MAXL >= 16) && BF>(tbase, d, Su, 1, qv, a.metric, inv_qn, Sdist);
            if (lane == 0) {
                hash_insert(hash, (uint32_t)hcap, v0);
            }
            wave_sync();
            // list entry `lane` (REGL)
            float rd = INFINITY;
            uint32_t ri = 0u;
            if (REGL) {
                if (lane == 0) {
                    rd = Sdist[0];
                    ri = v0;
                }
            } else if (lane == 0) {
                Ld[0] = Sdist[0];
                Li[0] = v0;
            }
            size = 1;
            int nvis = 1;
            bool spilled = false;
            int nlist = 0;  // ids set in the bitmap after the spill
            st_ndist = 1;
            int lb = 0;  // every entry before lb is expanded
            wave_sync();

            constexpr int NCW = (MAXL + 4) / 4;  // code dwords per edge (max)
            for (;;) {
                // pop: first unexpanded entry of the list
                int pos = -1;
                uint32_t vid;
                float dv, delta;
                const bool full = size >= efq;
                if (REGL) {
                    const uint64_t mk = ballot(lane < size && !(ri & kExpanded));
                    if (!mk) break;
                    pos = __ffsll((unsigned long long)mk) - 1;
                    vid = (uint32_t)__builtin_amdgcn_readlane((int)ri, pos) & kIdMask;
                    dv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rd), pos));
                    delta = full ? __int_as_float(__builtin_amdgcn_readlane(__float_as_int(rd), efq - 1))
                                 : INFINITY;
                    if (lane == pos) ri |= kExpanded;
                } else {
                    for (int c0 = lb; c0 < size; c0 += kWave) {
                        const int p = c0 + lane;
                        const uint64_t mk = ballot(p < size && !(Li[p] & kExpanded));
                        if (mk) {
                            pos = c0 + __ffsll((unsigned long long)mk) - 1;
                            break;
                        }
                    }
                    if (pos < 0) break;
                    lb = pos + 1;
                    vid = wave_uniform(Li[pos] & kIdMask);
                    dv = Ld[pos];
                    delta = full ? Ld[efq - 1] : INFINITY;
                    wave_sync();
                    if (lane == 0) Li[pos] = vid | kExpanded;
                }
                ++st_exp;
                const bool testing = (a.mode == 0 || a.mode == 2) && full;
                st_texp += testing ? 1 : 0;

                // ids, codes and scalars depend on v only: one round trip.
                // Every lane issues the same loads in straight-line code, the
                // id first, so that the visited filter waits for the id alone
                // while the record is in flight: lanes past R read edge R-1's
                // again, and the record is read through a buffer resource
                // whose range is the node's record, or empty when the
                // expansion runs no test (out-of-range buffer loads return
                // zero without touching memory).
                const int le = lane < R ? lane : R - 1;
                int32_t u = a.graph[(int64_t)vid * R + le];
                const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                    const_cast<uint8_t*>(a.rec) + (int64_t)vid * a.node_stride, 0,
                    testing ? a.node_stride : 0, kBufferRsrcWord3);
                float4 sc4;
                uint32_t cw[NCW];
                uint32_t csc = 0u;  // compact: the two scalar codes of the edge
                if (CP) {
                    // node header {g_lo, g_step, i_lo, i_step}, 4 code bytes
                    // and 2 scalar bytes of the edge
                    sc4 = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(rs, 0, 0, 0));
                    cw[0] = __builtin_amdgcn_raw_buffer_load_b32(rs, a.codes_off + 4 * le, 0, 0);
#pragma unroll
                    for (int i = 1; i < NCW; ++i) cw[i] = 0u;
                    csc = __builtin_amdgcn_raw_buffer_load_b16(rs, a.scal_off + 2 * le, 0, 0);
                } else {
                    if (H16) {
                        // halves: g_e/|e|, 1/|e|, w_reg, sqrt(L) w_res
                        const uint2 h = __builtin_bit_cast(
                            uint2, __builtin_amdgcn_raw_buffer_load_b64(rs, a.scal_off + 8 * le, 0, 0));
                        sc4 = make_float4((float)__builtin_bit_cast(_Float16, (uint16_t)(h.x & 0xffffu)),
                                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h.x >> 16)),
                                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h.y & 0xffffu)),
                                          (float)__builtin_bit_cast(_Float16, (uint16_t)(h.y >> 16)));
                    } else {
                        sc4 = __builtin_bit_cast(
                            float4, __builtin_amdgcn_raw_buffer_load_b128(rs, a.scal_off + 16 * le, 0, 0));
                    }
                    // the edge's codes, or in SimHash mode its two signature
                    // dwords (the dwords read past them, zero or another
                    // edge's bytes within the record, are cleared): one load
                    // shape for both modes
                    const bool sim = a.mode == 2;
                    const int cb = sim ? a.sig_off + 8 * le : a.codes_off + 4 * NCW * le;
                    load_words<NCW>(rs, cb, cw);  // zero past the codes of L
#pragma unroll
                    for (int i = 2; i < NCW; ++i) cw[i] = sim ? 0u : cw[i];
                }
                if (lane >= R) u = -1;
                const float sg = sc4.x, se = sc4.y, sw = sc4.z, sr = sc4.w;
                const bool valid = u >= 0;
                lc_edges += valid ? 1 : 0;
                bool vis = false;
                if (valid)
                    vis = spilled ? bitmap_test(bitmap, (uint32_t)u)
                                  : hash_lookup(hash, (uint32_t)hcap, (uint32_t)u);
                lc_skip += vis ? 1 : 0;
                const bool cand = valid && !vis;
                bool pass = cand;
                if (testing) {
                    int kind = -1;
                    if (cand && CP) {
                        // compact records: w_reg = 1, w_res = 0, decoded
                        // scalars (A_r a lower bound of the exact one), the
                        // quantile from the table (its bin's smallest T)
                        const float diff = (a.metric == 0) ? 0.5f * (dv - delta) : (dv - delta);
                        const uint32_t ci = csc >> 8;
                        if (ci == 255u) {
                            kind = 0;
                            pass = diff < 0.f;
                        } else {
                            const float gp = (a.metric == 0) ? fmaf((float)(csc & 0xFFu), sc4.y, sc4.x) : 0.f;
                            const float ie = fmaf((float)ci + (diff < 0.f ? 0.5f : -0.5f), sc4.w, sc4.z);
                            const float A = (a.metric != 1) ? fmaf(diff, ie, gp) * inv_qn : diff * ie;
                            if (A >= 1.f) {
                                kind = 1;
                                pass = false;
                            } else if (A <= 0.f) {
                                kind = 2;
                                pass = true;
                            } else {
                                kind = 3;
                                float h = 0.f;
#pragma unroll
                                for (int i = 1; i <= 4; ++i)  // zero entries past L
                                    h += tab[(int)((cw[0] >> ((i - 1) * 8)) & 0xFFu) * TW + i];
                                int b = (int)(A * (float)kCompactLutBins);
                                b = b < kCompactLutBins - 1 ? b : kCompactLutBins - 1;
                                pass = h >= a.aux[b];
                            }
                        }
                    } else if (cand) {
                        // full precision: sg = g_e, se = |e|; halves: sg =
                        // g_e/|e|, se = 1/|e| (infinite for a zero edge).
                        // sg is zero for angular and inner product; the
                        // angular distance already carries the 1/|q|.
                        const float diff = (a.metric == 0) ? 0.5f * (dv - delta) : (dv - delta);
                        const float num = H16 ? diff : ((a.metric == 0) ? sg + diff : diff);
                        const bool zero = H16 ? !(se < INFINITY) : se == 0.f;
                        const float A = H16 ? ((a.metric != 1) ? fmaf(diff, se, sg) * inv_qn : diff * se)
                                            : num * __builtin_amdgcn_rcpf((a.metric != 1 ? qn : 1.f) * se);
                        // zero-length edge: the sign of the numerator; A_r >= 1
                        // fails, A_r <= 0 passes, otherwise H against T
                        const bool ge1 = !zero && A >= 1.f;
                        const bool le0 = !zero && !ge1 && A <= 0.f;
                        kind = zero ? 0 : (ge1 ? 1 : (le0 ? 2 : 3));
                        bool hpass;
                        if (a.mode == 2) {
                            // SimHash: collisions of the 64 sign bits
                            const uint64_t es = ((uint64_t)cw[1 % NCW] << 32) | cw[0];
                            const int col = 64 - popc(es ^ qsig);
                            hpass = kind == 3 &&
                                    (float)col >= 64.f * (1.f - acosf(A) * 0.318309886183790672f) - a.hoeff;
                        } else {
                            // code byte c: direction c mod m, negative iff c >= m;
                            // the LDS table holds both signs, entry (i, c) at
                            // c (MAXL+1) + i (one multiply per lookup, the
                            // subspace in the instruction's offset); entries
                            // past L are zero and the padding codes are 0, so
                            // every lookup is issued without a branch, for
                            // every lane (the few that do not need H discard it)
                            auto signed_entry = [&](int i, uint32_t c) { return tab[(int)c * TW + i]; };
                            float tv[TW];
#pragma unroll
                            for (int i = 0; i <= MAXL; ++i)
                                tv[i] = signed_entry(i, (cw[i >> 2] >> ((i & 3) * 8)) & 0xFFu);
                            float h1 = 0.f;
#pragma unroll
                            for (int i = 1; i <= MAXL; ++i) h1 += tv[i];
                            const float H = sw * h1 + sr * tv[0];
                            const float var = sw * sw + sr * sr - a.kappa * A * A;
                            const float T = A * a.eta + a.c_eps * __builtin_amdgcn_sqrtf(var);
                            hpass = H >= T;
                        }
                        pass = zero ? num < 0.f : (ge1 ? false : (le0 ? true : hpass));
                    }
                    // every tested edge gets exactly one kind
                    lc_zero += kind == 0 ? 1 : 0;
                    lc_ge1 += kind == 1 ? 1 : 0;
                    lc_le0 += kind == 2 ? 1 : 0;
                    lc_h += kind == 3 ? 1 : 0;
                    lc_pass += (cand && pass) ? 1 : 0;
                }
                const uint64_t smask = ballot(pass);
                const int ns = popc(smask);
                if (ns == 0) continue;

                // visited := visited + survivors
                if (!spilled && nvis + ns > a.visit_limit) {
                    if (bm_unknown) {
                        for (int w = lane; w < (a.spill_bitmap_words >> 2); w += kWave)
                            reinterpret_cast<uint4*>(bitmap)[w] = make_uint4(0u, 0u, 0u, 0u);
                        wave_mem_order();
                    }
                    for (int t = lane; t < hcap; t += kWave) {
                        const uint32_t k = hash[t];
                        if (k != kEmpty) atomicOr(bitmap + (k >> 5), 1u << (k & 31u));
                    }
                    wave_mem_order();
                    spilled = true;
                    bm_unknown = true;
                    nlist = 0;
                    status |= kStatusSpill;
                }
                if (pass) {
                    const int t = popc(smask & lanemask_lt());
                    if (spilled) {
                        atomicOr(bitmap + ((uint32_t)u >> 5), 1u << ((uint32_t)u & 31u));
                        if (nlist + t < a.spill_list_cap) slist[nlist + t] = (uint32_t)u;
                    } else {
                        hash_insert(hash, (uint32_t)hcap, (uint32_t)u);
                    }
                    Su[t] = (uint32_t)u;
                }
                if (spilled) nlist += ns;
                nvis += ns;
                wave_sync();
                lead_distances<BF, (MAXL >= 16) && BF, LONG>(nw, coop, tbase, d, Su, ns, qv, a.metric,
                                                             inv_qn, Sdist, kCoopTraversal);
                st_ndist += ns;
                wave_sync();

                // survivors that enter the list stay in their own lanes
                // (lane t = survivor t) with their sort keys in registers
                bool keep = false;
                float dt = 0.f;
                uint32_t ut = 0;
                uint64_t skey = ~0ull;
                if (lane < ns) {
                    dt = Sdist[lane];
                    ut = Su[lane];
                    keep = !full || dt < delta;
                    if (keep) skey = sort_key(dt, ut);
                }
                const uint64_t km = ballot(keep);
                const int nS = popc(km);
                st_ins += nS;
                if (nS == 0) continue;

                if (REGL) {
                    // list entry i (lane i) moves up by the number of
                    // survivors below it; survivor t goes to (survivors below
                    // it) + (list entries below it).  Positions from cap = ef
                    // on are dropped (the launch guarantees cap = ef).
                    const bool inl = lane < size;
                    const uint64_t lk = inl ? sort_key(rd, ri) : ~0ull;
                    int rS = 0, lo = 0, sh = 0;
                    for (uint64_t mm = km; mm; mm &= mm - 1) {
                        const int t = __ffsll((unsigned long long)mm) - 1;
                        const uint64_t kt = readlane64(skey, t);
                        rS += kt < skey;
                        const bool below = inl && lk < kt;
                        sh += (inl && !below) ? 1 : 0;
                        const int nb = popc(ballot(below));
                        lo += (lane == t) ? nb : 0;
                    }
                    const int lpos = lane + sh;
                    const int spos = lo + rS;
                    wave_sync();  // Sdist / Su were read above
                    if (inl && lpos < cap) {
                        Sdist[lpos] = rd;
                        Su[lpos] = ri;
                    }
                    if (keep && spos < cap) {
                        Sdist[spos] = dt;
                        Su[spos] = ut;
                    }
                    const int total = size + nS < cap ? size + nS : cap;
                    wave_sync();
                    rd = lane < total ? Sdist[lane] : INFINITY;
                    ri = lane < total ? Su[lane] : 0u;
                    size = total;
                    wave_sync();
                    continue;
                }

                // merge in place: rank of each survivor among the survivors,
                // number of list entries below it (lo), and for each list
                // entry the number of survivors below it (its shift).  Keys
                // are broadcast from the survivor lanes; chunks of the list
                // move from the back so nothing is overwritten unread.
                int rS = 0;
                for (uint64_t mm = km; mm; mm &= mm - 1) {
                    const int t = __ffsll((unsigned long long)mm) - 1;
                    const uint64_t kt = readlane64(skey, t);
                    rS += kt < skey;
                }
                int lo = 0;
                for (int c0 = ((size - 1) / kWave) * kWave; c0 >= 0; c0 -= kWave) {
                    const int p = c0 + lane;
                    const bool in = p < size;
                    const float dd = in ? Ld[p] : 0.f;
                    const uint32_t id = in ? Li[p] : 0u;
                    const uint64_t lk = in ? sort_key(dd, id) : ~0ull;
                    int sh = 0;
                    for (uint64_t mm = km; mm; mm &= mm - 1) {
                        const int t = __ffsll((unsigned long long)mm) - 1;
                        const uint64_t kt = readlane64(skey, t);
                        const bool below = lk < kt;
                        const int nb = popc(ballot(below));
                        lo += (lane == t) ? nb : 0;
                        sh += (in && !below) ? 1 : 0;
                    }
                    wave_sync();
                    if (in && sh && p + sh < cap + slack) {
                        Ld[p + sh] = dd;
                        Li[p + sh] = id;
                    }
                    wave_sync();
                }
                const int mpos = keep ? lo + rS : 0x7fffffff;
                if (keep && mpos < cap + slack) {
                    Ld[mpos] = dt;
                    Li[mpos] = ut;
                }
                int minpos = mpos;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    const int other = __shfl_xor(minpos, o, kWave);
                    minpos = other < minpos ? other : minpos;
                }
                wave_sync();
                // compaction, front to back: entries beyond ef leave once
                // expanded, and at most cap entries stay (nothing to do when
                // cap = ef: everything beyond is dropped)
                const int total = size + nS;
                int w = efq < total ? efq : total;
                if (cap > efq) {
                    for (int c0 = w; c0 < total; c0 += kWave) {
                        const int p = c0 + lane;
                        const bool vld = p < total;
                        const uint32_t id = vld ? Li[p] : 0u;
                        const float dd = vld ? Ld[p] : 0.f;
                        const bool kp = vld && !(id & kExpanded);
                        const uint64_t kmask = ballot(kp);
                        const int ix = w + popc(kmask & lanemask_lt());
                        wave_sync();
                        if (kp && ix < cap + slack) {
                            Ld[ix] = dd;
                            Li[ix] = id;
                        }
                        wave_sync();
                        w += popc(kmask);
                    }
                } else {
                    w = total;
                }
                if (w > cap && pool == 0) status |= kStatusPoolFull;
                size = w < cap ? w : cap;
                minpos = wave_uniform(minpos);
                lb = lb < efq ? lb : efq;
                lb = lb < minpos ? lb : minpos;
                wave_sync();
            }
            if (spilled && nlist <= a.spill_list_cap) {
                // clear the words this query set: the ids the hash held at
                // the spill (it is unchanged since), then the listed ones
                wave_mem_order();  // the list's stores, before it is read back
                for (int t = lane; t < hcap; t += kWave) {
                    const uint32_t k = hash[t];
                    if (k != kEmpty) bitmap[k >> 5] = 0u;
                }
                for (int i = lane; i < nlist; i += kWave) bitmap[slist[i] >> 5] = 0u;
                wave_mem_order();
                bm_unknown = false;
            }
            if (REGL) {
                // the list to LDS for the output (and the re-rank)
                if (lane < size) {
                    Ld[lane] = rd;
                    Li[lane] = ri;
                }
                wave_sync();
            }
        } else {
            status |= kStatusZeroQuery;
        }

        const int kstride = wave_uniform(ca.kstride);
        if (BF && size > 0) {
            // precision form: the result list (first ef entries) re-ranked by
            // full-precision distances; entry t goes to its rank among them
            const int nr = size < efq ? size : efq;
            const float inv_qn = 1.f / qn;
            for (int c0 = 0; c0 < nr; c0 += kWave) {
                const int cnt = nr - c0 < kWave ? nr - c0 : kWave;
                if (lane < cnt) Su[lane] = Li[c0 + lane] & kIdMask;
                wave_sync();
                lead_distances<false, false, LONG>(nw, coop, a.base, d, Su, cnt, qv, a.metric, inv_qn,
                                                   Sdist, kCoopFull);
                wave_sync();
                if (lane < cnt) Ld[c0 + lane] = Sdist[lane];
                wave_sync();
            }
            for (int t = lane; t < nr; t += kWave) {
                const uint32_t id = Li[t] & kIdMask;
                const uint64_t key = sort_key(Ld[t], id);
                int rank = 0;
                for (int o = 0; o < nr; ++o) rank += sort_key(Ld[o], Li[o] & kIdMask) < key;
                if (rank < kq) {
                    ca.ids[qi * kstride + rank] = (int64_t)id;
                    ca.dists[qi * kstride + rank] = Ld[t];
                }
            }
            const int kout = kq < nr ? kq : nr;
            for (int t = kout + lane; t < kstride; t += kWave) {
                ca.ids[qi * kstride + t] = -1;
                ca.dists[qi * kstride + t] = INFINITY;
            }
        } else {
            // results: first k entries of the list, padded with (-1, +inf)
            for (int t = lane; t < kstride; t += kWave) {
                const bool ok = t < kq && t < size;
                ca.ids[qi * kstride + t] = ok ? (int64_t)(Li[t] & kIdMask) : (int64_t)-1;
                ca.dists[qi * kstride + t] = ok ? Ld[t] : INFINITY;
            }
        }
        const int st_edges = wave_sum_int(lc_edges), st_skip = wave_sum_int(lc_skip);
        const int st_ge1 = wave_sum_int(lc_ge1), st_le0 = wave_sum_int(lc_le0);
        const int st_h = wave_sum_int(lc_h), st_zero = wave_sum_int(lc_zero);
        const int st_pass = wave_sum_int(lc_pass);
        if (ca.stats && lane == 0) {
            int32_t* o = ca.stats + qi * kNumStats;
            o[0] = st_exp;
            o[1] = st_edges;
            o[2] = st_skip;
            o[3] = st_zero + st_ge1 + st_le0 + st_h;
            o[4] = st_ge1;
            o[5] = st_le0;
            o[6] = st_h;
            o[7] = st_zero;
            o[8] = st_pass;
            o[9] = st_ndist;
            o[10] = st_ins;
            o[11] = status;
            if (!ca.entries) o[12] = 0;  // else the descent's count, written before
            o[13] = st_texp;
        }
        wave_sync();
    }
}

// Split a batch with per-query list sizes into classes by effective ef
// (class c holds ef in (32 << (c-1), 32 << c], the last class the rest), as
// a stable counting sort: qperm lists the queries of class 0, then class 1,
// ..., each in query order; ranges[2c], ranges[2c+1] = begin, end of class c.
// One workgroup of 1024 threads.
constexpr int kMaxClasses = 8;

__device__ __forceinline__ int ef_class(int efq, int nclass)
{
    int c = 0;
    while (c < nclass - 1 && efq > (32 << c)) ++c;
    return c;
}

__global__ __launch_bounds__(1024) void k_classify(const int32_t* kq, const int32_t* efq, int k_all,
                                                   int ef_all, int64_t nq, int nclass,
                                                   int32_t* qperm, uint32_t* ranges)
{
    __shared__ uint32_t cnt[kMaxClasses];
    __shared__ uint32_t run[kMaxClasses];
    __shared__ uint32_t wc[16][kMaxClasses];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    auto cls = [&](int64_t i) {
        int k = kq ? kq[i] : k_all;
        k = k < 1 ? 1 : (k > k_all ? k_all : k);
        int e = efq ? efq[i] : ef_all;
        e = e > ef_all ? ef_all : e;
        e = e > k ? e : k;
        return ef_class(e, nclass);
    };
    if (tid < kMaxClasses) cnt[tid] = 0u;
    __syncthreads();
    for (int64_t i = tid; i < nq; i += 1024) atomicAdd(&cnt[cls(i)], 1u);
    __syncthreads();
    if (tid == 0) {
        uint32_t b = 0;
        for (int c = 0; c < kMaxClasses; ++c) {
            run[c] = b;
            ranges[2 * c] = b;
            b += c < nclass ? cnt[c] : 0u;
            ranges[2 * c + 1] = b;
        }
    }
    __syncthreads();
    for (int64_t b0 = 0; b0 < nq; b0 += 1024) {
        const int64_t i = b0 + tid;
        const int c = i < nq ? cls(i) : -1;
        int rank = 0;
        for (int cc = 0; cc < nclass; ++cc) {
            const uint64_t mk = ballot(c == cc);
            if (c == cc) rank = popc(mk & lanemask_lt());
            if (lane == 0) wc[wv][cc] = (uint32_t)popc(mk);
        }
        __syncthreads();
        if (c >= 0) {
            uint32_t off = run[c];
            for (int w = 0; w < wv; ++w) off += wc[w][c];
            qperm[off + rank] = (int32_t)i;
        }
        __syncthreads();
        if (tid < nclass) {
            uint32_t t = 0;
            for (int w = 0; w < 16; ++w) t += wc[w][tid];
            run[tid] += t;
        }
        __syncthreads();
    }
}

// zero the work counter (a kernel rather than a memset, so the sequence can
// be captured in a graph)
__global__ void k_zero_u32(uint32_t* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// The quantile table of the compact form, computed on the host and handed
// to the device as a kernel argument (a kernel node, so a captured search
// carries it), written to the workspace where the search reads it.
struct CompactLut {
    float v[kCompactLutBins];
};

__global__ __launch_bounds__(256) void k_store_lut(CompactLut t, float* lut)
{
    const int b = (int)threadIdx.x;
    if (b < kCompactLutBins) lut[b] = t.v[b];
}

}  // namespace peos
