// PEOs step (5): the projection table of every query, on the matrix cores.
//
// tables[q][i][j] = q'_i . a^i_j (i = 1..L) and tables[q][0][j] = q' . b_j,
// with q' = q/|q| and q'_i its i-th block (Sec. 4.2; the table is built once
// per query, Alg. 2).  As a matrix product this is Q x [B^T | blockdiag(A^i)^T]
// scaled by 1/|q| per row; the block-diagonal structure is kept (each
// subspace contracts over its own d/L coordinates only).
//
// Each 16-query x 16-direction output tile is one chain of
// v_mfma_f32_16x16x4f32 (fp32 in, fp32 accumulate): per K step of 4, lane l
// feeds A[row = l%16][k = l/16] (queries) and B[k = l/16][col = l%16]
// (directions), and receives D[row = 4*(l/16) + r][col = l%16], r = 0..3.
// The precision form stores the table as halves.
#pragma once

#include "peos_device.hpp"

namespace peos {

typedef float floatx4 __attribute__((ext_vector_type(4)));

struct QueryTableArgs {
    const float* queries;  // nq x d
    const float* dirs_a;   // L x m x dp
    const float* dirs_b;   // m x d
    float* tables;         // nq x (L+1) x m floats, or halves when half_out
    float* qnorms;         // nq
    int64_t nq;
    int d, L, m;
    int half_out;          // store the table as IEEE halves (round to nearest even)
    int staged;            // the tile's rows are staged in LDS (16 (d + 4) floats fit)
    const int32_t* perm;   // optional dimension permutation of the test
};

// One workgroup of kTableWaves waves per tile of 16 queries.  The tile's
// query rows are staged in LDS with coalesced 16-byte loads (row stride
// d + 4 floats, so the 16 rows x 4 consecutive k an MFMA step reads fall in
// 64 distinct banks; up to 61 KB at d = 960); the (L+1) x m/16 output tiles
// are dealt out to the waves.  With staged rows and no permutation both
// operands are read 16 bytes per lane: a group of four K steps per load.
constexpr int kTableWaves = 4;

// |q| of this lane's row (lane % 16) from the staged rows:
// sqrt((p0 + p1) + (p2 + p3)), p_j the fma chain of q_k^2 over k = j mod 4
// (one lane each, eight terms read together, then chained), combined by two
// xor shuffles, so that every lane of the row holds the same value.
__device__ __forceinline__ float staged_row_norm(const float* ql, int d, int kq)
{
    float ss = 0.f;
    int k = kq;
    for (; k + 28 < d; k += 32) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = ql[k + 4 * j];
#pragma unroll
        for (int j = 0; j < 8; ++j) ss = fmaf(v[j], v[j], ss);
    }
    for (; k < d; k += 4) ss = fmaf(ql[k], ql[k], ss);
    ss += __shfl_xor(ss, 16, kWave);
    ss += __shfl_xor(ss, 32, kWave);
    return sqrtf(ss);
}

// N consecutive K groups j.. of one tile: all loads first, then the MFMAs
// (straight-line code, so that no load waits behind another's wait)
template <int N>
__device__ __forceinline__ floatx4 mfma_groups(floatx4 acc, const float* av, const float* bv, int j, int k4)
{
    float4 bq[N], aq[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        bq[u] = *reinterpret_cast<const float4*>(bv + 16 * (j + u) + k4);
        aq[u] = *reinterpret_cast<const float4*>(av + 16 * (j + u) + k4);
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].x, bq[u].x, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].y, bq[u].y, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].z, bq[u].z, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].w, bq[u].w, acc, 0, 0, 0);
    }
    return acc;
}

// One round trip for a wave's whole work when it is at most 4 full-space
// groups (N of them, from group g0) and at most 4 subspace tiles of exactly
// one group each (d / L = 16; T tile slots, at least the wave's tiles): every
// load first, then the MFMAs in each accumulator's order.
template <int N, int T>
__device__ __forceinline__ void one_round(floatx4& part, floatx4 (&acc)[4], const float* ql,
                                          const float* brow, int g0, const float* const (&at)[4],
                                          const float* const (&bt)[4], int k4)
{
    float4 bq[N > 0 ? N : 1], aq[N > 0 ? N : 1], tb[T], ta[T];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        bq[u] = *reinterpret_cast<const float4*>(brow + 16 * (g0 + u) + k4);
        aq[u] = *reinterpret_cast<const float4*>(ql + 16 * (g0 + u) + k4);
    }
#pragma unroll
    for (int u = 0; u < T; ++u) {
        tb[u] = *reinterpret_cast<const float4*>(bt[u] + k4);
        ta[u] = *reinterpret_cast<const float4*>(at[u] + k4);
    }
#pragma unroll
    for (int u = 0; u < N; ++u) {
        part = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].x, bq[u].x, part, 0, 0, 0);
        part = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].y, bq[u].y, part, 0, 0, 0);
        part = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].z, bq[u].z, part, 0, 0, 0);
        part = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].w, bq[u].w, part, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < T; ++u) {
        floatx4 c = {0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[u].x, tb[u].x, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[u].y, tb[u].y, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[u].z, tb[u].z, c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_16x16x4f32(ta[u].w, tb[u].w, c, 0, 0, 0);
        acc[u] = c;
    }
}

template <int T>
__device__ __forceinline__ void one_round_n(int n0, floatx4& part, floatx4 (&acc)[4], const float* ql,
                                            const float* brow, int g0, const float* const (&at)[4],
                                            const float* const (&bt)[4], int k4)
{
    switch (n0) {
    case 4: one_round<4, T>(part, acc, ql, brow, g0, at, bt, k4); break;
    case 3: one_round<3, T>(part, acc, ql, brow, g0, at, bt, k4); break;
    case 2: one_round<2, T>(part, acc, ql, brow, g0, at, bt, k4); break;
    case 1: one_round<1, T>(part, acc, ql, brow, g0, at, bt, k4); break;
    default: one_round<0, T>(part, acc, ql, brow, g0, at, bt, k4); break;
    }
}

// m = 16, staged rows, no permutation (every workload's shape), a body of
// its own in which every wave takes the norms itself (no barrier between
// the norms and the products) and the loads of each round trip are issued
// together as straight-line code.
// The full-space tile (K = d, L times a subspace tile's K) is split over the
// waves, four K groups per round trip, and the parts summed at the end in
// the order (p0 + p1) + (p2 + p3); the subspace tiles go round robin (tile
// 1 + wv + 4 s to wave wv), four tiles per round trip, each taking its K
// groups, then its last dp mod 16 steps, in order.  When a wave's whole
// work fits one round trip (d / L = 16, at most 4 full-space groups and 4
// tiles per wave: d = 128, L = 8) it is requested at once.  A block of 16
// queries then takes as long as a kernel of the same grid that only reads
// its rows and writes its tables.  Rows past the batch are zero and not
// stored.
__device__ __forceinline__ void query_table16(const QueryTableArgs& a, float* qs, int nrows,
                                              int64_t q0, int wv, int lane)
{
#pragma clang fp contract(off)
    const int d = a.d, L = a.L;
    const int dp = d / L;
    const int ld = d + 4;
    const int row = lane & 15;  // A row, and B column (direction)
    const int kq = lane >> 4;   // K offset within a step
    const float* ql = qs + row * ld;

    const int ng = d >> 4;
    const int per = (ng + kTableWaves - 1) / kTableWaves;
    const int g0 = wv * per < ng ? wv * per : ng;
    const int g1 = g0 + per < ng ? g0 + per : ng;
    const float* brow = a.dirs_b + (int64_t)row * d;
    const int gpt = dp >> 4;
    const int ntw = L > wv ? (L - wv + kTableWaves - 1) / kTableWaves : 0;
    // operands of the wave's tiles sb .. sb + 3 (a slot past its last tile
    // repeats that tile: computed, not stored)
    auto tile_ptrs = [&](int sb, const float* (&at)[4], const float* (&bt)[4]) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = sb + u < ntw ? sb + u : ntw - 1;
            const int blk = wv + kTableWaves * s;  // subspace i - 1
            bt[u] = a.dirs_a + ((int64_t)blk * 16 + row) * dp;
            at[u] = ql + blk * dp;
        }
    };

    floatx4 part = {0.f, 0.f, 0.f, 0.f};
    floatx4 acc[4];
    const float* at[4];
    const float* bt[4];
    const int n0 = g1 - g0;
    const bool single = dp == 16 && n0 <= 4 && ntw >= 1 && ntw <= 4;
    if (single) {
        tile_ptrs(0, at, bt);
        if (ntw == 1) one_round_n<1>(n0, part, acc, ql, brow, g0, at, bt, 4 * kq);
        else if (ntw == 2) one_round_n<2>(n0, part, acc, ql, brow, g0, at, bt, 4 * kq);
        else one_round_n<4>(n0, part, acc, ql, brow, g0, at, bt, 4 * kq);
    } else {
        int j = g0;
        for (; j + 4 <= g1; j += 4) part = mfma_groups<4>(part, ql, brow, j, 4 * kq);
        switch (g1 - j) {
        case 3: part = mfma_groups<3>(part, ql, brow, j, 4 * kq); break;
        case 2: part = mfma_groups<2>(part, ql, brow, j, 4 * kq); break;
        case 1: part = mfma_groups<1>(part, ql, brow, j, 4 * kq); break;
        default: break;
        }
    }
    if (wv == kTableWaves - 1)
        for (int k0 = 16 * ng; k0 < d; k0 += 4)
            part = __builtin_amdgcn_mfma_f32_16x16x4f32(ql[k0 + kq], brow[k0 + kq], part, 0, 0, 0);

    const float nrm = staged_row_norm(ql, d, kq);
    const float inv = (nrm > 0.f && nrm < INFINITY) ? 1.f / nrm : 0.f;
    if (wv == 0 && kq == 0 && row < nrows) a.qnorms[q0 + row] = nrm;
    float invr[4];  // 1/|q| of output row 4 kq + r
#pragma unroll
    for (int r = 0; r < 4; ++r) invr[r] = __shfl(inv, 4 * kq + r, kWave);
    auto store = [&](const floatx4& v, int i) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int orow = 4 * kq + r;
            if (orow < nrows) {
                const float tv = v[r] * invr[r];
                const int64_t o = ((q0 + orow) * (L + 1) + i) * 16 + row;
                if (a.half_out) reinterpret_cast<_Float16*>(a.tables)[o] = (_Float16)tv;
                else a.tables[o] = tv;
            }
        }
    };

    if (single) {
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (u < ntw) store(acc[u], 1 + wv + kTableWaves * u);
    } else {
        for (int sb = 0; sb < ntw; sb += 4) {
            tile_ptrs(sb, at, bt);
#pragma unroll
            for (int u = 0; u < 4; ++u) acc[u] = floatx4{0.f, 0.f, 0.f, 0.f};
            for (int jg = 0; jg < gpt; ++jg) {
                float4 bq[4], aq[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bq[u] = *reinterpret_cast<const float4*>(bt[u] + 16 * jg + 4 * kq);
                    aq[u] = *reinterpret_cast<const float4*>(at[u] + 16 * jg + 4 * kq);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].x, bq[u].x, acc[u], 0, 0, 0);
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].y, bq[u].y, acc[u], 0, 0, 0);
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].z, bq[u].z, acc[u], 0, 0, 0);
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].w, bq[u].w, acc[u], 0, 0, 0);
                }
            }
            for (int k0 = 16 * gpt; k0 < dp; k0 += 4) {
                float bs[4], as[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    bs[u] = bt[u][k0 + kq];
                    as[u] = at[u][k0 + kq];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    acc[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[u], bs[u], acc[u], 0, 0, 0);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (sb + u < ntw) store(acc[u], 1 + wv + kTableWaves * (sb + u));
        }
    }

    // the parts to LDS (the staged rows are dead once every wave is past its
    // MFMAs and norms), then wave 0 sums them
    __syncthreads();
    *reinterpret_cast<floatx4*>(qs + (wv * 64 + lane) * 4) = part;
    __syncthreads();
    if (wv == 0) {
        floatx4 p[kTableWaves];
#pragma unroll
        for (int w = 0; w < kTableWaves; ++w) p[w] = *reinterpret_cast<const floatx4*>(qs + (w * 64 + lane) * 4);
        floatx4 sum;
#pragma unroll
        for (int r = 0; r < 4; ++r) sum[r] = (p[0][r] + p[1][r]) + (p[2][r] + p[3][r]);
        store(sum, 0);
    }
}

__global__ __launch_bounds__(kTableWaves * 64) void k_query_table(QueryTableArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) float qs[];  // 16 x (d + 4)
    __shared__ float inv_norm[16];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = wave_uniform(tid >> 6);  // (so that branches on it stay scalar)
    const int64_t q0 = (int64_t)blockIdx.x * 16;
    const int d = a.d, L = a.L, m = a.m;
    const int dp = d / L;
    const int ld = d + 4;
    const int nrows = (int)(a.nq - q0 < 16 ? a.nq - q0 : 16);

    // stage the tile in the original coordinate order (the norm is taken in
    // that order; a dimension permutation of the test is applied when the
    // operands are read).  Past 16 (d + 4) floats of LDS the rows are read
    // from global memory instead.
    const int nch = d >> 2;
    if (a.staged) {
        for (int c = tid; c < 16 * nch; c += kTableWaves * 64) {
            const int r = c / nch, k4 = (c - r * nch) * 4;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r < nrows)
                v = *reinterpret_cast<const float4*>(a.queries + (q0 + r) * (int64_t)d + k4);
            *reinterpret_cast<float4*>(qs + r * ld + k4) = v;
        }
    }
    __syncthreads();
    if (a.staged && !a.perm && m == 16) {
        query_table16(a, qs, nrows, q0, wv, lane);
        return;
    }

    const int row = lane & 15;
    const int kq = lane >> 4;
    const bool rv = row < nrows;
    // this lane's row: in LDS, or in global memory (rows past the batch read
    // row 0 and contribute zeros)
    const float* qrow = a.staged ? qs + row * ld : a.queries + (q0 + (rv ? row : 0)) * (int64_t)d;
    auto qget = [&](int kk) { return (a.staged || rv) ? qrow[kk] : 0.f; };
    if (wv == 0) {
        // |q| in the order of staged_row_norm, from LDS or global memory
        float nrm;
        if (a.staged) {
            nrm = staged_row_norm(qrow, d, kq);
        } else {
            float ss = 0.f;
            for (int k = kq; k < d; k += 4) {
                const float v = qget(k);
                ss = fmaf(v, v, ss);
            }
            ss += __shfl_xor(ss, 16, kWave);
            ss += __shfl_xor(ss, 32, kWave);
            nrm = sqrtf(ss);
        }
        if (kq == 0) {
            inv_norm[row] = (nrm > 0.f && nrm < INFINITY) ? 1.f / nrm : 0.f;
            if (row < nrows) a.qnorms[q0 + row] = nrm;
        }
    }
    __syncthreads();

    const int col = lane & 15;
    const int kb = lane >> 4;
    const int ntile = (L + 1) * (m >> 4);
    const bool fast = a.staged && !a.perm;

    // staged rows, no permutation: K in groups of 16, each one 16-byte load
    // per lane for either operand.  Within group j, step 4j + c takes
    // k = 16j + 4 (lane/16) + c from both operands (any assignment of the k
    // to the steps gives the same sum up to rounding, as long as A and B
    // agree).  Four groups' loads are issued before their MFMAs; then the
    // last k_len mod 16 step by step (k = k0 + lane/16).
    auto fast_tile = [&](floatx4 acc, int k_begin, const float* bv, int k_len) {
        const float* ql = qs + row * ld + k_begin;  // (an LDS pointer, so LDS reads)
        const int g1 = k_len >> 4;
        int j = 0;
        for (; j + 4 <= g1; j += 4) {
            float4 bq[4], aq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                bq[u] = *reinterpret_cast<const float4*>(bv + 16 * (j + u) + 4 * kb);
                aq[u] = *reinterpret_cast<const float4*>(ql + 16 * (j + u) + 4 * kq);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].x, bq[u].x, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].y, bq[u].y, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].z, bq[u].z, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[u].w, bq[u].w, acc, 0, 0, 0);
            }
        }
        for (; j < g1; ++j) {
            const float4 bq = *reinterpret_cast<const float4*>(bv + 16 * j + 4 * kb);
            const float4 aq = *reinterpret_cast<const float4*>(ql + 16 * j + 4 * kq);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.x, bq.x, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.y, bq.y, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.z, bq.z, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(aq.w, bq.w, acc, 0, 0, 0);
        }
        for (int k0 = 16 * g1; k0 < k_len; k0 += 4)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ql[k0 + kq], bv[k0 + kb], acc, 0, 0, 0);
        return acc;
    };

    for (int t = wv; t < ntile; t += kTableWaves) {
        const int i = t / (m >> 4);
        const int jdir = (t - i * (m >> 4)) * 16 + col;
        const int k_begin = (i == 0) ? 0 : (i - 1) * dp;
        const int k_len = (i == 0) ? d : dp;
        const float* bv = (i == 0) ? a.dirs_b + (int64_t)jdir * d
                                   : a.dirs_a + ((int64_t)(i - 1) * m + jdir) * dp;
        // operand k of this lane: coordinate k_begin + k of the (permuted) row
        auto qa = [&](int k) {
            const int kk = k_begin + k + kq;
            return qget(a.perm ? a.perm[kk] : kk);
        };
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        if (fast) {
            acc = fast_tile(acc, k_begin, bv, k_len);
        } else {
            int k0 = 0;
            for (; k0 + 32 <= k_len; k0 += 32) {
                float bb[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) bb[u] = bv[k0 + 4 * u + kb];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa(k0 + 4 * u), bb[u], acc, 0, 0, 0);
            }
            for (; k0 < k_len; k0 += 4)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(qa(k0), bv[k0 + kb], acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int orow = 4 * (lane >> 4) + r;
            if (orow < nrows) {
                const float tv = acc[r] * inv_norm[orow];
                const int64_t o = ((q0 + orow) * (L + 1) + i) * m + jdir;
                if (a.half_out) reinterpret_cast<_Float16*>(a.tables)[o] = (_Float16)tv;
                else a.tables[o] = tv;
            }
        }
    }
}

}  // namespace peos
