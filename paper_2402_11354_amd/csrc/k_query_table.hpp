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
// 64 distinct banks; up to 61 KB at d = 960); wave 0 takes the norms from LDS
// in the order below; the (L+1) x m/16 output tiles are dealt out to the
// waves, the full-space tile (K = d, L times a subspace tile's K) split over
// all of them when m = 16.  Both operands are read 16 bytes per lane: a group
// of four K steps per load.
constexpr int kTableWaves = 4;

__global__ __launch_bounds__(kTableWaves * 64) void k_query_table(QueryTableArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) float qs[];  // 16 x (d + 4)
    __shared__ float inv_norm[16];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = tid >> 6;
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

    const int row = lane & 15;
    const int kq = lane >> 4;
    const bool rv = row < nrows;
    // this lane's row: in LDS, or in global memory (rows past the batch read
    // row 0 and contribute zeros)
    const float* qrow = a.staged ? qs + row * ld : a.queries + (q0 + (rv ? row : 0)) * (int64_t)d;
    auto qget = [&](int kk) { return (a.staged || rv) ? qrow[kk] : 0.f; };
    if (wv == 0) {
        // |q| = sqrt((p0 + p1) + (p2 + p3)), p_j the fma chain of q_k^2 over
        // k = j mod 4 (one lane each), combined by two xor shuffles
        // (eight terms are read together, then chained; LDS reads when staged)
        float ss = 0.f;
        int k = kq;
        if (a.staged) {
            const float* ql = qs + row * ld;
            for (; k + 28 < d; k += 32) {
                float v[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) v[j] = ql[k + 4 * j];
#pragma unroll
                for (int j = 0; j < 8; ++j) ss = fmaf(v[j], v[j], ss);
            }
        }
        for (; k < d; k += 4) {
            const float v = qget(k);
            ss = fmaf(v, v, ss);
        }
        ss += __shfl_xor(ss, 16, kWave);
        ss += __shfl_xor(ss, 32, kWave);
        const float nrm = sqrtf(ss);
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
    // agree).  Four groups' loads are issued before their MFMAs.  Groups
    // [g0, g1) of a tile whose K range starts at query coordinate k_begin
    // and at bv in the direction row; with rem, the last k_len mod 16 step by
    // step (k = k0 + lane/16).
    auto fast_groups = [&](floatx4 acc, int k_begin, const float* bv, int g0, int g1, int k_len, bool rem) {
        const float* ql = qs + row * ld + k_begin;  // (an LDS pointer, so LDS reads)
        int j = g0;
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
        if (rem)
            for (int k0 = 16 * (k_len >> 4); k0 < k_len; k0 += 4)
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(ql[k0 + kq], bv[k0 + kb], acc, 0, 0, 0);
        return acc;
    };
    auto store_tile = [&](floatx4 acc, int i, int jdir) {
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
    };

    // with m = 16 (one full-space tile) and the fast path, the full-space
    // tile's K groups are split over the waves (its chain is L times longer
    // than a subspace tile's) and the parts summed at the end; the other
    // tiles go round robin
    const bool split = fast && m == 16;
    floatx4 part = {0.f, 0.f, 0.f, 0.f};
    if (split) {
        const int ng = d >> 4;
        const int per = (ng + kTableWaves - 1) / kTableWaves;
        const int g0 = wv * per < ng ? wv * per : ng;
        const int g1 = g0 + per < ng ? g0 + per : ng;
        part = fast_groups(part, 0, a.dirs_b + (int64_t)col * d, g0, g1, d, wv == kTableWaves - 1);
    }
    for (int t = split ? 1 + wv : wv; t < ntile; t += kTableWaves) {
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
            acc = fast_groups(acc, k_begin, bv, 0, k_len >> 4, k_len, true);
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
        store_tile(acc, i, jdir);
    }
    if (split) {
        // the parts to LDS (the staged rows are dead once every wave is past
        // its MFMAs), then wave 0 sums them in the order (p0 + p1) + (p2 + p3)
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
            store_tile(sum, 0, col);
        }
    }
}

}  // namespace peos
