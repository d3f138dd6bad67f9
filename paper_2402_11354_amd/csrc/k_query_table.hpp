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

// One workgroup of kTableWaves waves per tile of 16 queries.  The tile's query
// rows are staged in LDS with coalesced 16-byte loads (row stride d + 4
// floats, so the 16 rows x 4 consecutive k an MFMA step reads fall in 64
// distinct banks; up to 61 KB at d = 960); wave 0 takes the norms from LDS in
// the order below; the
// (L+1) x m/16 output tiles are dealt out to the waves, each running its
// contraction over K with the direction operands of 8 steps loaded before
// their MFMAs.
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
        float ss = 0.f;
        for (int k = kq; k < d; k += 4) {
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
