// PEOs step (5): the projection table of every query, on the matrix cores.
//
// tables[q][i][j] = q'_i . a^i_j (i = 1..L) and tables[q][0][j] = q' . b_j,
// with q' = q/|q| and q'_i its i-th block (Sec. 4.2; the table is built once
// per query, Alg. 2).  As a matrix product this is Q x [B^T | blockdiag(A^i)^T]
// scaled by 1/|q| per row; the block-diagonal structure is kept (each
// subspace contracts over its own d/L coordinates only).
//
// One wave computes 16 queries x 16 directions with v_mfma_f32_16x16x4f32
// (fp32 in, fp32 accumulate): per K step of 4, lane l feeds A[row = l%16][k =
// l/16] (queries) and B[k = l/16][col = l%16] (directions), and receives
// D[row = 4*(l/16) + r][col = l%16], r = 0..3.  The precision form stores
// the table as halves.
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
    const int32_t* perm;   // optional dimension permutation of the test
};

__global__ __launch_bounds__(64) void k_query_table(QueryTableArgs a)
{
#pragma clang fp contract(off)
    __shared__ float inv_norm[16];
    const int lane = lane_id();
    const int row = lane & 15;
    const int kq = lane >> 4;
    const int64_t q0 = (int64_t)blockIdx.x * 16;
    const int64_t qrow = q0 + row;
    const bool valid = qrow < a.nq;
    const int d = a.d, L = a.L, m = a.m;
    const int dp = d / L;
    const float* qv = a.queries + (valid ? qrow : 0) * (int64_t)d;

    // |q| = sqrt((p0 + p1) + (p2 + p3)), p_j the fma chain of q_k^2 over
    // k = j mod 4 (one lane each), combined by two xor shuffles
    float ss = 0.f;
    if (valid)
        for (int k = kq; k < d; k += 4) ss = fmaf(qv[k], qv[k], ss);
    ss += __shfl_xor(ss, 16, kWave);
    ss += __shfl_xor(ss, 32, kWave);
    const float nrm = sqrtf(ss);
    if (kq == 0) {
        inv_norm[row] = (nrm > 0.f && nrm < INFINITY) ? 1.f / nrm : 0.f;
        if (valid) a.qnorms[qrow] = nrm;
    }
    __syncthreads();

    const int col = lane & 15;
    const int kb = lane >> 4;
    for (int nt = 0; nt < m; nt += 16) {
        const int jdir = nt + col;
        for (int i = 0; i <= L; ++i) {
            floatx4 acc = {0.f, 0.f, 0.f, 0.f};
            const int k_begin = (i == 0) ? 0 : (i - 1) * dp;
            const int k_len = (i == 0) ? d : dp;
            const float* bv = (i == 0) ? a.dirs_b + (int64_t)jdir * d
                                       : a.dirs_a + ((int64_t)(i - 1) * m + jdir) * dp;
            for (int k0 = 0; k0 < k_len; k0 += 4) {
                const int kk = k_begin + k0 + kq;
                const float av = valid ? qv[a.perm ? a.perm[kk] : kk] : 0.f;
                const float bvv = bv[k0 + kb];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bvv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int orow = 4 * (lane >> 4) + r;
                const int64_t qq = q0 + orow;
                if (qq < a.nq) {
                    const float t = acc[r] * inv_norm[orow];
                    const int64_t o = (qq * (L + 1) + i) * m + jdir;
                    if (a.half_out) reinterpret_cast<_Float16*>(a.tables)[o] = (_Float16)t;
                    else a.tables[o] = t;
                }
            }
        }
    }
}

}  // namespace peos
