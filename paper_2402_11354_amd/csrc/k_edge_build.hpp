// PEOs steps (1)-(3) for every edge: one workgroup (one wave) per node v,
// four edges of v at a time, sixteen lanes per edge.
//
// For edge e = x_u - x_v (Sec. 4.2 of the paper):
//   (1) e = e_reg + e_res with e_reg the orthogonal projection of e on the
//       direction [e_i / (sqrt(L) |e_i|)]_i (a zero block contributes zero);
//       w_reg = |e_reg| / |e|, w_res = |e_res| / |e|;
//   (2) the projection vectors a^i_j, b_j are inputs;
//   (3) code e[i] = sign * argmax_j |e_i . a^i_j| per subspace, and e[0] the
//       same over e_res and b_j.
// The codes are integers decided by floating point, so they are computed in
// single precision with one fixed operation order, element for element:
//   e_k = x_u[k] - x_v[k]; s_i = sqrt(fma chain of e_k^2 over block i);
//   p_ij = fma chain over the block of e_k * a^i_j[k] (ascending, from 0);
//   j* = first j with the largest |p_ij|, negative sign iff p_ij* < 0;
//   c = (s_1 + ... + s_L) / L' (L' = nonzero blocks, sequential adds);
//   e_res_k = fma(-(c / s_i), e_k, e_k); p_0j = fma chain over all k.
// A code byte is j* + m * [sign < 0].
//
// Compact records (L <= 4; the experiments' compact form keeps w_reg = 1,
// w_res = 0 and two one-byte scalars per edge): the record starts with the
// node header {g_lo, g_step, i_lo, i_step}, then 4 code bytes per edge (byte
// i-1 = e[i]), then 2 scalar bytes per edge: cg = floor((gp - g_lo)/g_step)
// and ci = rint((ie - i_lo)/i_step) (255: zero-length edge), with gp =
// g_e/|e| (l2; 0 otherwise) and ie = 1/|e| in single precision:
//   ne2 = S_1 + ... + S_L (S_i the block's fma chain), ne = sqrt(ne2),
//   |x|^2 = fma chain over the original coordinates in order,
//   gp = (0.5 (|u|^2 - |v|^2)) / ne, ie = 1 / ne,
//   g_lo..g_hi, i_lo..i_hi over the node's edges of nonzero length,
//   g_step = (g_hi - g_lo)/255, i_step = (i_hi - i_lo)/254.
// The rounding directions make the search's A_r a lower bound of the exact
// one (g rounded down; 1/|e| decoded half a step towards the safe side).
#pragma once

#include "peos_device.hpp"

namespace peos {

struct EdgeBuildArgs {
    const float* base;
    const int32_t* graph;
    const float* dirs_a;  // L x m x dp
    const float* dirs_b;  // m x d
    uint8_t* rec;         // n x node_stride bytes
    int32_t* err;         // graph-validation flag (0 = ok)
    int64_t n;
    int64_t node_stride, codes_off, scal_off;
    int d, R, L, m, metric;
    int half_scalars;  // precision form: scalars as four halves per edge
    const int32_t* perm;  // optional dimension permutation: coordinate k of
                          // the test's vectors is original coordinate perm[k]
    const float* sdirs;   // 64 x d SimHash vectors, or null
    int64_t sig_off;      // SimHash signatures within a record
    int compact;          // compact records (see above)
};

constexpr int kCompactZeroEdge = 255;

// LDS: xv[d] | e[4][d] | s[4][L] | row[R] | compact: gp[R] | ie[R] | kind[R]
__global__ __launch_bounds__(64) void k_edge_build(EdgeBuildArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ float smem[];
    const int64_t v = blockIdx.x;
    if (v >= a.n) return;
    const int d = a.d, R = a.R, L = a.L, m = a.m;
    const int dp = d / L;
    float* xv = smem;
    float* ebuf = xv + d;
    float* sblk = ebuf + 4 * d;
    int32_t* row = reinterpret_cast<int32_t*>(sblk + 4 * L);
    float* cgp = reinterpret_cast<float*>(row + R);
    float* cie = cgp + R;
    int32_t* ckd = reinterpret_cast<int32_t*>(cie + R);
    const int lane = lane_id();
    const bool compact = a.compact != 0;
    const int g = lane >> 4;   // edge slot within the wave
    const int s = lane & 15;   // lane within the edge's group

    const float* xvg = a.base + v * (int64_t)d;
    float nv2 = 0.f;
    for (int k = lane; k < d; k += kWave) {
        float x = xvg[a.perm ? a.perm[k] : k];
        xv[k] = x;
        nv2 = fmaf(x, x, nv2);
    }
    nv2 = wave_sum(nv2);
    // compact records: |v|^2 as one fma chain in coordinate order
    float nv2c = 0.f;
    if (compact) {
        for (int k = 0; k < d; ++k) nv2c = fmaf(xvg[k], xvg[k], nv2c);
    }
    for (int j = lane; j < R; j += kWave) row[j] = a.graph[v * R + j];
    __syncthreads();

    // graph validation: id range, self loop, repeated id in the row
    for (int j = lane; j < R; j += kWave) {
        int32_t u = row[j];
        bool bad = (u < -1) || (u >= a.n) || (u == v);
        if (u >= 0)
            for (int jj = 0; jj < j; ++jj) bad |= (row[jj] == u);
        if (bad) atomicOr(a.err, 1);
    }

    uint8_t* rv = a.rec + v * a.node_stride;
    uint8_t* codes = rv + a.codes_off;
    // full records: round_up(B + 1, 4) code bytes per edge with B the
    // search kernel's subspace bound (8, 16 or 32; zero past L), byte 0 the
    // residual code; compact: 4 bytes, byte i-1 = e[i]
    const int cbytes = compact ? 4 : (((L <= 8 ? 8 : (L <= 16 ? 16 : 32)) + 4) & ~3);
    const int cfirst = compact ? 0 : 1;
    float* scal = reinterpret_cast<float*>(rv + a.scal_off);

    for (int j0 = 0; j0 < R; j0 += 4) {
        const int j = j0 + g;
        // an out-of-range id is never dereferenced (it is reported through err)
        int32_t u = (j < R) ? row[j] : -1;
        if (u >= a.n) u = -1;
        float* e = ebuf + g * d;
        float* sb = sblk + g * L;
        float nu2 = 0.f, ne2 = 0.f;
        if (u >= 0) {
            const float* xu = a.base + (int64_t)u * d;
            for (int k = s; k < d; k += 16) {
                float x = xu[a.perm ? a.perm[k] : k];
                float t = x - xv[k];
                e[k] = t;
                nu2 = fmaf(x, x, nu2);
                ne2 = fmaf(t, t, ne2);
            }
        }
        nu2 = group_sum<16>(nu2);
        ne2 = group_sum<16>(ne2);
        __syncthreads();
        // block norms, fixed order
        if (u >= 0) {
            for (int i = s; i < L; i += 16) {
                float ss = 0.f;
                for (int t = 0; t < dp; ++t) ss = fmaf(e[i * dp + t], e[i * dp + t], ss);
                sb[i] = sqrtf(ss);
            }
        }
        // compact scalars in the order stated above (one lane per edge)
        if (compact && s == 0 && j < R) {
            int kd = 0;
            float gp = 0.f, ie = 0.f;
            if (u >= 0) {
                float ne2c = 0.f;
                for (int i = 0; i < L; ++i) {
                    float ss = 0.f;
                    for (int t = 0; t < dp; ++t) ss = fmaf(e[i * dp + t], e[i * dp + t], ss);
                    ne2c = ne2c + ss;
                }
                const float ne = sqrtf(ne2c);
                kd = 2;
                if (ne > 0.f) {
                    kd = 1;
                    if (a.metric == 0) {
                        const float* xu = a.base + (int64_t)u * d;
                        float nu2c = 0.f;
                        for (int k = 0; k < d; ++k) nu2c = fmaf(xu[k], xu[k], nu2c);
                        gp = (0.5f * (nu2c - nv2c)) / ne;
                    }
                    ie = 1.f / ne;
                }
            }
            cgp[j] = gp;
            cie[j] = ie;
            ckd[j] = kd;
        }
        // subspace codes
        for (int i = 0; i < L; ++i) {
            float best = -1.f, bp = 0.f;
            int bj = 0;
            if (u >= 0) {
                for (int jj = s; jj < m; jj += 16) {
                    const float* av = a.dirs_a + ((int64_t)i * m + jj) * dp;
                    float p = 0.f;
                    for (int t = 0; t < dp; ++t) p = fmaf(e[i * dp + t], av[t], p);
                    float ap = fabsf(p);
                    if (ap > best) { best = ap; bj = jj; bp = p; }
                }
            }
            // first maximum across the group: larger |p|, ties to smaller j
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                float ob = __shfl_xor(best, o, 16);
                int oj = __shfl_xor(bj, o, 16);
                float op = __shfl_xor(bp, o, 16);
                if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; bp = op; }
            }
            if (s == 0 && j < R)
                codes[j * cbytes + cfirst + i] = (u >= 0) ? (uint8_t)(bj + (bp < 0.f ? m : 0)) : 0;
        }
        if (compact) {
            if (s == 0 && j < R)
                for (int pz = L; pz < 4; ++pz) codes[j * cbytes + pz] = 0;
            __syncthreads();
            continue;
        }
        __syncthreads();
        // SimHash signature of e (before e is overwritten by its residual):
        // bit i = [e . c_i >= 0], an fma chain over the coordinates in
        // order; lane s of the edge's group computes bits s, s+16, s+32, s+48
        if (a.sdirs) {
            uint32_t lo = 0u, hi = 0u;
            if (u >= 0) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int i = s + 16 * r;
                    const float* cv = a.sdirs + (int64_t)i * d;
                    float p = 0.f;
                    for (int k = 0; k < d; ++k) p = fmaf(e[k], cv[k], p);
                    if (p >= 0.f) {
                        if (i < 32) lo |= 1u << i;
                        else hi |= 1u << (i - 32);
                    }
                }
            }
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                lo |= (uint32_t)__shfl_xor((int)lo, o, 16);
                hi |= (uint32_t)__shfl_xor((int)hi, o, 16);
            }
            if (s == 0 && j < R)
                *reinterpret_cast<uint2*>(rv + a.sig_off + 8 * j) = make_uint2(lo, hi);
        }
        // regular part: c = sum(s_i) / L', residual in place
        float c = 0.f;
        int nz = 0;
        if (u >= 0) {
            float sum = 0.f;
            for (int i = 0; i < L; ++i) {
                sum = sum + sb[i];
                nz += sb[i] > 0.f;
            }
            c = nz > 0 ? sum / (float)nz : 0.f;
        }
        __syncthreads();
        float nr2 = 0.f;
        if (u >= 0) {
            for (int k = s; k < d; k += 16) {
                const float sk = sb[k / dp];
                const float r = sk > 0.f ? c / sk : 0.f;
                const float ek = e[k];
                const float t = fmaf(-r, ek, ek);
                e[k] = t;
                nr2 = fmaf(t, t, nr2);
            }
        }
        nr2 = group_sum<16>(nr2);
        __syncthreads();
        // residual code
        {
            float best = -1.f, bp = 0.f;
            int bj = 0;
            if (u >= 0) {
                for (int jj = s; jj < m; jj += 16) {
                    const float* bv = a.dirs_b + (int64_t)jj * d;
                    float p = 0.f;
                    for (int k = 0; k < d; ++k) p = fmaf(e[k], bv[k], p);
                    float ap = fabsf(p);
                    if (ap > best) { best = ap; bj = jj; bp = p; }
                }
            }
#pragma unroll
            for (int o = 8; o >= 1; o >>= 1) {
                float ob = __shfl_xor(best, o, 16);
                int oj = __shfl_xor(bj, o, 16);
                float op = __shfl_xor(bp, o, 16);
                if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; bp = op; }
            }
            if (s == 0 && j < R) {
                codes[j * cbytes] = (u >= 0) ? (uint8_t)(bj + (bp < 0.f ? m : 0)) : 0;
                for (int pz = L + 1; pz < cbytes; ++pz) codes[j * cbytes + pz] = 0;
            }
        }
        // scalars: g_e, |e|, w_reg, sqrt(L) w_res; in the precision form
        // the halves of g_e/|e|, 1/|e| (infinite for a zero edge), w_reg,
        // sqrt(L) w_res
        if (s == 0 && j < R) {
            float ge = 0.f, ne = 0.f, wreg = 0.f, swres = 0.f;
            if (u >= 0) {
                ne = sqrtf(ne2);
                if (ne > 0.f) {
                    wreg = fminf(1.f, c * sqrtf((float)nz) / ne);
                    swres = sqrtf((float)L) * fminf(1.f, sqrtf(nr2) / ne);
                } else {
                    wreg = 1.f;
                    swres = 0.f;
                }
                if (a.metric == 0) ge = 0.5f * (nu2 - nv2);
            }
            if (a.half_scalars) {
                const float gp = ne > 0.f ? ge / ne : 0.f;
                const float ie = ne > 0.f ? 1.f / ne : INFINITY;
                _Float16* hs = reinterpret_cast<_Float16*>(rv + a.scal_off) + 4 * j;
                hs[0] = (_Float16)(u >= 0 ? gp : 0.f);
                hs[1] = (_Float16)(u >= 0 ? ie : 0.f);
                hs[2] = (_Float16)wreg;
                hs[3] = (_Float16)swres;
            } else {
                *reinterpret_cast<float4*>(scal + 4 * j) = make_float4(ge, ne, wreg, swres);
            }
        }
        __syncthreads();
    }
    if (!compact) return;
    // compact: node ranges (min / max are exact in any order) and the codes
    __syncthreads();
    float glo = INFINITY, ghi = -INFINITY, ilo = INFINITY, ihi = -INFINITY;
    for (int j = 0; j < R; ++j) {
        if (ckd[j] != 1) continue;
        glo = fminf(glo, cgp[j]);
        ghi = fmaxf(ghi, cgp[j]);
        ilo = fminf(ilo, cie[j]);
        ihi = fmaxf(ihi, cie[j]);
    }
    if (!(glo <= ghi)) glo = ghi = ilo = ihi = 0.f;  // no edge of nonzero length
    const float gstep = (ghi - glo) / 255.f;
    const float istep = (ihi - ilo) / 254.f;
    if (lane == 0) *reinterpret_cast<float4*>(rv) = make_float4(glo, gstep, ilo, istep);
    for (int j = lane; j < R; j += kWave) {
        uint32_t cg = 0u, ci = 0u;
        if (ckd[j] == 2) ci = kCompactZeroEdge;
        if (ckd[j] == 1) {
            if (gstep > 0.f) {
                const float c = floorf((cgp[j] - glo) / gstep);
                cg = (uint32_t)(c < 0.f ? 0.f : (c > 255.f ? 255.f : c));
            }
            if (istep > 0.f) {
                const float c = rintf((cie[j] - ilo) / istep);
                ci = (uint32_t)(c < 0.f ? 0.f : (c > 254.f ? 254.f : c));
            }
        }
        reinterpret_cast<uint16_t*>(rv + a.scal_off)[j] = (uint16_t)(cg | (ci << 8));
    }
}

// Energy of the edge coordinates for the optional dimension permutation:
// partial[b][j] = sum over the edges (v, u) of the nodes v = b, b + grid, ...
// of (x_u[j] - x_v[j])^2, in that fixed order (threads over coordinates).
__global__ __launch_bounds__(256) void k_edge_energy(const float* base, const int32_t* graph,
                                                     int64_t n, int d, int R, float* partial)
{
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        float acc = 0.f;
        for (int64_t v = blockIdx.x; v < n; v += gridDim.x) {
            const float xv = base[v * d + j];
            for (int r = 0; r < R; ++r) {
                const int32_t u = graph[v * R + r];
                if (u < 0 || u >= n) continue;
                const float t = base[(int64_t)u * d + j] - xv;
                acc = fmaf(t, t, acc);
            }
        }
        partial[(int64_t)blockIdx.x * d + j] = acc;
    }
}

// bfloat16 copy of the base (round to nearest even), the traversal copy of
// the precision form
__global__ void k_to_bf16(const float* x, uint16_t* y, int64_t count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        uint32_t u = __float_as_uint(x[i]);
        if ((u & 0x7f800000u) != 0x7f800000u) u += 0x7fffu + ((u >> 16) & 1u);
        y[i] = (uint16_t)(u >> 16);
    }
}

}  // namespace peos
