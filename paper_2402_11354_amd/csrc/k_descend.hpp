// Entry descent through upper layers.  The experiments run PEOs on HNSW
// graphs, whose base-layer search (Alg. 1) starts from the node a greedy
// walk down sparser upper layers reaches: in each layer, from the current
// node, take the closest of its neighbours in that layer (distance, then id)
// while it is closer than the current node, then continue from the same node
// one layer below; the node reached in the lowest upper layer is the entry.
//
// One wave per query; per step, one lane per neighbour row, the neighbours'
// distances gathered with the search's own canonical single-precision order
// (so the walk takes exactly the decisions the search's distances would),
// and a wave minimum over (distance, id) keys.  Every walk ends: each move
// strictly lowers the (distance, id) key of the current node, the layers are
// checked on the host (rows in range, `down` goes one layer down), and a step
// cap bounds the loop regardless.
#pragma once

#include "k_search.hpp"

namespace peos {

struct DescendArgs {
    const float* base;
    const uint16_t* base16;  // bfloat16 traversal copy, or null
    const float* queries;    // nq x d
    const float* qnorms;     // nq
    const int32_t* node;     // rows: base id
    const int32_t* adj;      // rows x ru: rows of the neighbours, -1 = none
    const int32_t* down;     // rows: row one layer below, -1 in the lowest upper layer
    int32_t* entries;        // out: nq entry nodes
    int32_t* stats;          // out: column 12 (distances of the walk), or null
    int32_t nq, d, ru, top, metric, max_steps;
};

// LDS: qv[d] | ids[64] | dists[64] | rows[64]
template <bool BF>
__global__ __launch_bounds__(64) void k_descend(DescendArgs a)
{
#pragma clang fp contract(off)
    extern __shared__ __align__(16) unsigned char sm[];
    const int d = a.d;
    float* qv = reinterpret_cast<float*>(sm);
    uint32_t* Su = reinterpret_cast<uint32_t*>(qv + d);
    float* Sdist = reinterpret_cast<float*>(Su + kWave);
    int32_t* Srow = reinterpret_cast<int32_t*>(Sdist + kWave);
    const int lane = lane_id();
    const void* tbase = BF ? (const void*)a.base16 : (const void*)a.base;
    for (int64_t qi = blockIdx.x; qi < a.nq; qi += gridDim.x) {
        const float qn = a.qnorms[qi];
        int32_t cur = a.top;
        int nd = 0;
        if (qn > 0.f && qn < INFINITY) {
            const float inv_qn = 1.f / qn;
            for (int t = lane; t < d; t += kWave) qv[t] = a.queries[qi * d + t];
            if (lane == 0) Su[0] = (uint32_t)a.node[cur];
            wave_sync();
            distances<BF>(tbase, d, Su, 1, qv, a.metric, inv_qn, Sdist);
            wave_sync();
            uint64_t kcur = sort_key(Sdist[0], Su[0]);
            nd = 1;
            wave_sync();
            for (int step = 0; step < a.max_steps; ++step) {
                const int32_t nb = lane < a.ru ? a.adj[(int64_t)cur * a.ru + lane] : -1;
                const bool valid = nb >= 0;
                const uint64_t mk = ballot(valid);
                const int ns = popc(mk);
                if (valid) {
                    const int pos = popc(mk & lanemask_lt());
                    Su[pos] = (uint32_t)a.node[nb];
                    Srow[pos] = nb;
                }
                wave_sync();
                if (ns > 0) distances<BF>(tbase, d, Su, ns, qv, a.metric, inv_qn, Sdist);
                wave_sync();
                nd += ns;
                // smallest (distance, id) among the current node and its neighbours
                uint64_t key = lane < ns ? sort_key(Sdist[lane], Su[lane]) : kcur;
                const int32_t row = lane < ns ? Srow[lane] : cur;
                uint64_t kmin = key;
#pragma unroll
                for (int o = 1; o < kWave; o <<= 1) {
                    const uint64_t ok = __shfl_xor(kmin, o, kWave);
                    kmin = ok < kmin ? ok : kmin;
                }
                wave_sync();
                if (kmin == kcur) {
                    const int32_t dn = a.down[cur];
                    if (dn < 0) break;
                    cur = dn;  // the same node one layer below
                } else {
                    const uint64_t hit = ballot(key == kmin);
                    cur = __shfl(row, __ffsll((unsigned long long)hit) - 1, kWave);
                    kcur = kmin;
                }
            }
        }
        if (lane == 0) {
            a.entries[qi] = a.node[cur];
            if (a.stats) a.stats[qi * kNumStats + 12] = nd;
        }
        wave_sync();
    }
}

}  // namespace peos
