/*
 * peos.h -- C ABI of the PEOs-routed graph search library for MI355X (gfx950).
 *
 * The library implements the search of Lu, Xiao and Ishikawa, "Probabilistic
 * Routing for Graph-Based Approximate Nearest Neighbor Search" (ICML 2024):
 * best-first search over a fixed proximity graph (Alg. 1) in which every
 * unvisited neighbour of the expanded node is first screened by the PEOs
 * routing test (Sec. 4.2, steps (1)-(6); Alg. 2), and only neighbours that
 * pass get an exact distance.
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers (hipMalloc'ed or torch CUDA
 *     tensors) unless marked "host".  The caller owns all memory; the library
 *     never allocates device memory and keeps no pointer after a call returns,
 *     except that a peos_index records the base, graph and index_mem pointers
 *     given to peos_build_tables, which must stay valid until peos_free.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Work is enqueued asynchronously on it unless stated otherwise.
 *   - Return value: PEOS_OK (0) or a negative PEOS_E* code.  No exception
 *     crosses the ABI.  peos_last_error() returns a thread-local message for
 *     the last failing call on this thread.
 *   - Row-major layouts throughout.
 */
#ifndef PEOS_H
#define PEOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define PEOS_OK 0
#define PEOS_EINVAL (-1)   /* an argument is out of range or inconsistent      */
#define PEOS_ENOSPACE (-2) /* a caller buffer is smaller than required          */
#define PEOS_EHIP (-3)     /* a HIP runtime call failed                         */
#define PEOS_EGRAPH (-4)   /* graph row with an out-of-range id, self loop or
                              repeated neighbour                               */
#define PEOS_EDEVICE (-5)  /* no gfx950 device is current                       */
#define PEOS_EBUSY (-6)    /* serving: the request queue is full; retry later    */

/* metrics.  L2: squared Euclidean distance |x - q|^2.  ANGULAR: 1 - x.q/|q|,
 * the cosine distance when base vectors have unit norm (Sec. 3 of the paper
 * reduces both to inner products; the test uses the MIPS numerator of the
 * "Extension to MIPS" appendix, which is exact for this distance). */
#define PEOS_METRIC_L2 0
#define PEOS_METRIC_ANGULAR 1
/* IP: maximum inner product search ("Extension to MIPS" appendix), distance
 * -x.q (results ordered by decreasing inner product; base rows of any norm).
 * The test takes A_r = (p.q - v.q)/(|q||e|) = (dist_v - delta)/(|q||e|),
 * p the result of smallest inner product; everything else is as for L2. */
#define PEOS_METRIC_IP 2

/* search modes.  PEOS: neighbours are screened by the routing test.
 * EXHAUSTIVE: the test is off (every unvisited neighbour gets a distance),
 * i.e. Alg. 1 with RoutingTest returning true. */
#define PEOS_MODE_PEOS 0
#define PEOS_MODE_EXHAUSTIVE 1
/* SIMHASH: the SimHash test of Sec. 3 ("SimHash Test") on the residual edge
 * e = u - v instead of the PEOs test: A_r as in step (6); A_r >= 1 fails,
 * A_r <= 0 passes; otherwise u passes iff the number of the 64 sign
 * projections on which e and q agree is at least
 * 64 (1 - arccos(A_r)/pi) - sqrt(64 ln(1/eps) / 2) (Hoeffding's bound on the
 * Binomial collision count at the boundary angle).  Needs an index built with
 * PEOS_FLAG_SIMHASH. */
#define PEOS_MODE_SIMHASH 2
/* index flags: the precision form (storage only; arithmetic stays single
 * precision).
 * PEOS_FLAG_BF16_BASE: index_mem also holds a bfloat16 copy of the base
 *   (round to nearest even); the search's traversal distances read it, and
 *   the result list (first ef entries) is re-ranked by single-precision
 *   distances on the full base before the first k are returned.
 * PEOS_FLAG_FP16: the per-edge scalars are stored as four IEEE halves
 *   {g_e/|e|, 1/|e| (infinite for a zero-length edge), w_reg, sqrt(L) w_res}
 *   and the projection tables as halves; the test of step (6) then takes
 *   A_r = (g_e/|e| + (dist_v - delta)/2 * 1/|e|) / |q| (l2) or
 *   (dist_v - delta)/|e| (angular) or (dist_v - delta)/(|e||q|) (IP), the
 *   same quantity as the full form's. */
#define PEOS_FLAG_BF16_BASE 1
#define PEOS_FLAG_FP16 2
/* PEOS_FLAG_SIMHASH: the records also hold, per edge, the 64 sign bits
 * [e . c_i >= 0] of the residual edge against the 64 vectors of
 * peos_build_options.simhash_dirs (for PEOS_MODE_SIMHASH). */
#define PEOS_FLAG_SIMHASH 4
/* PEOS_FLAG_COMPACT: the compact records of the experiments ("Indexing Cost",
 * "Scalability"): for L <= 4, w_reg = 1 and w_res = 0 for every edge (no
 * residual code), and two one-byte scalars per edge against ranges kept once
 * per node.  Record of node v: {g_lo, g_step, i_lo, i_step} (4 floats), then
 * 4 code bytes per edge (byte i-1 = e[i]), then 2 bytes per edge: cg =
 * floor((g_e/|e| - g_lo)/g_step) and ci = rint((1/|e| - i_lo)/i_step), with
 * ci = 255 for a zero-length edge (g_e/|e| is 0 for ANGULAR and IP).  The test
 * decodes g = g_lo + cg g_step and 1/|e| = i_lo + (ci +- 1/2) i_step, the
 * half step taken so that (dist_v - delta)/|e| is not overestimated, so its
 * A_r is at most the exact one; H = sum_i sgn(e[i]) T_i[|e[i]|]; T is read
 * from a table of 256 bins over A_r in [0, 1), bin b holding T(b/256) of
 * step (6) with w = (1, 0), rounded down (the smallest T of the bin: T grows
 * with A_r, so the quantile is never above the true one, as Sec. 4.3 allows).
 * Needs L <= 4; does not combine with PEOS_FLAG_FP16 or PEOS_FLAG_SIMHASH. */
#define PEOS_FLAG_COMPACT 8

/* per-query status bits written to stats[.. + PEOS_STAT_STATUS] */
#define PEOS_STATUS_ZERO_QUERY 1    /* |q| = 0 or not finite: outputs padded  */
#define PEOS_STATUS_POOL_FULL 2     /* the candidate list reached the kernel's
                                       capacity with pool = 0 (see peos_search) */
#define PEOS_STATUS_VISITED_SPILL 4 /* visited set moved from LDS to HBM       */

/* per-query statistics: PEOS_NSTATS int32 per query, in this order */
#define PEOS_STAT_EXPANSIONS 0   /* nodes popped and expanded                 */
#define PEOS_STAT_EDGES 1        /* valid neighbour ids enumerated            */
#define PEOS_STAT_VISITED_SKIPS 2/* neighbours skipped as already visited     */
#define PEOS_STAT_TESTS 3        /* routing tests run                          */
#define PEOS_STAT_TEST_GE1 4     /* tests decided by A_r >= 1 (fail)           */
#define PEOS_STAT_TEST_LE0 5     /* tests decided by A_r <= 0 (pass)           */
#define PEOS_STAT_TEST_H 6       /* tests decided by H >= T_r                  */
#define PEOS_STAT_TEST_ZERO 7    /* tests on zero-length edges                 */
#define PEOS_STAT_PASSES 8       /* tests passed                               */
#define PEOS_STAT_NDIST 9        /* exact distances computed (entry included)  */
#define PEOS_STAT_INSERTED 10    /* distances that entered the candidate list  */
#define PEOS_STAT_STATUS 11      /* PEOS_STATUS_* bits                         */
#define PEOS_STAT_DESCENT 12     /* distances of the upper-layer descent (0
                                    without upper layers)                      */
#define PEOS_STAT_TEST_EXPANSIONS 13 /* expansions that ran the test (list
                                    full; each loads the node's whole record) */
#define PEOS_NSTATS 14

typedef struct peos_index peos_index;
typedef struct peos_graph peos_graph;

/* Byte layout of the per-node edge records inside index_mem (for tests and
 * tools; the search needs nothing but the handle).  Record of node v starts at
 * v * node_stride.  Codes: edge j (to graph[v*R + j]) owns code_bytes =
 * round_up(B+1, 4) bytes at codes_offset + j*code_bytes, B = 8, 16 or 32 the
 * smallest of these >= L: byte 0 = residual code e[0], bytes 1..L = subspace
 * codes e[i], then zero padding.  A code
 * byte c encodes the index j* = c mod m of the extreme projection vector and
 * its sign (negative iff c >= m).  Scalars: edge j owns 4 floats at
 * scalars_offset + 16*j: g_e = (|u|^2 - |v|^2)/2 (zero for ANGULAR and IP), |e|,
 * w_reg, sqrt(L)*w_res; with PEOS_FLAG_FP16, 4 halves at scalars_offset + 8*j
 * (see PEOS_FLAG_FP16).  With PEOS_FLAG_COMPACT the record starts with the
 * node header at offset 0, code_bytes = 4 and scalar_bytes = 2 (see
 * PEOS_FLAG_COMPACT).  With PEOS_FLAG_BF16_BASE the bfloat16 copy of the
 * base (n x d) starts at bf16_offset. */
typedef struct {
    int64_t n;
    int32_t d, R, L, m, metric, flags, entry;
    int64_t node_stride;    /* bytes */
    int64_t codes_offset;   /* bytes, within a record */
    int64_t scalars_offset; /* bytes, within a record */
    int64_t code_bytes;     /* bytes of codes per edge */
    int64_t scalar_bytes;   /* bytes of scalars per edge (16, or 8 with halves) */
    int64_t bf16_offset;    /* bytes, within index_mem; 0 without the copy */
    int64_t simhash_offset; /* bytes, within a record: 8 bytes per edge (bit i =
                               sign i), 0 without PEOS_FLAG_SIMHASH */
} peos_layout;

/*
 * peos_index_bytes -- size the caller-owned index memory.
 * Implements: storage of PEOS steps (1)-(3) results per edge (Sec. 4.3,
 * "Implementation of PEOs": codes and scalars are precomputed at build time).
 * n, d, R, L, m: base size, dimension, max out-degree, subspaces, projection
 * vectors per subspace.  flags: 0, or PEOS_FLAG_* (the precision form, the
 * SimHash signatures, the compact records).
 * Outputs (host pointers): index_bytes = bytes of index_mem;
 * build_ws_bytes = bytes of the build workspace.  Pure, no device work.
 * Errors: PEOS_EINVAL if n < 1, d < 1, R < 1, L < 1, d % L != 0, d/L % 4 != 0,
 * m < 16, m % 16 != 0, 2*m > 256, an unknown flag, PEOS_FLAG_COMPACT with
 * L > 4 or with PEOS_FLAG_FP16 / PEOS_FLAG_SIMHASH, or a null output pointer.
 */
int peos_index_bytes(int64_t n, int32_t d, int32_t R, int32_t L, int32_t m, int32_t flags,
                     size_t* index_bytes, size_t* build_ws_bytes);

/*
 * peos_build_tables -- PEOs steps (1)-(3) for every edge of the graph
 * (Sec. 4.2: orthogonal decomposition e = e_reg + e_res of e = u - v, the
 * extreme-value codes e[0..L] against the projection vectors, and the weights
 * w_reg, w_res), plus the per-edge scalars the test of step (6) needs.
 *   base    n x d float, the vectors (ANGULAR expects unit-norm rows),
 *           16-byte aligned (rows are read as float4).
 *   graph   n x R int32 neighbour ids, -1 = no edge; ids in [0, n), no self
 *           loops and no repeated id within a row.
 *   entry   entry node v0 of the search (Alg. 1), in [0, n).
 *   dirs_a  L x m x (d/L) float: vectors a^i_j of subspace i (step (2)),
 *           16-byte aligned (the projection table reads them as float4).
 *   dirs_b  m x d float: full-space vectors b_j (step (2)), 16-byte aligned.
 *   metric  PEOS_METRIC_*.
 *   index_mem / index_bytes  caller buffer sized by peos_index_bytes, 16-byte aligned.
 *   ws / ws_bytes            build workspace (peos_index_bytes).
 *   out     (host) receives a handle; free it with peos_free.
 * The handle records base, graph, dirs_a, dirs_b and index_mem (not copied).
 * Synchronous: returns after the build finished on `stream` (it reads back a
 * graph-validation flag).  Errors: PEOS_EINVAL, PEOS_ENOSPACE, PEOS_EGRAPH
 * (the index is not created), PEOS_EHIP, PEOS_EDEVICE.
 */
int peos_build_tables(const float* base, int64_t n, int32_t d, const int32_t* graph, int32_t R,
                      int32_t entry, int32_t L, int32_t m, const float* dirs_a,
                      const float* dirs_b, int32_t metric, int32_t flags, void* index_mem,
                      size_t index_bytes, void* ws, size_t ws_bytes, void* stream,
                      peos_index** out);

/*
 * peos_dimension_permutation -- the optional dimension permutation of the
 * paper's appendix "Dimension Permutation" (also Sec. 4.3): per coordinate j
 * the energy sum over the graph's edges (v, u) of (x_u[j] - x_v[j])^2
 * (proportional to Avg(e_j)); the dimensions sorted by ascending energy
 * (ties: smaller index) are handed out in d/L rounds of L, each to the
 * subspace with the largest running energy among those not yet served in
 * the round (ties: smaller subspace).  perm (host, d int32) receives
 * perm[i*(d/L) + t] = the original coordinate placed at coordinate t of
 * sub-vector i.  ws: device workspace of peos_dimension_permutation_ws_bytes.
 * Synchronous on `stream`.  Errors: PEOS_EINVAL, PEOS_ENOSPACE, PEOS_EHIP.
 */
int peos_dimension_permutation_ws_bytes(int32_t d, size_t* ws_bytes);
int peos_dimension_permutation(const float* base, int64_t n, int32_t d, const int32_t* graph,
                               int32_t R, int32_t L, int32_t* perm, void* ws, size_t ws_bytes,
                               void* stream);
/*
 * peos_build_tables_ex -- peos_build_tables with options (opt may be NULL):
 *   perm          device, d int32, a permutation of 0..d-1, or NULL: steps
 *                 (1)-(3) and the projection tables of step (5) take
 *                 coordinate k of every vector from original coordinate
 *                 perm[k]; distances and everything else use the original
 *                 coordinates (the permutation changes neither the graph nor
 *                 the guarantee).  Kept by the index: must stay valid until
 *                 peos_free.  Not with PEOS_FLAG_SIMHASH.
 *   simhash_dirs  device, 64 x d float, required by PEOS_FLAG_SIMHASH: the
 *                 sign-projection vectors of the SimHash test (kept by the
 *                 index: the search projects each query on them).
 * Errors as peos_build_tables.
 */
typedef struct {
    const int32_t* perm;
    const float* simhash_dirs;
} peos_build_options;
int peos_build_tables_ex(const float* base, int64_t n, int32_t d, const int32_t* graph, int32_t R,
                         int32_t entry, int32_t L, int32_t m, const float* dirs_a,
                         const float* dirs_b, int32_t metric, int32_t flags,
                         const peos_build_options* opt, void* index_mem, size_t index_bytes,
                         void* ws, size_t ws_bytes, void* stream, peos_index** out);
/* Fill *out (host) with the record layout of an index.  Errors: PEOS_EINVAL. */
int peos_index_layout(const peos_index* index, peos_layout* out);

/* Release a handle (host memory only; device buffers belong to the caller). */
void peos_free(peos_index* index);

/*
 * peos_set_upper_layers -- give the index HNSW-style upper layers, so that
 * every search starts from the node a greedy descent through them reaches
 * instead of the fixed entry.  Implements the entry of Alg. 1 on the
 * hierarchical graphs the experiments use (HNSW): in each upper layer, from
 * the current node, move to the closest of its neighbours in that layer
 * (distance, then id) while it is closer than the current node, then
 * continue from the same node one layer below; the node reached in the
 * lowest upper layer is v0.  The descent runs on the GPU before the search
 * (kernel k_descend), with the search's distances; its distance count goes
 * to PEOS_STAT_DESCENT.
 * Layout: the rows of all upper layers together, layer 1 (the lowest upper
 * layer) first; layer l is rows [layer_start[l-1], layer_start[l]).
 *   node (device, rows int32)     base id of row r, in [0, n)
 *   adj  (device, rows x R int32) rows of r's neighbours in r's own layer,
 *                                  -1 = none; no self loop
 *   down (device, rows int32)     row of the same node in the layer below,
 *                                  -1 for the rows of layer 1
 *   layer_start (host, levels + 1 int64), top = the starting row (in the
 *   top layer).
 * The arrays are not copied (the caller keeps them alive while the index
 * uses them); they are checked once here (synchronously, through a host
 * copy): ranges, same-layer adjacency, `down` onto the same node one layer
 * lower.  layers = NULL removes the upper layers.
 * Errors: PEOS_EINVAL (bad sizes, levels not in [1, 32], R not in [1, 64],
 * a check above fails), PEOS_EHIP.
 */
typedef struct {
    int32_t levels;
    int32_t R;
    int64_t rows;
    int64_t top;
    const int64_t* layer_start; /* host */
    const int32_t* node;        /* device */
    const int32_t* adj;         /* device */
    const int32_t* down;        /* device */
} peos_upper_layers;

int peos_set_upper_layers(peos_index* index, const peos_upper_layers* layers);

/*
 * peos_query_tables -- PEOs step (5): the per-query projection table, built
 * once per query (Alg. 2, "only once and used throughout the search").
 *   queries  nq x d float, 16-byte aligned.
 *   tables   out, nq x (L+1) x m float: row 0 = q'.b_j, row i = q'_i . a^i_j
 *            with q' = q/|q| and q'_i its i-th block (not renormalized);
 *            IEEE halves (nq x (L+1) x m x 2 bytes) if the index has
 *            PEOS_FLAG_FP16.
 *   qnorms   out, nq float: |q| (0 for a zero query, whose table is 0).
 * Runs the dense query-by-direction product on the matrix cores.
 * Errors: PEOS_EINVAL (null pointer with nq > 0, nq < 0, queries not 16-byte
 * aligned), PEOS_EHIP.
 */
int peos_query_tables(const peos_index* index, const float* queries, int64_t nq, float* tables,
                      float* qnorms, void* stream);

/*
 * peos_search_ws_bytes -- workspace of peos_search / peos_search_tables for
 * nq queries with list sizes up to efmax and candidate-pool capacity `pool`
 * (as in peos_search): per query the projection table, norm, class order and
 * descent entry, and per resident workgroup (at most min(nq, 4096)) a spill
 * region for queries whose visited set outgrows the LDS hash (a bitmap of n
 * bits and, from n = 2^19 on, a list of 4,096 ids).  Output *ws_bytes
 * (host).  Errors: PEOS_EINVAL.
 */
int peos_search_ws_bytes(const peos_index* index, int64_t nq, int32_t efmax, int32_t pool,
                         size_t* ws_bytes);

/*
 * peos_search_tables -- Alg. 1 with the PEOs test (steps (4) and (6), Alg. 2)
 * for nq queries whose tables come from peos_query_tables.
 *   queries, tables, qnorms  as produced/consumed by peos_query_tables.
 *   k, ef    per-query int32 arrays (device), or NULL to use k_all / ef_all
 *            for every query.  The effective list size is max(ef, k) (efs >= K
 *            in Sec. 3).  1 <= k <= kstride, ef <= 4096.
 *   kstride  row stride (entries) of ids/dists.
 *   pool     capacity of the candidate list (R plus the queue P of Alg. 1,
 *            held as one list sorted by (distance, id)).  pool = 0: the queue
 *            is unbounded as printed in Alg. 1, up to the kernel's capacity
 *            (a query that reaches it gets PEOS_STATUS_POOL_FULL and from then
 *            on behaves as pool = that capacity); 0 < pool <= max(ef, k): the
 *            HNSW stopping rule (stop when R holds no unexpanded node);
 *            pool > max(ef, k): a bounded queue of pool entries; pool in
 *            [-16, -1]: a bounded queue of |pool| x (that query's list size)
 *            entries, at most 8192.
 *   eps      error bound epsilon of probabilistic routing (Def. 3.2), in
 *            (0, 0.5]; ignored by EXHAUSTIVE.
 *   mode     PEOS_MODE_* (SIMHASH needs PEOS_FLAG_SIMHASH).
 *   ids      out, nq x kstride int64: first k results ordered by (distance,
 *            id), then -1.
 *   dists    out, nq x kstride float: their distances (squared l2,
 *            1 - x.q/|q|, or -x.q), then +inf.
 *   stats    out, nq x PEOS_NSTATS int32, or NULL.
 *   ws       workspace of peos_search_ws_bytes(index, nq, efmax, pool).
 * Launch: with per-query ef (ef != NULL) the batch is split on the device
 * into classes of effective list size (<= 32, <= 64, ..., doubling, the last
 * class up to max(ef_all, k_all)), and each class runs as its own persistent
 * launch whose LDS plan fits its largest list, largest class first; results
 * do not depend on the split.
 * Search semantics (where the paper leaves a choice): the entry node is
 * distance-computed and visited first; delta is read once per expansion;
 * a neighbour is visited only once its distance is computed; a survivor
 * enters the list if R was not full or its distance is < delta.
 * Errors: PEOS_EINVAL (also when the list and visited set of the largest
 * list size do not fit the 64 KB of LDS one workgroup may use: about ef =
 * 3000 under the HNSW rule, 2048 with the unbounded queue), PEOS_ENOSPACE,
 * PEOS_EHIP.
 */
int peos_search_tables(const peos_index* index, const float* queries, const float* tables,
                       const float* qnorms, int64_t nq, const int32_t* k, const int32_t* ef,
                       int32_t k_all, int32_t ef_all, int32_t kstride, int32_t pool, float eps,
                       int32_t mode, int64_t* ids, float* dists, int32_t* stats, void* ws,
                       size_t ws_bytes, void* stream);

/*
 * peos_search -- peos_query_tables followed by peos_search_tables, with the
 * tables and norms kept in the workspace.  Arguments as above; ws must hold
 * peos_search_ws_bytes(index, nq, efmax, pool) bytes.
 */
int peos_search(const peos_index* index, const float* queries, int64_t nq, const int32_t* k,
                const int32_t* ef, int32_t k_all, int32_t ef_all, int32_t kstride, int32_t pool,
                float eps, int32_t mode, int64_t* ids, float* dists, int32_t* stats, void* ws,
                size_t ws_bytes, void* stream);

/*
 * peos_search_static -- peos_search without a workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops
 * that must not call hipMalloc, harnesses that forbid it).  Arguments,
 * results and errors are those of peos_search, minus ws / ws_bytes.
 * The workspace is a device array inside the library of
 * PEOS_STATIC_SCRATCH_BYTES bytes, one per device, held until the process
 * ends; the call allocates nothing.  Its per-query part (projection tables,
 * norms, class order, descent entries: about ((L+1) m + 3) x 4 bytes per
 * query) must fit in it with one workgroup's spill region (the visited
 * bitmap, n/8 bytes, and from n = 2^19 on a 16 KB list of the ids a spilled
 * query set), else the call returns PEOS_ENOSPACE before any work is
 * enqueued; the rest holds the spill regions of the resident workgroups,
 * so a large n limits how many queries run at once (speed only, never
 * results).  Every call on a device
 * uses that device's one array: calls that overlap on one device (other
 * streams or threads, or a captured call replayed while another runs) race
 * and must be serialised by the caller.  The array keeps the last call's
 * contents; every call writes what it reads before reading it.
 */
#define PEOS_STATIC_SCRATCH_BYTES (64u << 20)
int peos_search_static(const peos_index* index, const float* queries, int64_t nq,
                       const int32_t* k, const int32_t* ef, int32_t k_all, int32_t ef_all,
                       int32_t kstride, int32_t pool, float eps, int32_t mode, int64_t* ids,
                       float* dists, int32_t* stats, void* stream);

/*
 * Launch plan of an index's searches.  The plan changes speed only, never a
 * result (except through the list capacity with pool = 0, see listcap); it
 * belongs to the index: overrides set here apply to every later search on
 * that index (peos_search, peos_search_tables, captured graphs created
 * afterwards, servers over it) and to no other index.  Not to be called while
 * another thread searches the same index.
 *
 * peos_set_search_tuning -- overrides for every launch (0 keeps the
 * automatic choice):
 *   hash_cap   visited-hash capacity in LDS, 64..16384 entries (rounded down
 *              to a multiple of 4); a query that visits more than 7/8 of it
 *              moves its visited set to a bitmap in the workspace
 *              (PEOS_STATUS_VISITED_SPILL);
 *   listcap    candidate-list capacity in LDS (rounded up to a multiple of 64
 *              and to at least max(pool, ef)); with pool = 0 it is the
 *              kernel capacity that PEOS_STATUS_POOL_FULL refers to.  Setting
 *              it also keeps the list in LDS where it would otherwise live in
 *              registers (capacity = ef <= 64);
 *   slots      resident workgroups of the persistent grid, 1..4096;
 *   waves      wavefronts per query, 1, 2 or 4 (0 automatic: 4 or 2 when
 *              every query of the batch can still be resident at once,
 *              else 1).  One workgroup of that many waves searches a query:
 *              wave 0 runs the search and all of them gather the survivor
 *              rows, each row still reduced by one wave in the fixed order,
 *              so results do not depend on it.
 * Errors: PEOS_EINVAL for a null index or values out of range.
 */
int peos_set_search_tuning(peos_index* index, int32_t hash_cap, int32_t listcap, int32_t slots,
                           int32_t waves);

/*
 * peos_set_long_rows -- allow (1, the default) or forbid (0) the search
 * kernel's long-vector variant for later searches on this index.  The
 * variant is chosen for d > 512 and L > 8 with the list in LDS when at most
 * 8 waves per CU would be resident anyway (the list and visited hash fill
 * the LDS share of more, or the batch is at most 8 queries per CU): it may
 * use the registers of two waves per SIMD and gathers 8 rows of up to 1024
 * coordinates per round trip, in the same fixed summation order, so results
 * do not depend on it.  Errors: PEOS_EINVAL for a null index or other values.
 */
int peos_set_long_rows(peos_index* index, int32_t enable);

/*
 * peos_set_class_tuning -- overrides of one ef class of a split batch (see
 * peos_search_tables; class c holds lists of size <= 32 << c, c in [0, 8)):
 * visited-hash capacity, resident workgroups and waves per query as in
 * peos_set_search_tuning, 0 = automatic.  They take precedence over
 * peos_set_search_tuning's for that class.  Errors: PEOS_EINVAL for a null
 * index or values out of range.
 */
int peos_set_class_tuning(peos_index* index, int32_t cls, int32_t hash_cap, int32_t slots,
                          int32_t waves);
/*
 * peos_graph_create -- capture one peos_search call (projection tables,
 * class split and search launches; no memset nodes) into an executable HIP
 * graph, so that a batch of the same shape is issued with one launch.
 * Arguments as for peos_search; every pointer is baked into the graph, so the
 * caller refills queries (and k, ef) in place between launches and reads
 * ids/dists/stats after each.  The index's launch plan in effect at capture
 * time is frozen in the graph.  Output *out (host); release with peos_graph_destroy.
 * Errors: as peos_search, PEOS_EINVAL for nq = 0, PEOS_EHIP if capture or
 * instantiation fails.
 */
int peos_graph_create(const peos_index* index, const float* queries, int64_t nq, const int32_t* k,
                      const int32_t* ef, int32_t k_all, int32_t ef_all, int32_t kstride,
                      int32_t pool, float eps, int32_t mode, int64_t* ids, float* dists,
                      int32_t* stats, void* ws, size_t ws_bytes, peos_graph** out);
/* Launch a captured search on `stream` (asynchronous).  Errors: PEOS_EINVAL,
 * PEOS_EHIP.  Launches of one graph must not overlap (they share the
 * workspace). */
int peos_graph_launch(peos_graph* graph, void* stream);
/* Release a captured search. */
void peos_graph_destroy(peos_graph* graph);
/*
 * Serving form: a request loop with continuous batching over one index.
 * Unlike the calls above, a server allocates: device buffers for each launch
 * slot (hipMalloc) and pinned host staging (hipHostMalloc), at open time.
 *
 * Requests of 1..max_batch queries, each request with its own k and ef, wait
 * in a FIFO.  Whenever one of the server's launch slots is free, the longest
 * prefix of the FIFO that fits max_batch queries becomes one batch (per-query
 * k and ef) and is issued on that slot's stream: copy in, projection tables
 * (peos_query_tables), ef-class split and search (peos_search_tables), copy
 * out.  Batches on different slots overlap on the device, so requests that
 * arrive while others are running start as soon as a slot and LDS free up.
 * Admission: a batch is issued only while the LDS held by its resident waves
 * plus that of the batches in flight fits lds_budget; the HBM budget caps the
 * number of slots at open time; submit refuses work beyond max_pending
 * queued queries (PEOS_EBUSY).  A query's result does not depend on the
 * batch it ran in.  Single-threaded: one thread drives a server.
 */
typedef struct peos_server peos_server;
typedef struct {
    int32_t max_batch;    /* queries per launch, and per request             */
    int32_t max_k;        /* largest k of a request                          */
    int32_t max_ef;       /* largest ef of a request (ef := max(ef, k))      */
    int32_t max_inflight; /* launch slots (streams), 1..16                    */
    int32_t max_pending;  /* queued queries before submit returns PEOS_EBUSY  */
    int32_t pool;         /* stopping rule for all requests, as peos_search  */
    int32_t mode;         /* PEOS_MODE_*                                     */
    int32_t launch_waves; /* resident waves one launch may hold, 0 = all     */
    float eps;            /* in (0, 0.5] for PEOS_MODE_PEOS                  */
    float reserved;
    size_t hbm_budget;    /* device bytes for all slots, 0 = no limit        */
    size_t lds_budget;    /* LDS bytes of all launches in flight, 0 = device */
} peos_serve_config;
/* Open a server on the current device (the index's).  *out (host).  Errors:
 * PEOS_EINVAL (config out of range), PEOS_ENOSPACE (not one slot fits
 * hbm_budget), PEOS_EHIP (allocation), PEOS_EDEVICE. */
int peos_serve_open(const peos_index* index, const peos_serve_config* cfg, peos_server** out);
/* Queue a request: queries (host, nq x d float), k, ef; the results are
 * written to ids (host, nq x k int64) and dists (host, nq x k float) when the
 * request completes (see peos_serve_poll); all three buffers must stay valid
 * until then.  *ticket (host) identifies the request.  May issue batches.
 * Errors: PEOS_EINVAL, PEOS_EBUSY (queue full, nothing queued), PEOS_EHIP. */
int peos_serve_submit(peos_server* server, const float* queries, int32_t nq, int32_t k, int32_t ef,
                      int64_t* ids, float* dists, uint64_t* ticket);
/* Progress: collect finished batches (their requests' results are copied
 * out), issue waiting requests on free slots, and return up to max_done
 * tickets of completed requests in done (host), their count in *n_done.
 * wait != 0: if nothing has completed, block until the oldest batch in flight
 * does.  Errors: PEOS_EINVAL, PEOS_EHIP. */
int peos_serve_poll(peos_server* server, int32_t wait, uint64_t* done, int32_t max_done,
                    int32_t* n_done);
/* Eight counters (host int64): launches, requests completed, queries
 * completed, largest batch, batches in flight, queries waiting, launch slots,
 * LDS bytes in flight.  Errors: PEOS_EINVAL. */
int peos_serve_counters(const peos_server* server, int64_t* out);
/* Wait for the work in flight and release the server (requests still queued
 * are dropped). */
void peos_serve_close(peos_server* server);
/* Message for a return code, and the thread-local message of the last error. */
/*
 * peos_probe_gather -- calibration, not part of the search: `waves` waves
 * each gather `iters` x 16 random 512-byte rows of `rows` (n_rows x 128
 * float, 16-byte aligned) the way the search gathers survivor rows (8 lanes
 * per row, 16 rows in flight per wave), and write one checksum per wave to
 * sink (waves floats).  Asynchronous on `stream`; the caller times it.  It
 * gives the practical HBM ceiling of the search's access pattern (the
 * roofline's denominator is the nominal 8 TB/s).
 * Errors: PEOS_EINVAL, PEOS_EDEVICE, PEOS_EHIP.
 */
int peos_probe_gather(const float* rows, int64_t n_rows, int32_t waves, int32_t iters,
                      float* sink, void* stream);

const char* peos_strerror(int code);
const char* peos_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PEOS_H */
