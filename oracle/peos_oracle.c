/*
 * PEOs oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar CPU implementation of what the PEOs-routed graph
 * search computes (Lu, Xiao, Ishikawa, "Probabilistic Routing for
 * Graph-Based Approximate Nearest Neighbor Search", ICML 2024).  It exists to
 * check the HIP library and shares no code with it.  Only the test suite, the
 * smoke entry and the CPU-baseline leg of the benchmark may load it.
 *
 * Arithmetic is double precision, except for the one place where floating
 * point decides an integer: the edge codes of PEOs step (3) are argmaxes, and
 * they are decided in single precision with the fixed operation order given
 * in edge_codes_fp32() below -- the precision the GPU builder uses -- so both
 * sides take the same integer decisions.
 *
 * Paper sections followed:
 *   - Alg. 1 (graph-based ANNS with routing) and its text in Sec. 3;
 *   - Sec. 4.2 "PEOs Test", steps (1)-(6), and Alg. 2;
 *   - the residual-edge remedy of Sec. 4.1 (test on e = u - v, q normalized);
 *   - Appendix "Extension to MIPS" for the angular numerator.
 * Readings where the paper is silent (visited-on-distance, delta snapshot per
 * expansion, (dist, id) order, single sorted list with expanded flags,
 * zero-block handling, closed-form quantile) are stated where they apply.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_L2 0
#define OR_ANGULAR 1
#define OR_IP 2 /* maximum inner product: dist = -x.q (appendix, Extension to MIPS) */
#define OR_MODE_PEOS 0
#define OR_MODE_EXHAUSTIVE 1
#define OR_MODE_SIMHASH 2

/* counters, per query */
enum {
    C_EXPANSIONS = 0, /* nodes popped and expanded                        */
    C_EDGES,          /* valid neighbour ids enumerated                   */
    C_VISITED_SKIPS,  /* neighbours skipped because already visited       */
    C_TESTS,          /* PEOs tests run (R full, neighbour unvisited)     */
    C_TEST_GE1,       /* tests decided by A >= 1 (fail)                   */
    C_TEST_LE0,       /* tests decided by A <= 0 (pass)                   */
    C_TEST_H,         /* tests decided by H >= T                          */
    C_TEST_ZERO,      /* tests on a zero-length edge (decided by sign)    */
    C_PASSES,         /* tests that passed                                */
    C_NDIST,          /* exact distances computed (entry included)        */
    C_INSERTED,       /* distances that entered the merge                 */
    C_TEST_EXPANSIONS,/* expansions with R full under a routing test      */
    C_NCOUNT
};

/* fragile-decision flags, per query */
#define F_HT 1     /* |H - T| tiny                                     */
#define F_A1 2     /* A close to 1                                     */
#define F_A0 4     /* A close to 0                                     */
#define F_DELTA 8  /* d_u close to delta                               */
#define F_ORDER 16 /* two list entries with nearly equal distances     */

/* ------------------------------------------------------------------ */
/* inverse standard normal CDF, by bisection on the CDF written with erfc */
/* ------------------------------------------------------------------ */
static double norm_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

double oracle_norm_ppf(double p)
{
    if (!(p > 0.0) || !(p < 1.0)) return NAN;
    double lo = -40.0, hi = 40.0;
    for (int it = 0; it < 400; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (norm_cdf(mid) < p) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi);
}

/* ------------------------------------------------------------------ */
/* Steps (1)-(3): one edge record                                      */
/* ------------------------------------------------------------------ */

/*
 * Codes of PEOs step (3), decided in single precision.  Operation order:
 *   e_k   = x_u[k] - x_v[k]
 *   s_i   = sqrtf(sum_k e_k*e_k)         (fmaf chain over the block, k ascending)
 *   p_ij  = sum_t e_{i,t} * a^i_j[t]     (fmaf chain, t ascending, from 0)
 *   code_i: j* = first j maximizing |p_ij|; sign negative iff p_ij* < 0
 *   L'    = number of blocks with s_i > 0
 *   c     = (s_1 + ... + s_L) / L'       (sequential adds, one divide)
 *   r_i   = c / s_i  (0 when s_i == 0)
 *   eres_k = fmaf(-r_i, e_k, e_k)
 *   code_0 as code_i, over eres and the full-space vectors b_j (fmaf chain
 *          over k = 0..d-1).
 * The encoding is (j* - 1) + m * [sign < 0] with j* counted from 1, i.e. a
 * byte in [0, 2m).  Block 0 is the residual code e[0], blocks 1..L are e[i].
 * margin[i] returns the relative gap between the two largest |p| (a near-tie
 * diagnostic only).
 */
/* ------------------------------------------------------------------ */
/* Storage roundings of the precision form                              */
/* ------------------------------------------------------------------ */
/*
 * Nearest IEEE binary16 value of x (ties to even), as a double: 11
 * significant bits for |x| >= 2^-14, a fixed step of 2^-24 below (subnormal
 * numbers), and infinity from 65520 on (the first value that rounds past the
 * largest finite half, 65504).  rint() rounds to nearest even.
 */
double oracle_round_half(double x)
{
    if (!isfinite(x) || x == 0.0) return x;
    const double ax = fabs(x);
    double r;
    if (ax < ldexp(1.0, -14)) {
        r = rint(ax * ldexp(1.0, 24)) * ldexp(1.0, -24);
    } else {
        int e;
        frexp(ax, &e);                  /* ax = f * 2^e, f in [0.5, 1) */
        const double ulp = ldexp(1.0, e - 11);
        r = rint(ax / ulp) * ulp;
        if (r > 65504.0) r = INFINITY;
    }
    return x < 0 ? -r : r;
}

/* Nearest bfloat16 value of a float (ties to even): the float's upper 16
 * bits after rounding its lower 16 bits away. */
float oracle_round_bf16(float x)
{
    uint32_t u;
    memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return x; /* inf, nan */
    u += 0x7fffu + ((u >> 16) & 1u);
    u &= 0xffff0000u;
    float r;
    memcpy(&r, &u, 4);
    return r;
}

static void edge_codes_fp32(const float* xv, const float* xu, int d, int L, int m,
                            const float* A, const float* B, float* ework, float* eres,
                            uint8_t* codes, double* margin)
{
    const int dp = d / L;
    float s[256];
    for (int k = 0; k < d; ++k) ework[k] = xu[k] - xv[k];
    int nonzero = 0;
    for (int i = 0; i < L; ++i) {
        float ss = 0.0f;
        for (int t = 0; t < dp; ++t) ss = fmaf(ework[i * dp + t], ework[i * dp + t], ss);
        s[i] = sqrtf(ss);
        if (s[i] > 0.0f) ++nonzero;
    }
    for (int i = 0; i < L; ++i) {
        int best = 0;
        float bv = -1.0f, second = -1.0f, bp = 0.0f;
        for (int j = 0; j < m; ++j) {
            const float* a = A + ((size_t)i * m + j) * dp;
            float p = 0.0f;
            for (int t = 0; t < dp; ++t) p = fmaf(ework[i * dp + t], a[t], p);
            float ap = fabsf(p);
            if (ap > bv) { second = bv; bv = ap; best = j; bp = p; }
            else if (ap > second) second = ap;
        }
        codes[1 + i] = (uint8_t)(best + (bp < 0.0f ? m : 0));
        if (margin) margin[1 + i] = bv > 0.0f ? (double)(bv - second) / (double)bv : 1.0;
    }
    float c = 0.0f;
    if (nonzero > 0) {
        float sum = 0.0f;
        for (int i = 0; i < L; ++i) sum = sum + s[i];
        c = sum / (float)nonzero;
    }
    for (int i = 0; i < L; ++i) {
        float r = s[i] > 0.0f ? c / s[i] : 0.0f;
        for (int t = 0; t < dp; ++t) {
            float ek = ework[i * dp + t];
            eres[i * dp + t] = fmaf(-r, ek, ek);
        }
    }
    {
        int best = 0;
        float bv = -1.0f, second = -1.0f, bp = 0.0f;
        for (int j = 0; j < m; ++j) {
            const float* b = B + (size_t)j * d;
            float p = 0.0f;
            for (int k = 0; k < d; ++k) p = fmaf(eres[k], b[k], p);
            float ap = fabsf(p);
            if (ap > bv) { second = bv; bv = ap; best = j; bp = p; }
            else if (ap > second) second = ap;
        }
        codes[0] = (uint8_t)(best + (bp < 0.0f ? m : 0));
        if (margin) margin[0] = bv > 0.0f ? (double)(bv - second) / (double)bv : 1.0;
    }
}

/*
 * Scalars of steps (1) and (6), in double precision, from the definitions.
 * Step (1): e = e_reg + e_res with e_reg the orthogonal projection of e on
 * the direction g = [e_i / (sqrt(L) |e_i|)]_i.  When every block is nonzero g
 * is a unit vector and w_reg = sum_i |e_i| / (sqrt(L) |e|); a zero block
 * contributes a zero component to g (the paper leaves this case open), and
 * the projection is still taken on the line spanned by g.
 * out[0] = |e|, out[1] = w_reg, out[2] = w_res, out[3] = |u|^2, out[4] = |v|^2.
 */
static void edge_scalars_fp64(const float* xv, const float* xu, int d, int L, double* ework,
                              double* out)
{
    const int dp = d / L;
    double s[256];
    double ne2 = 0.0, nu2 = 0.0, nv2 = 0.0;
    for (int k = 0; k < d; ++k) {
        ework[k] = (double)xu[k] - (double)xv[k];
        ne2 += ework[k] * ework[k];
        nu2 += (double)xu[k] * (double)xu[k];
        nv2 += (double)xv[k] * (double)xv[k];
    }
    for (int i = 0; i < L; ++i) {
        double ss = 0.0;
        for (int t = 0; t < dp; ++t) ss += ework[i * dp + t] * ework[i * dp + t];
        s[i] = sqrt(ss);
    }
    double ne = sqrt(ne2);
    double wreg = 1.0, wres = 0.0;
    if (ne > 0.0) {
        /* g and e.g, |g|^2 */
        double eg = 0.0, gg = 0.0;
        for (int i = 0; i < L; ++i) {
            if (s[i] <= 0.0) continue;
            for (int t = 0; t < dp; ++t) {
                double g = ework[i * dp + t] / (sqrt((double)L) * s[i]);
                eg += ework[i * dp + t] * g;
                gg += g * g;
            }
        }
        /* e_reg = (e.g / g.g) g ; e_res = e - e_reg */
        double nreg2 = 0.0, nres2 = 0.0;
        for (int i = 0; i < L; ++i) {
            for (int t = 0; t < dp; ++t) {
                double g = s[i] > 0.0 ? ework[i * dp + t] / (sqrt((double)L) * s[i]) : 0.0;
                double ereg = (eg / gg) * g;
                double eres = ework[i * dp + t] - ereg;
                nreg2 += ereg * ereg;
                nres2 += eres * eres;
            }
        }
        wreg = sqrt(nreg2) / ne;
        wres = sqrt(nres2) / ne;
    }
    out[0] = ne;
    out[1] = wreg;
    out[2] = wres;
    out[3] = nu2;
    out[4] = nv2;
}

typedef struct {
    uint8_t codes[257];
    double norm_e, w_reg, w_res, nu2, nv2;
    double margin_min;
} edge_rec;

static void edge_record(const float* xv, const float* xu, int d, int L, int m, const float* A,
                        const float* B, float* fw1, float* fw2, double* dw, edge_rec* r)
{
    double margin[257];
    edge_codes_fp32(xv, xu, d, L, m, A, B, fw1, fw2, r->codes, margin);
    double sc[5];
    edge_scalars_fp64(xv, xu, d, L, dw, sc);
    r->norm_e = sc[0];
    r->w_reg = sc[1];
    r->w_res = sc[2];
    r->nu2 = sc[3];
    r->nv2 = sc[4];
    double mm = 1.0;
    for (int i = 0; i <= L; ++i) if (margin[i] < mm) mm = margin[i];
    r->margin_min = mm;
}

/*
 * Public: records of every edge of a graph.  codes: n*R*(L+1) bytes, edge
 * (v, j) at [(v*R + j)*(L+1) + i], i = 0 residual code, 1..L block codes.
 * scal: n*R*4 doubles {|e|, w_reg, w_res, g_e = (|u|^2 - |v|^2)/2}.
 * margin: n*R doubles.  Padding edges (id < 0) are left zero.
 */
typedef struct {
    const float *base, *A, *B;
    const int32_t* graph;
    int64_t n, v0, v1;
    int d, R, L, m;
    uint8_t* codes;
    double *scal, *margin;
} build_job;

static void* build_worker(void* arg)
{
    build_job* j = (build_job*)arg;
    float* fw1 = (float*)malloc(sizeof(float) * j->d);
    float* fw2 = (float*)malloc(sizeof(float) * j->d);
    double* dw = (double*)malloc(sizeof(double) * j->d);
    edge_rec r;
    for (int64_t v = j->v0; v < j->v1; ++v) {
        for (int e = 0; e < j->R; ++e) {
            int32_t u = j->graph[v * j->R + e];
            size_t idx = (size_t)v * j->R + e;
            if (u < 0) continue;
            edge_record(j->base + (size_t)v * j->d, j->base + (size_t)u * j->d, j->d, j->L, j->m,
                        j->A, j->B, fw1, fw2, dw, &r);
            memcpy(j->codes + idx * (j->L + 1), r.codes, (size_t)j->L + 1);
            j->scal[idx * 4 + 0] = r.norm_e;
            j->scal[idx * 4 + 1] = r.w_reg;
            j->scal[idx * 4 + 2] = r.w_res;
            j->scal[idx * 4 + 3] = 0.5 * (r.nu2 - r.nv2);
            if (j->margin) j->margin[idx] = r.margin_min;
        }
    }
    free(fw1);
    free(fw2);
    free(dw);
    return NULL;
}

int oracle_build_tables(const float* base, int64_t n, int d, const int32_t* graph, int R, int L,
                        int m, const float* A, const float* B, uint8_t* codes, double* scal,
                        double* margin, int nthreads)
{
    if (L <= 0 || d % L || L > 255 || m <= 0 || 2 * m > 256 || d / L > 4096) return -1;
    if (nthreads < 1) nthreads = 1;
    memset(codes, 0, (size_t)n * R * (L + 1));
    memset(scal, 0, sizeof(double) * (size_t)n * R * 4);
    if (margin) memset(margin, 0, sizeof(double) * (size_t)n * R);
    pthread_t th[256];
    build_job jobs[256];
    if (nthreads > 256) nthreads = 256;
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (build_job){base, A, B, graph, n, n * t / nthreads, n * (t + 1) / nthreads,
                              d, R, L, m, codes, scal, margin};
        pthread_create(&th[t], NULL, build_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* Public: one edge record (tests). scal as in oracle_build_tables. */
int oracle_edge_record(const float* xv, const float* xu, int d, int L, int m, const float* A,
                       const float* B, uint8_t* codes, double* scal, double* margin_min)
{
    if (L <= 0 || d % L || L > 255 || 2 * m > 256) return -1;
    float* fw1 = (float*)malloc(sizeof(float) * d);
    float* fw2 = (float*)malloc(sizeof(float) * d);
    double* dw = (double*)malloc(sizeof(double) * d);
    edge_rec r;
    edge_record(xv, xu, d, L, m, A, B, fw1, fw2, dw, &r);
    memcpy(codes, r.codes, (size_t)L + 1);
    scal[0] = r.norm_e;
    scal[1] = r.w_reg;
    scal[2] = r.w_res;
    scal[3] = 0.5 * (r.nu2 - r.nv2);
    if (margin_min) *margin_min = r.margin_min;
    free(fw1);
    free(fw2);
    free(dw);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Step (5): projection table of one query                             */
/* ------------------------------------------------------------------ */
/*
 * T[0][j] = q'.b_j and T[i][j] = q'_i . a^i_j (i = 1..L), q' = q/|q| and q'_i
 * the i-th block of q' (not renormalized: the combination in Sec. 5.1 needs
 * sum_i |q'_i|^2 = 1).  table: (L+1) x m doubles.
 */
void oracle_query_table(const float* q, int d, int L, int m, const float* A, const float* B,
                        double* table)
{
    const int dp = d / L;
    double qn = 0.0;
    for (int k = 0; k < d; ++k) qn += (double)q[k] * (double)q[k];
    qn = sqrt(qn);
    for (int j = 0; j < m; ++j) {
        double acc = 0.0;
        for (int k = 0; k < d; ++k) acc += ((double)q[k] / qn) * (double)B[(size_t)j * d + k];
        table[j] = acc;
    }
    for (int i = 0; i < L; ++i)
        for (int j = 0; j < m; ++j) {
            double acc = 0.0;
            for (int t = 0; t < dp; ++t)
                acc += ((double)q[i * dp + t] / qn) * (double)A[((size_t)i * m + j) * dp + t];
            table[(size_t)(1 + i) * m + j] = acc;
        }
}

/* signed table lookup for a code byte: sgn(e[i]) * T[i][|e[i]|] */
static double lookup(const double* table, int m, int i, uint8_t c)
{
    int j = c % m;
    double v = table[(size_t)i * m + j];
    return c >= m ? -v : v;
}

/* ------------------------------------------------------------------ */
/* Steps (4) and (6): the routing test                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    double eta;   /* sqrt(2 L ln m)                       */
    double c_eps; /* standard-normal eps-quantile          */
    double tau;   /* relative width of a fragile decision  */
    int L, m, metric;
} test_params;

/* precision-form flags (the library's index flags of the same values) */
#define LP_BF16_BASE 1  /* traversal distances on the bfloat16-rounded base  */
#define LP_FP16 2       /* edge scalars and projection tables stored as half */

/*
 * Threshold of step (4)/(6): the eps-quantile of
 * N(x sqrt(2 L ln m), w_reg^2 + L w_res^2 - L x^2/(L+1)), written in closed
 * form as mean + sd * Phi^{-1}(eps) (the normal quantile identity used in the
 * proof of the guarantee).  The paper reads it from a lookup table; the
 * closed form is that table's exact value.
 */
double oracle_threshold(double A, double w_reg, double w_res, int L, double eta, double c_eps)
{
    double var = w_reg * w_reg + (double)L * w_res * w_res - (double)L * A * A / (double)(L + 1);
    return A * eta + c_eps * sqrt(var);
}

/*
 * Step (6) for edge e = (v, u) against the furthest result p.  num is the
 * numerator of A_r written as in the paper: |u|^2/2 - r - v.q with
 * r = |p|^2/2 - p.q for l2, and with the two squared norms removed for the
 * angular and inner-product metrics (= p.q - v.q, the form the appendix gives
 * for MIPS, p the result of smallest inner product).  A_r = num / (|q| |e|).
 * Returns 1 = pass, 0 = fail.  kind: 0 zero-length edge, 1 A>=1, 2 A<=0,
 * 3 H-vs-T.  flags receives the fragile bits of this decision.
 */
static int routing_test(const test_params* tp, const edge_rec* er, const double* table,
                        double num, double qnorm, double* outA, double* outH, double* outT,
                        int* kind, int* flags, int num_exact)
{
    const double tau = tp->tau;
    *outA = NAN;
    *outH = NAN;
    *outT = NAN;
    /* num_exact: the sign of the numerator is the same in any precision (see
       numerator_is_exact), so A_r near 0 is not a fragile decision */
    const int exact0 = num_exact;
    if (er->norm_e == 0.0) {
        *kind = 0;
        if (!exact0 && fabs(num) <= tau * fabs(qnorm)) *flags |= F_A0;
        return num < 0.0;
    }
    double A = num / (qnorm * er->norm_e);
    *outA = A;
    if (fabs(A - 1.0) < tau) *flags |= F_A1;
    if (!exact0 && fabs(A) < tau) *flags |= F_A0;
    if (A >= 1.0) { *kind = 1; return 0; }
    if (A <= 0.0) { *kind = 2; return 1; }
    *kind = 3;
    double H1 = 0.0;
    for (int i = 1; i <= tp->L; ++i) H1 += lookup(table, tp->m, i, er->codes[i]);
    double H2 = lookup(table, tp->m, 0, er->codes[0]);
    double H = er->w_reg * H1 + sqrt((double)tp->L) * er->w_res * H2;
    double T = oracle_threshold(A, er->w_reg, er->w_res, tp->L, tp->eta, tp->c_eps);
    *outH = H;
    *outT = T;
    if (fabs(H - T) < tau * (fabs(H) + fabs(T) + 1e-30)) *flags |= F_HT;
    return H >= T;
}

/*
 * Step (6) in the precision form.  The edge's scalars are stored as halves:
 * gp = g_e / |e| with g_e = (|u|^2 - |v|^2)/2 (0 for angular), ie = 1/|e|,
 * wr = w_reg, sr = sqrt(L) w_res, each the nearest half of its exact value;
 * the table entries are the nearest halves of the exact table.  The
 * numerator of A_r is taken from the search's own distances, which is the
 * same quantity: |u|^2/2 - r - v.q = g_e + (dist_v - delta)/2 for squared
 * l2, (dist_v - delta) |q| for angular with dist = 1 - x.q/|q|, and
 * dist_v - delta for the inner product with dist = -x.q; so A_r = (gp +
 * (dist_v - delta)/2 * ie) / |q|, (dist_v - delta) * ie, or (dist_v - delta)
 * * ie / |q| respectively.  An edge whose 1/|e| is not finite
 * as a half (|e| = 0, or below the half range) is decided by the sign of the
 * numerator, as a zero-length edge.
 */
static int routing_test_lowp(const test_params* tp, const edge_rec* er, const double* table16,
                             double dv, double delta, double qnorm, double* outA, double* outH,
                             double* outT, int* kind, int* flags, int v_is_p)
{
    const double tau = tp->tau;
    const int L = tp->L;
    *outA = NAN;
    *outH = NAN;
    *outT = NAN;
    const double diff = tp->metric == OR_L2 ? 0.5 * (dv - delta) : (dv - delta);
    const double ie = er->norm_e > 0.0 ? oracle_round_half(1.0 / er->norm_e) : INFINITY;
    const int exact0 = v_is_p && tp->metric != OR_L2;
    if (!isfinite(ie)) {
        *kind = 0;
        if (!v_is_p && fabs(diff) <= tau * (fabs(dv) + fabs(delta))) *flags |= F_A0;
        return diff < 0.0;
    }
    const double gp = tp->metric == OR_L2
                          ? oracle_round_half(0.5 * (er->nu2 - er->nv2) / er->norm_e) : 0.0;
    const double wr = oracle_round_half(er->w_reg);
    const double sr = oracle_round_half(sqrt((double)L) * er->w_res);
    const double A = tp->metric == OR_ANGULAR ? diff * ie : (gp + diff * ie) / qnorm;
    *outA = A;
    if (fabs(A - 1.0) < tau) *flags |= F_A1;
    if (!exact0 && fabs(A) < tau) *flags |= F_A0;
    if (A >= 1.0) { *kind = 1; return 0; }
    if (A <= 0.0) { *kind = 2; return 1; }
    *kind = 3;
    double H1 = 0.0;
    for (int i = 1; i <= L; ++i) H1 += lookup(table16, tp->m, i, er->codes[i]);
    const double H2 = lookup(table16, tp->m, 0, er->codes[0]);
    const double H = wr * H1 + sr * H2;
    const double var = wr * wr + sr * sr - (double)L * A * A / (double)(L + 1);
    const double T = A * tp->eta + tp->c_eps * sqrt(var);
    *outH = H;
    *outT = T;
    if (fabs(H - T) < tau * (fabs(H) + fabs(T) + 1e-30)) *flags |= F_HT;
    return H >= T;
}

/* ------------------------------------------------------------------ */
/* SimHash test (Sec. 3, "SimHash Test", with the residual-edge remedy) */
/* ------------------------------------------------------------------ */
/*
 * Sign bits of nb random projections, decided in single precision with one
 * fixed order (an fmaf chain over the coordinates in increasing order):
 * bit i = [v . c_i >= 0].  bits receives (nb + 63) / 64 words.
 */
static void simhash_bits_fp32(const float* v, int d, const float* C, int nb, uint64_t* bits)
{
    for (int w = 0; w < (nb + 63) / 64; ++w) bits[w] = 0;
    for (int i = 0; i < nb; ++i) {
        float p = 0.0f;
        for (int k = 0; k < d; ++k) p = fmaf(v[k], C[(size_t)i * d + k], p);
        if (p >= 0.0f) bits[i >> 6] |= 1ull << (i & 63);
    }
}

/*
 * The test on e = u - v: A_r as in the PEOs test; A_r >= 1 fails, A_r <= 0
 * passes; otherwise the angle threshold is theta_r = arccos(A_r) (d_u < delta
 * iff the angle of e and q is below it), the collision count of nb sign
 * projections of e and q is Binomial(nb, 1 - theta/pi), and Hoeffding's
 * inequality gives the threshold that a boundary edge (theta = theta_r)
 * exceeds with probability >= 1 - eps:
 *   pass iff #Col >= nb (1 - theta_r / pi) - sqrt(nb ln(1/eps) / 2).
 */
static int routing_test_simhash(const test_params* tp, double norm_e, int col, int nb,
                                double num, double qnorm, double eps, int* kind, int* flags,
                                int num_exact)
{
    const double tau = tp->tau;
    const int exact0 = num_exact;
    if (norm_e == 0.0) {
        *kind = 0;
        if (!exact0 && fabs(num) <= tau * fabs(qnorm)) *flags |= F_A0;
        return num < 0.0;
    }
    const double A = num / (qnorm * norm_e);
    if (fabs(A - 1.0) < tau) *flags |= F_A1;
    if (!exact0 && fabs(A) < tau) *flags |= F_A0;
    if (A >= 1.0) { *kind = 1; return 0; }
    if (A <= 0.0) { *kind = 2; return 1; }
    *kind = 3;
    const double pi = 3.14159265358979323846;
    const double T = nb * (1.0 - acos(A) / pi) - sqrt(nb * log(1.0 / eps) / 2.0);
    if (fabs((double)col - T) < 1e-3) *flags |= F_HT;
    return (double)col >= T;
}

/* Public: sign bits (for the pins). */
void oracle_simhash_bits(const float* v, int d, const float* C, int nb, uint64_t* bits)
{
    simhash_bits_fp32(v, d, C, nb, bits);
}

/* ------------------------------------------------------------------ */
/* The compact form (experiments, "Indexing Cost" and "Scalability")   */
/* ------------------------------------------------------------------ */
/*
 * For L <= 4 the paper keeps per edge only the L sub-vector codes and two
 * one-byte scalars, and sets w_reg = 1, w_res = 0 for every edge (the
 * residual part is small at such L).  The test then reads
 *   H = sum_{i=1..L} sgn(e[i]) T_i[|e[i]|],
 *   T(A) = A eta + c_eps sqrt(1 - L A^2 / (L+1))   (step (6) with w = (1, 0)),
 * and takes T from a lookup table over A: Sec. 4.3 allows a quantile slightly
 * below the true one, which keeps the guarantee's direction because T grows
 * with A.
 *
 * Readings (the paper gives no byte format):
 *  - the two bytes of an edge carry g_e/|e| (l2 only: it combines |u|^2 with
 *    the node's |v|^2, the paper's "norm of u") and 1/|e| ("norm of e"), each
 *    an affine 8-bit code against a range kept once per node as four floats
 *    {g_lo, g_step, i_lo, i_step};
 *  - the codes are directed so that the test's A_r never exceeds the exact
 *    one: g_e/|e| is rounded down; 1/|e| is rounded to nearest and decoded
 *    half a step up when dist_v - delta < 0, half a step down otherwise, so
 *    (dist_v - delta)/|e| is never overestimated.  Code 255 of 1/|e| marks a
 *    zero-length edge, decided by the sign of the numerator;
 *  - the table has COMPACT_LUT_BINS bins over A in [0, 1); bin b holds
 *    T(b / bins) rounded down to single precision, the smallest T of the bin;
 *  - the integer codes are decided in single precision in this order:
 *    S_i = fmaf chain of e_k^2 over block i (k ascending, the test's
 *    coordinates), ne2 = S_1 + ... + S_L (sequential adds), ne = sqrtf(ne2);
 *    |x|^2 = fmaf chain of x_k^2 over the original coordinates, ascending;
 *    gp = (0.5f * (|u|^2 - |v|^2)) / ne (zero for angular and inner product);
 *    ie = 1.0f / ne; g_lo, g_hi, i_lo, i_hi = min / max over the node's edges
 *    with ne > 0; g_step = (g_hi - g_lo) / 255.0f, i_step = (i_hi - i_lo) /
 *    254.0f; cg = floorf((gp - g_lo) / g_step) in [0, 255], ci = rintf((ie -
 *    i_lo) / i_step) in [0, 254] (0 when the step is 0).
 */
#define LP_COMPACT 8
#define COMPACT_LUT_BINS 256
static double dot64(const float* a, const float* b, int d);
#define COMPACT_ZERO_EDGE 255

typedef struct {
    float glo, gstep, ilo, istep;
} compact_hdr;

static float sqnorm32(const float* x, int d)
{
    float acc = 0.0f;
    for (int k = 0; k < d; ++k) acc = fmaf(x[k], x[k], acc);
    return acc;
}

/* gp and ie of edge (v, u) with xv_t, xu_t on the test's coordinates; returns
   0 for a zero-length edge */
static int compact_values(const float* xv_t, const float* xu_t, float nv2, float nu2, int d,
                          int L, int metric, float* gp, float* ie)
{
    const int dp = d / L;
    float ne2 = 0.0f;
    for (int i = 0; i < L; ++i) {
        float ss = 0.0f;
        for (int t = 0; t < dp; ++t) {
            const float e = xu_t[i * dp + t] - xv_t[i * dp + t];
            ss = fmaf(e, e, ss);
        }
        ne2 = ne2 + ss;
    }
    const float ne = sqrtf(ne2);
    *gp = 0.0f;
    *ie = 0.0f;
    if (!(ne > 0.0f)) return 0;
    if (metric == OR_L2) *gp = (0.5f * (nu2 - nv2)) / ne;
    *ie = 1.0f / ne;
    return 1;
}

/* header of node v and the scalar codes of its R edges (padding edges 0);
   wv, wu: d floats of work space each */
static void compact_node(const float* base, int d, const int32_t* row, int R, int L, int metric,
                         const int32_t* perm, int32_t v, float* wv, float* wu, float* gpw,
                         float* iew, int* kindw, compact_hdr* h, uint8_t* cg, uint8_t* ci)
{
    const float* xv = base + (size_t)v * d;
    const float nv2 = sqnorm32(xv, d);
    for (int k = 0; k < d; ++k) wv[k] = perm ? xv[perm[k]] : xv[k];
    float glo = INFINITY, ghi = -INFINITY, ilo = INFINITY, ihi = -INFINITY;
    for (int j = 0; j < R; ++j) {
        const int32_t u = row[j];
        kindw[j] = 0;
        if (u < 0) continue;
        const float* xu = base + (size_t)u * d;
        for (int k = 0; k < d; ++k) wu[k] = perm ? xu[perm[k]] : xu[k];
        if (compact_values(wv, wu, nv2, sqnorm32(xu, d), d, L, metric, &gpw[j], &iew[j])) {
            kindw[j] = 1;
            if (gpw[j] < glo) glo = gpw[j];
            if (gpw[j] > ghi) ghi = gpw[j];
            if (iew[j] < ilo) ilo = iew[j];
            if (iew[j] > ihi) ihi = iew[j];
        } else {
            kindw[j] = 2;
        }
    }
    if (!(glo <= ghi)) glo = ghi = ilo = ihi = 0.0f; /* no edge of nonzero length */
    h->glo = glo;
    h->gstep = (ghi - glo) / 255.0f;
    h->ilo = ilo;
    h->istep = (ihi - ilo) / 254.0f;
    for (int j = 0; j < R; ++j) {
        cg[j] = 0;
        ci[j] = 0;
        if (kindw[j] == 2) ci[j] = COMPACT_ZERO_EDGE;
        if (kindw[j] != 1) continue;
        if (h->gstep > 0.0f) {
            float c = floorf((gpw[j] - glo) / h->gstep);
            cg[j] = (uint8_t)(c < 0.0f ? 0.0f : (c > 255.0f ? 255.0f : c));
        }
        if (h->istep > 0.0f) {
            float c = rintf((iew[j] - ilo) / h->istep);
            ci[j] = (uint8_t)(c < 0.0f ? 0.0f : (c > 254.0f ? 254.0f : c));
        }
    }
}

/* the quantile table: entry b = T(b / bins) with w_reg = 1, w_res = 0,
   rounded down to single precision */
void oracle_compact_lut(int L, int m, double eps, float* lut)
{
    const double eta = sqrt(2.0 * L * log((double)m));
    const double c_eps = oracle_norm_ppf(eps);
    for (int b = 0; b < COMPACT_LUT_BINS; ++b) {
        const double A = (double)b / COMPACT_LUT_BINS;
        const double t = oracle_threshold(A, 1.0, 0.0, L, eta, c_eps);
        float f = (float)t;
        if ((double)f > t) f = nextafterf(f, -INFINITY);
        lut[b] = f;
    }
}

/*
 * Step (6) in the compact form, on the decoded scalars and the traversal
 * distances dist_v, delta (A_r = (gp + diff ie) / |q| for l2 and inner
 * product, diff ie for angular, diff = (dist_v - delta)/2 for l2 and
 * dist_v - delta otherwise).  codes[1..L] are the sub-vector codes.
 */
static int routing_test_compact(const test_params* tp, const compact_hdr* h, uint8_t cg,
                                uint8_t ci, const uint8_t* codes, const double* table,
                                const float* lut, double dv, double delta, double qnorm,
                                double* outA, double* outH, double* outT, int* kind, int* flags,
                                int v_is_p)
{
    const double tau = tp->tau;
    *outA = NAN;
    *outH = NAN;
    *outT = NAN;
    const double diff = tp->metric == OR_L2 ? 0.5 * (dv - delta) : (dv - delta);
    if (ci == COMPACT_ZERO_EDGE) {
        *kind = 0;
        if (!v_is_p && fabs(diff) <= tau * (fabs(dv) + fabs(delta))) *flags |= F_A0;
        return diff < 0.0;
    }
    const double gp = tp->metric == OR_L2 ? (double)h->glo + (double)cg * (double)h->gstep : 0.0;
    const double ie = (double)h->ilo + ((double)ci + (diff < 0.0 ? 0.5 : -0.5)) * (double)h->istep;
    const double A = tp->metric == OR_ANGULAR ? diff * ie : (gp + diff * ie) / qnorm;
    const int exact0 = v_is_p && tp->metric != OR_L2;
    *outA = A;
    if (fabs(A - 1.0) < tau) *flags |= F_A1;
    if (!exact0 && fabs(A) < tau) *flags |= F_A0;
    if (A >= 1.0) { *kind = 1; return 0; }
    if (A <= 0.0) { *kind = 2; return 1; }
    *kind = 3;
    double H = 0.0;
    for (int i = 1; i <= tp->L; ++i) H += lookup(table, tp->m, i, codes[i]);
    const double x = A * COMPACT_LUT_BINS;
    int b = (int)floor(x);
    if (b > COMPACT_LUT_BINS - 1) b = COMPACT_LUT_BINS - 1;
    /* A within single-precision rounding of a bin edge: the GPU evaluates A
       with about eight roundings of 2^-24 relative to the magnitude of the
       terms of its numerator (the decodes, the product, the sum, 1/|q|), so
       a margin of 2^-20 of that magnitude covers it; inside it the two
       precisions may take neighbouring bins */
    const double amag = tp->metric == OR_ANGULAR ? fabs(diff * ie)
                                                 : (fabs(gp) + fabs(diff * ie)) / qnorm;
    if (fabs(x - floor(x + 0.5)) < ldexp(amag, -20) * COMPACT_LUT_BINS) *flags |= F_HT;
    const double T = (double)lut[b];
    *outH = H;
    *outT = T;
    if (fabs(H - T) < tau * (fabs(H) + fabs(T) + 1e-30)) *flags |= F_HT;
    return H >= T;
}

/* Public: compact records of a graph.  hdr: n x 4 floats {g_lo, g_step, i_lo,
   i_step}; cg, ci: n x R bytes.  perm optional.  Returns 0, or -1. */
int oracle_compact_tables(const float* base, int64_t n, int d, const int32_t* graph, int R, int L,
                          int metric, const int32_t* perm, float* hdr, uint8_t* cg, uint8_t* ci)
{
    if (n <= 0 || d <= 0 || R <= 0 || L <= 0 || L > 4 || d % L) return -1;
    float* wv = (float*)malloc(sizeof(float) * (size_t)d);
    float* wu = (float*)malloc(sizeof(float) * (size_t)d);
    float* gpw = (float*)malloc(sizeof(float) * (size_t)R);
    float* iew = (float*)malloc(sizeof(float) * (size_t)R);
    int* kw = (int*)malloc(sizeof(int) * (size_t)R);
    for (int64_t v = 0; v < n; ++v) {
        compact_hdr h;
        compact_node(base, d, graph + (size_t)v * R, R, L, metric, perm, (int32_t)v, wv, wu, gpw,
                     iew, kw, &h, cg + (size_t)v * R, ci + (size_t)v * R);
        hdr[4 * v + 0] = h.glo;
        hdr[4 * v + 1] = h.gstep;
        hdr[4 * v + 2] = h.ilo;
        hdr[4 * v + 3] = h.istep;
    }
    free(wv);
    free(wu);
    free(gpw);
    free(iew);
    free(kw);
    return 0;
}

/* Public: one compact test (pins).  hdr: 4 floats; codes: L+1 bytes (code 0
   unused); dv, delta: the traversal distances.  out = {A, H, T, kind}. */
int oracle_compact_test(const float* hdr, int cg, int ci, const uint8_t* codes, const float* q,
                        int d, int L, int m, const float* A, const float* B, int metric,
                        double eps, double dv, double delta, double* out)
{
    if (L <= 0 || L > 4 || d % L) return -1;
    double* table = (double*)malloc(sizeof(double) * (size_t)(L + 1) * m);
    float lut[COMPACT_LUT_BINS];
    oracle_query_table(q, d, L, m, A, B, table);
    oracle_compact_lut(L, m, eps, lut);
    test_params tp = {sqrt(2.0 * L * log((double)m)), oracle_norm_ppf(eps), 1e-5, L, m, metric};
    compact_hdr h = {hdr[0], hdr[1], hdr[2], hdr[3]};
    double a, hh, t;
    int kind, flags = 0;
    int pass = routing_test_compact(&tp, &h, (uint8_t)cg, (uint8_t)ci, codes, table, lut, dv,
                                    delta, sqrt(dot64(q, q, d)), &a, &hh, &t, &kind, &flags, 0);
    out[0] = a;
    out[1] = hh;
    out[2] = t;
    out[3] = kind;
    free(table);
    return pass;
}

/* ------------------------------------------------------------------ */
/* Optional dimension permutation (appendix "Dimension Permutation")   */
/* ------------------------------------------------------------------ */
/*
 * Avg(e_j) = mean over the graph's edges of the squared j-th coordinate of
 * e = x_u - x_v.  The dimensions are sorted by ascending Avg (ties: smaller
 * index first) and handed out in d/L rounds of L: in each round the next L
 * dimensions, in that order, go one each to the subspace with the largest
 * running sum of Avg among those not yet served this round (ties: smaller
 * subspace index).  perm[i*d' + t] = the dimension that subspace i received
 * in round t, i.e. coordinate t of sub-vector i of the permuted vector.
 * avg (optional, d doubles) receives Avg.  Returns 0, or -1 on bad arguments.
 */
int oracle_dimension_permutation(const float* base, int64_t n, int d, const int32_t* graph, int R,
                                 int L, int32_t* perm, double* avg_out)
{
    if (n <= 0 || d <= 0 || R <= 0 || L <= 0 || d % L) return -1;
    const int dp = d / L;
    double* avg = (double*)calloc((size_t)d, sizeof(double));
    int* order = (int*)malloc(sizeof(int) * (size_t)d);
    double* sum = (double*)calloc((size_t)L, sizeof(double));
    int* served = (int*)malloc(sizeof(int) * (size_t)L);
    int* fill = (int*)calloc((size_t)L, sizeof(int));
    int64_t ne = 0;
    for (int64_t v = 0; v < n; ++v)
        for (int r = 0; r < R; ++r) {
            const int32_t u = graph[(size_t)v * R + r];
            if (u < 0) continue;
            ++ne;
            for (int j = 0; j < d; ++j) {
                const double t = (double)base[(size_t)u * d + j] - (double)base[(size_t)v * d + j];
                avg[j] += t * t;
            }
        }
    for (int j = 0; j < d; ++j) avg[j] = ne > 0 ? avg[j] / (double)ne : 0.0;
    /* ascending Avg, ties by index (insertion sort: d is small) */
    for (int j = 0; j < d; ++j) order[j] = j;
    for (int a = 1; a < d; ++a) {
        const int x = order[a];
        int b = a - 1;
        while (b >= 0 && (avg[order[b]] > avg[x] || (avg[order[b]] == avg[x] && order[b] > x))) {
            order[b + 1] = order[b];
            --b;
        }
        order[b + 1] = x;
    }
    for (int round = 0; round < dp; ++round) {
        for (int i = 0; i < L; ++i) served[i] = 0;
        for (int j = 0; j < L; ++j) {
            const int dim = order[round * L + j];
            int best = -1;
            for (int i = 0; i < L; ++i)
                if (!served[i] && (best < 0 || sum[i] > sum[best])) best = i;
            served[best] = 1;
            sum[best] += avg[dim];
            perm[(size_t)best * dp + fill[best]] = dim;
            fill[best]++;
        }
    }
    if (avg_out) memcpy(avg_out, avg, sizeof(double) * (size_t)d);
    free(avg);
    free(order);
    free(sum);
    free(served);
    free(fill);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Alg. 1 with the routing hook                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    double dist;
    int32_t id;
    int32_t expanded;
} rentry;

static int rcmp(const void* a, const void* b)
{
    const rentry* x = (const rentry*)a;
    const rentry* y = (const rentry*)b;
    if (x->dist < y->dist) return -1;
    if (x->dist > y->dist) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

static double dot64(const float* a, const float* b, int d)
{
    double s = 0.0;
    for (int k = 0; k < d; ++k) s += (double)a[k] * (double)b[k];
    return s;
}

static double dist64(const float* x, const float* q, double qnorm, int d, int metric)
{
    if (metric == OR_L2) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
            double t = (double)x[k] - (double)q[k];
            s += t * t;
        }
        return s;
    }
    if (metric == OR_IP) return -dot64(x, q, d);
    return 1.0 - dot64(x, q, d) / qnorm;
}

/*
 * Distances in single precision, in one fixed summation order (used for the
 * search's ordering and comparison decisions when the oracle runs in the
 * precision of the GPU kernel).  The d coordinates are read in chunks of four
 * (chunk c = coordinates 4c..4c+3); chunk c belongs to segment c mod 16; each
 * segment is an fmaf chain over its chunks in increasing c (coordinates in
 * order), for l2 of t*t with t = x - q, for angular of x*q; the 16 segment
 * sums are added as a fixed binary tree: (0+1), (2+3), ... then pairs of
 * those, and so on.  Angular distance = fmaf(-s, 1/|q|, 1), with |q| =
 * sqrtf((p0 + p1) + (p2 + p3)), p_j the fmaf chain of q_k^2 over k = j mod 4.
 * With bf16 set, every coordinate of x is first rounded to bfloat16 (the
 * traversal copy of the precision form).
 */
static float qnorm32(const float* q, int d)
{
    float p[4];
    for (int j = 0; j < 4; ++j) {
        float acc = 0.0f;
        for (int k = j; k < d; k += 4) acc = fmaf(q[k], q[k], acc);
        p[j] = acc;
    }
    return sqrtf((p[0] + p[1]) + (p[2] + p[3]));
}

static float dist32(const float* x, const float* q, int d, int metric, float inv_qn, int bf16)
{
    float seg[16];
    const int nch = d / 4;
    for (int s = 0; s < 16; ++s) {
        float acc = 0.0f;
        for (int c = s; c < nch; c += 16) {
            for (int t = 0; t < 4; ++t) {
                const float xv = bf16 ? oracle_round_bf16(x[4 * c + t]) : x[4 * c + t];
                const float qv = q[4 * c + t];
                if (metric == OR_L2) {
                    const float df = xv - qv;
                    acc = fmaf(df, df, acc);
                } else {
                    acc = fmaf(xv, qv, acc);
                }
            }
        }
        seg[s] = acc;
    }
    for (int w = 16; w > 1; w /= 2)
        for (int i = 0; i < w / 2; ++i) seg[i] = seg[2 * i] + seg[2 * i + 1];
    if (metric == OR_IP) return -seg[0];
    return metric == OR_L2 ? seg[0] : fmaf(-seg[0], inv_qn, 1.0f);
}

typedef struct {
    const float *base, *A, *B, *queries;
    const int32_t *graph, *k, *ef;
    int64_t n, q0, q1;
    int d, R, L, m, metric, mode, entry, kstride, pool, fp32, lowp;
    const int32_t* perm; /* dimension permutation of the test, or NULL */
    const float* simhash; /* nb x d sign-projection vectors (SimHash mode) */
    int nb;
    const int32_t* entries; /* per-query entry node (upper-layer descent), or NULL */
    double eps, tau;
    int64_t* out_ids;
    double* out_dist;
    double* out_dist64;
    int64_t* counters;
    int32_t* fragile;
    int32_t* status;
} search_job;

/*
 * One query of Alg. 1.  Readings (where the paper leaves a choice):
 *  - the entry node is distance-computed, put in R and marked visited first;
 *  - R (results, at most ef) and the priority queue P are kept as ONE list
 *    sorted by (distance, id) whose entries carry an "expanded" flag.  Its
 *    first ef entries are R.  An entry beyond position ef stays only while
 *    unexpanded (it is in P but was pushed out of R).  Popping P = taking the
 *    first unexpanded entry of the list; the loop ends when there is none
 *    ("until P is empty").  The list holds at most `pool` entries (the worst
 *    unexpanded ones beyond that are dropped from P); pool = ef is the HNSW
 *    stopping rule, an unbounded pool is Alg. 1 as printed;
 *  - delta (and p, the entry at position ef) are read once per expansion,
 *    before v's neighbours are tested, and the survivors are merged after all
 *    of them (the paper tests 16 edges at once with SIMD);
 *  - a neighbour is visited (never distance-computed again) only once its
 *    exact distance has been computed, so one that fails the test from v can
 *    pass from a later node (the residual-edge remedy);
 *  - a survivor enters the list when R was not full or its distance is
 *    < delta.
 */
/*
 * When is the sign of the test's numerator the same in single precision as in
 * double?  The numerator of A_r (step (6)) is, for l2, g_e + (dist_v -
 * delta)/2 with g_e = (|u|^2 - |v|^2)/2, and for the inner product dist_v -
 * delta.  If every coordinate of x_u, x_v, x_p and q is an integer and the
 * squared norms and distances involved stay below 2^22, each of these terms
 * is a sum of integer products whose every partial sum is an integer below
 * 2^24 -- exact in single precision in any summation order -- and the
 * numerator itself is a multiple of 1/2 below 2^23, also exact.  Its sign
 * (the A_r <= 0 decision) then cannot depend on the precision, so a small
 * |A_r| is not a fragile decision.  The same holds for angular and inner
 * product when v = p (the numerator is then exactly 0 on both sides).
 */
static int integer_valued(const float* x, int d)
{
    for (int k = 0; k < d; ++k)
        if (!(fabsf(x[k]) < 16777216.0f) || x[k] != floorf(x[k])) return 0;
    return 1;
}

/* The same argument for a comparison of two search distances (list order,
   d_u against delta): with q and both vectors integer-valued and squared l2
   distances (or |inner products|) below 2^24, single precision computes both
   exactly, so their order cannot depend on the precision. */
static int distances_are_exact(const search_job* j, int q_int, int32_t a, int32_t b, double da,
                               double db)
{
    const double lim = 16777216.0; /* 2^24 */
    if (!q_int || (j->metric != OR_L2 && j->metric != OR_IP)) return 0;
    if (!(fabs(da) < lim) || !(fabs(db) < lim)) return 0;
    return integer_valued(j->base + (size_t)a * j->d, j->d) &&
           integer_valued(j->base + (size_t)b * j->d, j->d);
}

static int numerator_is_exact(int metric, int v_is_p, int ints, double nu2, double nv2, double dv,
                              double delta)
{
    const double lim = 4194304.0; /* 2^22 */
    if (metric != OR_L2 && v_is_p) return 1;
    if (!ints) return 0;
    if (metric == OR_L2) return nu2 < lim && nv2 < lim && dv < lim && delta < lim;
    if (metric == OR_IP) return fabs(dv) < lim && fabs(delta) < lim;
    return 0;
}

/* work space of the compact form: the node header and edge codes of the
   node being expanded, and the quantile table */
typedef struct {
    compact_hdr h;
    uint8_t *cg, *ci;
    float *wv, *wu, *gpw, *iew;
    int* kw;
    float lut[COMPACT_LUT_BINS];
} compact_ws;

static void search_one(const search_job* j, int64_t qi, const test_params* tp, uint8_t* visited,
                       rentry* R, rentry* S, double* table, float* fw1, float* fw2, double* dw,
                       compact_ws* cw)
{
    const int d = j->d;
    const float* q = j->queries + (size_t)qi * d;
    const int kq = j->k ? j->k[qi] : 1;
    int efq = j->ef ? j->ef[qi] : kq;
    if (efq < kq) efq = kq;
    /* list capacity: pool > 0 fixed (at least ef), pool < 0 |pool| x ef,
       pool = 0 unbounded */
    const int cap = j->pool > efq ? j->pool
                  : (j->pool > 0 ? efq
                  : (j->pool < 0 ? -j->pool * efq : (int)(j->n < INT32_MAX ? j->n : INT32_MAX)));
    int64_t* cnt = j->counters + (size_t)qi * C_NCOUNT;
    int flags = 0;
    memset(cnt, 0, sizeof(int64_t) * C_NCOUNT);
    double qnorm = sqrt(dot64(q, q, d));
    const float qn32 = qnorm32(q, d);
    const float inv_qn32 = 1.0f / qn32;
#define DIST(xp) (j->fp32 ? (double)dist32((xp), q, d, j->metric, inv_qn32, j->lowp & LP_BF16_BASE) \
                          : dist64((xp), q, qnorm, d, j->metric))
    if (!(qnorm > 0.0) || !isfinite(qnorm) || (j->fp32 && !(qn32 > 0.0f && isfinite(qn32)))) {
        j->status[qi] = -1;
        for (int t = 0; t < j->kstride; ++t) {
            j->out_ids[(size_t)qi * j->kstride + t] = -1;
            j->out_dist[(size_t)qi * j->kstride + t] = INFINITY;
            if (j->out_dist64) j->out_dist64[(size_t)qi * j->kstride + t] = INFINITY;
        }
        return;
    }
    /* the test works on permuted coordinates (codes, scalars, table); the
       distances on the original ones */
    float* qperm = NULL;
    if (j->perm) {
        qperm = (float*)malloc(sizeof(float) * (size_t)d);
        for (int k = 0; k < d; ++k) qperm[k] = q[j->perm[k]];
    }
    uint64_t qsig[4] = {0, 0, 0, 0};
    if (j->mode == OR_MODE_SIMHASH) simhash_bits_fp32(q, d, j->simhash, j->nb, qsig);
    const int q_int = !j->lowp && integer_valued(q, d);
    if (j->mode == OR_MODE_PEOS) {
        oracle_query_table(qperm ? qperm : q, d, j->L, j->m, j->A, j->B, table);
        if (j->lowp & LP_FP16)
            for (int t = 0; t < (j->L + 1) * j->m; ++t) table[t] = oracle_round_half(table[t]);
    }

    memset(visited, 0, (size_t)j->n);
    int size = 0;
    const int32_t v0 = j->entries ? j->entries[qi] : j->entry;
    const float* x0 = j->base + (size_t)v0 * d;
    R[0].dist = DIST(x0);
    R[0].id = v0;
    R[0].expanded = 0;
    size = 1;
    visited[v0] = 1;
    cnt[C_NDIST]++;

    edge_rec er;
    for (;;) {
        int pos = -1;
        for (int i = 0; i < size; ++i)
            if (!R[i].expanded) { pos = i; break; }
        if (pos < 0) break;
        R[pos].expanded = 1;
        cnt[C_EXPANSIONS]++;
        const int32_t v = R[pos].id;
        const float* xv = j->base + (size_t)v * d;
        const int full = (size >= efq);
        const double dv = R[pos].dist;
        const double delta = full ? R[efq - 1].dist : INFINITY;
        const int32_t p = full ? R[efq - 1].id : -1;
        if (full && j->mode != OR_MODE_EXHAUSTIVE) cnt[C_TEST_EXPANSIONS]++;
        double vq = 0.0, r = 0.0;
        int vp_int = 0; /* x_v, x_p and q integer-valued (see numerator_is_exact) */
        if (full && j->mode != OR_MODE_EXHAUSTIVE) {
            const float* xp = j->base + (size_t)p * d;
            vq = dot64(xv, q, d);
            if (j->metric == OR_L2) r = 0.5 * dot64(xp, xp, d) - dot64(xp, q, d);
            else r = -dot64(xp, q, d);
            vp_int = q_int && integer_valued(xv, d) && integer_valued(xp, d);
        }
        int ns = 0;
        int have_hdr = 0;
        for (int e = 0; e < j->R; ++e) {
            int32_t u = j->graph[(size_t)v * j->R + e];
            if (u < 0) continue;
            cnt[C_EDGES]++;
            if (visited[u]) { cnt[C_VISITED_SKIPS]++; continue; }
            const float* xu = j->base + (size_t)u * d;
            int pass = 1;
            if (full && j->mode == OR_MODE_SIMHASH) {
                /* e = u - v, |e| and g_e in double; signature in single */
                double ne2 = 0.0, nu2 = 0.0, nv2 = 0.0;
                float* e = fw1 + d;
                for (int k = 0; k < d; ++k) {
                    e[k] = xu[k] - xv[k];
                    const double t = (double)xu[k] - (double)xv[k];
                    ne2 += t * t;
                    nu2 += (double)xu[k] * xu[k];
                    nv2 += (double)xv[k] * xv[k];
                }
                uint64_t es[4];
                simhash_bits_fp32(e, d, j->simhash, j->nb, es);
                int diff = 0;
                for (int w = 0; w < (j->nb + 63) / 64; ++w) diff += __builtin_popcountll(es[w] ^ qsig[w]);
                double num;
                if (j->metric == OR_L2) num = 0.5 * nu2 - r - vq;
                else num = -r - vq;
                (void)nv2;
                int kind;
                const int ex = numerator_is_exact(j->metric, v == p,
                                                  vp_int && integer_valued(xu, d), nu2, nv2, dv,
                                                  delta);
                pass = routing_test_simhash(tp, sqrt(ne2), j->nb - diff, j->nb, num, qnorm, j->eps,
                                            &kind, &flags, ex);
                cnt[C_TESTS]++;
                cnt[kind == 0 ? C_TEST_ZERO : kind == 1 ? C_TEST_GE1 : kind == 2 ? C_TEST_LE0 : C_TEST_H]++;
                if (pass) cnt[C_PASSES]++;
            } else if (full && j->mode == OR_MODE_PEOS && (j->lowp & LP_COMPACT)) {
                /* compact form: the node's header and scalar codes (a build
                   product, taken over all of v's edges), the sub-vector
                   codes of this edge */
                if (!have_hdr) {
                    compact_node(j->base, d, j->graph + (size_t)v * j->R, j->R, j->L, j->metric,
                                 j->perm, v, cw->wv, cw->wu, cw->gpw, cw->iew, cw->kw, &cw->h,
                                 cw->cg, cw->ci);
                    have_hdr = 1;
                }
                uint8_t codes[257];
                if (j->perm) {
                    float* xvp = fw1 + d;
                    float* xup = fw2 + d;
                    for (int k = 0; k < d; ++k) {
                        xvp[k] = xv[j->perm[k]];
                        xup[k] = xu[j->perm[k]];
                    }
                    edge_codes_fp32(xvp, xup, d, j->L, j->m, j->A, j->B, fw1, fw2, codes, NULL);
                } else {
                    edge_codes_fp32(xv, xu, d, j->L, j->m, j->A, j->B, fw1, fw2, codes, NULL);
                }
                double A, H, T;
                int kind;
                pass = routing_test_compact(tp, &cw->h, cw->cg[e], cw->ci[e], codes, table,
                                            cw->lut, dv, delta, qnorm, &A, &H, &T, &kind, &flags,
                                            v == p);
                cnt[C_TESTS]++;
                cnt[kind == 0 ? C_TEST_ZERO : kind == 1 ? C_TEST_GE1 : kind == 2 ? C_TEST_LE0 : C_TEST_H]++;
                if (pass) cnt[C_PASSES]++;
            } else if (full && j->mode == OR_MODE_PEOS) {
                if (j->perm) {
                    float* xvp = fw1 + d;
                    float* xup = fw2 + d;
                    for (int k = 0; k < d; ++k) {
                        xvp[k] = xv[j->perm[k]];
                        xup[k] = xu[j->perm[k]];
                    }
                    edge_record(xvp, xup, d, j->L, j->m, j->A, j->B, fw1, fw2, dw, &er);
                } else {
                    edge_record(xv, xu, d, j->L, j->m, j->A, j->B, fw1, fw2, dw, &er);
                }
                double num;
                if (j->lowp & LP_BF16_BASE) {
                    /* the numerator from the search's own (bfloat16 traversal)
                       distances: g_e + (dist_v - delta)/2 for l2, and
                       (dist_v - delta) |q| for angular -- equal to the
                       expression below on exact distances */
                    if (j->metric == OR_L2) num = 0.5 * (er.nu2 - er.nv2) + 0.5 * (dv - delta);
                    else if (j->metric == OR_IP) num = dv - delta;
                    else num = (dv - delta) * qnorm;
                } else if (j->metric == OR_L2) {
                    num = 0.5 * er.nu2 - r - vq;
                } else {
                    num = -r - vq;
                }
                double A, H, T;
                int kind;
                if (j->lowp & LP_FP16)
                    pass = routing_test_lowp(tp, &er, table, dv, delta, qnorm, &A, &H, &T, &kind,
                                             &flags, v == p);
                else
                    pass = routing_test(tp, &er, table, num, qnorm, &A, &H, &T, &kind, &flags,
                                        numerator_is_exact(j->metric, v == p,
                                                           vp_int && integer_valued(xu, d),
                                                           er.nu2, er.nv2, dv, delta));
                cnt[C_TESTS]++;
                cnt[kind == 0 ? C_TEST_ZERO : kind == 1 ? C_TEST_GE1 : kind == 2 ? C_TEST_LE0 : C_TEST_H]++;
                if (pass) cnt[C_PASSES]++;
            }
            if (!pass) continue;
            visited[u] = 1;
            cnt[C_NDIST]++;
            double du = DIST(xu);
            if (!j->fp32 && full && fabs(du - delta) < j->tau * fabs(delta) &&
                !distances_are_exact(j, q_int, u, p, du, delta))
                flags |= F_DELTA;
            if (!full || du < delta) {
                S[ns].dist = du;
                S[ns].id = u;
                S[ns].expanded = 0;
                ++ns;
                cnt[C_INSERTED]++;
            }
        }
        /* list := sort(list u S) by (distance, id); keep the first ef, keep
           later entries only while unexpanded, at most `pool` in total */
        memcpy(R + size, S, sizeof(rentry) * (size_t)ns);
        int tot = size + ns;
        qsort(R, (size_t)tot, sizeof(rentry), rcmp);
        if (!j->fp32) {
            /* which entries stay, in which order, and which one is popped next
               all follow the order of the merged list up to the first entry
               the capacity drops: a query is fragile if two adjacent entries
               of that stretch have distances within tau */
            int kept = 0, last = tot - 1;
            for (int i = 0; i < tot; ++i) {
                if (i >= efq && R[i].expanded) continue;
                if (kept >= cap) {
                    last = i;
                    break;
                }
                ++kept;
            }
            for (int i = 1; i <= last; ++i) {
                double a = R[i - 1].dist, b = R[i].dist;
                double sc = fabs(a) > fabs(b) ? fabs(a) : fabs(b);
                if (a != b && fabs(a - b) < j->tau * sc &&
                    !distances_are_exact(j, q_int, R[i - 1].id, R[i].id, a, b))
                    flags |= F_ORDER;
            }
        }
        int w = 0;
        for (int i = 0; i < tot; ++i) {
            if (i >= efq && R[i].expanded) continue;
            if (w >= cap) break;
            R[w++] = R[i];
        }
        size = w;
    }
    if (j->lowp & LP_BF16_BASE) {
        /* precision form: the result list (first ef entries) re-ranked by
           single-precision distances on the full-precision base */
        const int nr = size < efq ? size : efq;
        for (int i = 0; i < nr; ++i)
            R[i].dist = (double)dist32(j->base + (size_t)R[i].id * d, q, d, j->metric, inv_qn32, 0);
        qsort(R, (size_t)nr, sizeof(rentry), rcmp);
    }
    for (int t = 0; t < j->kstride; ++t) {
        int64_t o = (size_t)qi * j->kstride + t;
        if (t < kq && t < size) {
            j->out_ids[o] = R[t].id;
            j->out_dist[o] = R[t].dist;
            if (j->out_dist64)
                j->out_dist64[o] = dist64(j->base + (size_t)R[t].id * d, q, qnorm, d, j->metric);
        } else {
            j->out_ids[o] = -1;
            j->out_dist[o] = INFINITY;
            if (j->out_dist64) j->out_dist64[o] = INFINITY;
        }
    }
    j->fragile[qi] = flags;
    j->status[qi] = 0;
    free(qperm);
#undef DIST
}

static void* search_worker(void* arg)
{
    search_job* j = (search_job*)arg;
    int efmax = 1;
    for (int64_t qi = j->q0; qi < j->q1; ++qi) {
        int kq = j->k ? j->k[qi] : 1;
        int e = j->ef ? j->ef[qi] : kq;
        if (e < kq) e = kq;
        if (e > efmax) efmax = e;
    }
    test_params tp;
    tp.L = j->L;
    tp.m = j->m;
    tp.metric = j->metric;
    tp.tau = j->tau;
    tp.eta = sqrt(2.0 * (double)j->L * log((double)j->m));
    tp.c_eps = oracle_norm_ppf(j->eps);
    uint8_t* visited = (uint8_t*)malloc((size_t)j->n);
    int64_t lcap = j->pool > 0 ? (j->pool > efmax ? j->pool : efmax)
                 : (j->pool < 0 ? (int64_t)-j->pool * efmax : j->n);
    rentry* R = (rentry*)malloc(sizeof(rentry) * (size_t)(lcap + j->R + 1));
    rentry* S = (rentry*)malloc(sizeof(rentry) * (size_t)(j->R + 1));
    double* table = (double*)malloc(sizeof(double) * (size_t)(j->L + 1) * j->m);
    float* fw1 = (float*)malloc(sizeof(float) * 2 * (size_t)j->d);
    float* fw2 = (float*)malloc(sizeof(float) * 2 * (size_t)j->d);
    double* dw = (double*)malloc(sizeof(double) * j->d);
    compact_ws cw;
    cw.cg = (uint8_t*)malloc((size_t)j->R);
    cw.ci = (uint8_t*)malloc((size_t)j->R);
    cw.wv = (float*)malloc(sizeof(float) * (size_t)j->d);
    cw.wu = (float*)malloc(sizeof(float) * (size_t)j->d);
    cw.gpw = (float*)malloc(sizeof(float) * (size_t)j->R);
    cw.iew = (float*)malloc(sizeof(float) * (size_t)j->R);
    cw.kw = (int*)malloc(sizeof(int) * (size_t)j->R);
    if (j->lowp & LP_COMPACT) oracle_compact_lut(j->L, j->m, j->eps, cw.lut);
    for (int64_t qi = j->q0; qi < j->q1; ++qi)
        search_one(j, qi, &tp, visited, R, S, table, fw1, fw2, dw, &cw);
    free(cw.cg);
    free(cw.ci);
    free(cw.wv);
    free(cw.wu);
    free(cw.gpw);
    free(cw.iew);
    free(cw.kw);
    free(visited);
    free(R);
    free(S);
    free(table);
    free(fw1);
    free(fw2);
    free(dw);
    return NULL;
}

/* ------------------------------------------------------------------ */
/* Entry descent through upper layers (the HNSW graphs of Sec. 6)      */
/* ------------------------------------------------------------------ */
/*
 * The paper runs PEOs on HNSW (and NSSG) graphs and searches the base layer
 * from an entry node (Alg. 1, v0).  In HNSW that entry comes from a greedy
 * walk down sparser upper layers: in each layer, from the current node, look
 * at all its neighbours in that layer and move to the closest one (distance,
 * then id) while it is closer than the current node; then continue from the
 * same node one layer below.  The node reached in the lowest upper layer is
 * v0.
 * Layout: the rows of all upper layers together; node[r] = base id of row
 * r; adj[r * Ru + j] = rows of its neighbours in the same layer (-1 = none);
 * down[r] = row of the same node one layer below (-1 in the lowest upper
 * layer); top = starting row.  Distances are the search's (dist32 in the
 * GPU's precision, with the bfloat16 base under LP_BF16_BASE, else dist64).
 * out_entry[q] = v0; out_ndist[q] = distances computed (the start included);
 * fragile[q] |= F_ORDER when two compared distances are within tau.
 */
static double descend_dist(const float* x, const float* q, double qnorm, float inv_qn32, int d,
                           int metric, int fp32, int lowp)
{
    return fp32 ? (double)dist32(x, q, d, metric, inv_qn32, lowp & LP_BF16_BASE)
                : dist64(x, q, qnorm, d, metric);
}

int oracle_descend(const float* base, int64_t n, int d, int metric, const int32_t* node,
                   const int32_t* adj, const int32_t* down, int64_t rows, int Ru, int top,
                   const float* queries, int64_t nq, int fp32, int lowp, double tau,
                   int32_t* out_entry, int64_t* out_ndist, int32_t* fragile)
{
    if (n <= 0 || d <= 0 || rows <= 0 || Ru <= 0 || top < 0 || top >= rows) return -1;
    fp32 = fp32 || lowp;
    for (int64_t qi = 0; qi < nq; ++qi) {
        const float* q = queries + (size_t)qi * d;
        const double qnorm = sqrt(dot64(q, q, d));
        const float inv_qn32 = 1.0f / qnorm32(q, d);
        int flags = 0;
        int64_t nd = 1;
        int64_t cur = top;
        double dcur = descend_dist(base + (size_t)node[cur] * d, q, qnorm, inv_qn32, d, metric,
                                   fp32, lowp);
        for (;;) {
            for (;;) {
                int64_t best = cur;
                double bd = dcur;
                for (int j = 0; j < Ru; ++j) {
                    const int32_t nb = adj[(size_t)cur * Ru + j];
                    if (nb < 0) continue;
                    const double dd = descend_dist(base + (size_t)node[nb] * d, q, qnorm,
                                                   inv_qn32, d, metric, fp32, lowp);
                    ++nd;
                    const double sc = fabs(dd) > fabs(bd) ? fabs(dd) : fabs(bd);
                    if (dd != bd && fabs(dd - bd) < tau * sc) flags |= F_ORDER;
                    if (dd < bd || (dd == bd && node[nb] < node[best])) {
                        best = nb;
                        bd = dd;
                    }
                }
                if (best == cur) break;
                cur = best;
                dcur = bd;
            }
            if (down[cur] < 0) break;
            cur = down[cur];
        }
        out_entry[qi] = node[cur];
        if (out_ndist) out_ndist[qi] = nd;
        if (fragile) fragile[qi] = flags;
    }
    return 0;
}

/*
 * Public: batched search.  k and ef are per-query arrays (ef := max(ef, k)).
 * pool: capacity of the candidate list (0: unbounded, Alg. 1 as printed;
 * positive values below ef act as ef, the HNSW stopping rule; negative:
 * |pool| times each query's ef).
 * fp32: 0 = distances in double precision; 1 = the search's distance
 * decisions (order, delta, insertion) taken on the single-precision
 * distances of dist32(), the precision of the GPU kernel.  out_dist then
 * holds those values and out_dist64 (optional) the double-precision ones.
 * out_ids / out_dist: nq x kstride, first k entries of R, padded (-1, +inf).
 * Distances: squared l2, 1 - x.q/|q| for the angular metric, or -x.q for
 * the inner product (the largest inner products first).
 * counters: nq x C_NCOUNT int64; fragile: nq flag words; status: 0 ok, -1
 * zero/non-finite query.  lowp: precision-form flags (LP_*, implies fp32):
 * LP_FP16 takes the routing test on half-rounded scalars and tables
 * (routing_test_lowp); LP_BF16_BASE takes the traversal distances on the
 * bfloat16-rounded base (and the numerator of A_r from them) and re-ranks the
 * final result list with full-precision single-precision distances before
 * the first k are taken.  perm (optional, d entries): the dimension
 * permutation of the test -- edge records and the table are taken on the
 * permuted coordinates, distances on the original ones.  mode
 * OR_MODE_SIMHASH takes the SimHash test (routing_test_simhash) with the nb
 * sign-projection vectors simhash (nb x d) instead of the PEOs test.
 * entries (optional, nq ids): each query's entry node v0 (from
 * oracle_descend) instead of the common entry.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_search(const float* base, int64_t n, int d, const int32_t* graph, int R, int entry,
                  int L, int m, const float* A, const float* B, int metric, const float* queries,
                  int64_t nq, const int32_t* k, const int32_t* ef, int kstride, int pool,
                  double eps, int mode, double tau, int fp32, int lowp, const int32_t* perm,
                  const float* simhash, int nb, const int32_t* entries, int nthreads,
                  int64_t* out_ids,
                  double* out_dist, double* out_dist64, int64_t* counters, int32_t* fragile,
                  int32_t* status)
{
    if (n <= 0 || d <= 0 || R <= 0 || entry < 0 || entry >= n) return -1;
    if (mode == OR_MODE_PEOS && (L <= 0 || d % L || L > 255 || m < 2 || 2 * m > 256)) return -1;
    if (mode != OR_MODE_EXHAUSTIVE && !(eps > 0.0 && eps <= 0.5)) return -1;
    if (mode == OR_MODE_SIMHASH && (!simhash || nb < 1 || nb > 256)) return -1;
    if ((lowp & LP_COMPACT) && (L > 4 || (lowp & LP_FP16) || mode == OR_MODE_SIMHASH)) return -1;
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    if (nthreads > nq) nthreads = (int)(nq > 0 ? nq : 1);
    pthread_t th[256];
    search_job jobs[256];
    for (int t = 0; t < nthreads; ++t) {
        jobs[t] = (search_job){base, A, B, queries, graph, k, ef, n, nq * t / nthreads,
                               nq * (t + 1) / nthreads, d, R, L, m, metric, mode, entry, kstride,
                               pool, fp32 || (lowp & (LP_BF16_BASE | LP_FP16)), lowp, perm,
                               simhash, nb, entries, eps, tau,
                               out_ids,
                               out_dist, out_dist64, counters, fragile, status};
        pthread_create(&th[t], NULL, search_worker, &jobs[t]);
    }
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* Public: one routing test, for the pins.  Returns pass (1/0); out = {A, H, T, kind}.
 * lowp & LP_FP16: the precision-form test (routing_test_lowp) with dist_v and
 * delta the single-precision distances of v and p.  simhash (nb x d): the
 * SimHash test instead; H is then the collision count. */
int oracle_test_edge(const float* xv, const float* xu, const float* xp, const float* q, int d,
                     int L, int m, const float* A, const float* B, int metric, double eps,
                     int lowp, const float* simhash, int nb, double* out)
{
    float* fw1 = (float*)malloc(sizeof(float) * d);
    float* fw2 = (float*)malloc(sizeof(float) * d);
    double* dw = (double*)malloc(sizeof(double) * d);
    double* table = (double*)malloc(sizeof(double) * (size_t)(L + 1) * m);
    edge_rec er;
    edge_record(xv, xu, d, L, m, A, B, fw1, fw2, dw, &er);
    oracle_query_table(q, d, L, m, A, B, table);
    test_params tp = {sqrt(2.0 * L * log((double)m)), oracle_norm_ppf(eps), 1e-5, L, m, metric};
    double qnorm = sqrt(dot64(q, q, d));
    double vq = dot64(xv, q, d);
    double r = metric == OR_L2 ? 0.5 * dot64(xp, xp, d) - dot64(xp, q, d) : -dot64(xp, q, d);
    double num = metric == OR_L2 ? 0.5 * er.nu2 - r - vq : -r - vq;
    double a, h, t;
    int kind, flags = 0;
    int pass;
    if (simhash) {
        float* e = (float*)malloc(sizeof(float) * d);
        for (int k = 0; k < d; ++k) e[k] = xu[k] - xv[k];
        uint64_t es[4], qs[4];
        simhash_bits_fp32(e, d, simhash, nb, es);
        simhash_bits_fp32(q, d, simhash, nb, qs);
        int diff = 0;
        for (int w = 0; w < (nb + 63) / 64; ++w) diff += __builtin_popcountll(es[w] ^ qs[w]);
        free(e);
        a = er.norm_e > 0.0 ? num / (qnorm * er.norm_e) : NAN;
        h = nb - diff;
        t = NAN;
        pass = routing_test_simhash(&tp, er.norm_e, nb - diff, nb, num, qnorm, eps, &kind, &flags, 0);
    } else if (lowp & LP_FP16) {
        for (int i = 0; i < (L + 1) * m; ++i) table[i] = oracle_round_half(table[i]);
        const float iq = 1.0f / qnorm32(q, d);
        const double dv = dist32(xv, q, d, metric, iq, 0), dp = dist32(xp, q, d, metric, iq, 0);
        pass = routing_test_lowp(&tp, &er, table, dv, dp, qnorm, &a, &h, &t, &kind, &flags, 0);
    } else {
        pass = routing_test(&tp, &er, table, num, qnorm, &a, &h, &t, &kind, &flags, 0);
    }
    out[0] = a;
    out[1] = h;
    out[2] = t;
    out[3] = kind;
    free(fw1);
    free(fw2);
    free(dw);
    free(table);
    return pass;
}
