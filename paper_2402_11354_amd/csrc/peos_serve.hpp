// Serving form of the search: a request loop over one index with continuous
// batching (declarations and contracts: include/peos.h, peos_serve_*).
//
// Requests (1..max_batch queries sharing k and ef) wait in a FIFO.  Each of
// up to max_inflight launch slots owns a stream, device buffers and pinned
// staging.  Whenever a slot is free, the requests at the head of the FIFO
// are packed into one batch (per-query k and ef, so one launch serves
// requests of different sizes) and issued: copy in, projection tables, ef
// class split, search launches, copy out, all asynchronous on the slot's
// stream.  Batches on different slots run on the device at the same time.
// Admission: a batch is issued only while the LDS its resident waves hold,
// added to that of the batches in flight, stays within the LDS budget (a
// batch that would oversubscribe the CUs waits for one to finish instead of
// queueing behind it in the hardware); device memory is bounded at open
// time by the HBM budget, which caps the number of slots.  Results do not
// depend on how requests are batched.
#pragma once

#include <deque>
#include <vector>

namespace {

struct ServeRequest {
    uint64_t ticket;
    const float* q;
    int32_t nq, k, ef;
    int64_t* ids;
    float* dists;
};

struct ServeSlot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* dmem = nullptr;
    void* hmem = nullptr;
    float* d_q = nullptr;
    int32_t* d_k = nullptr;
    int32_t* d_ef = nullptr;
    int64_t* d_ids = nullptr;
    float* d_dists = nullptr;
    void* d_ws = nullptr;
    size_t ws_bytes = 0;
    float* h_q = nullptr;
    int32_t* h_k = nullptr;
    int32_t* h_ef = nullptr;
    int64_t* h_ids = nullptr;
    float* h_dists = nullptr;
    std::vector<ServeRequest> reqs;
    int64_t lds = 0;
    bool busy = false;
};

}  // namespace

struct peos_server {
    const peos_index* ix;
    peos_serve_config cfg;
    int64_t lds_budget, lds_inflight;
    int launch_waves;
    std::vector<ServeSlot> slots;
    std::deque<ServeRequest> pending;
    int64_t pending_q;
    std::deque<uint64_t> finished;
    uint64_t next_ticket;
    int64_t n_launches, n_queries, n_requests, max_batch_seen;
};

namespace {

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

void release_slot(ServeSlot& s)
{
    if (s.stream) (void)hipStreamSynchronize(s.stream);
    if (s.done) (void)hipEventDestroy(s.done);
    if (s.stream) (void)hipStreamDestroy(s.stream);
    if (s.dmem) (void)hipFree(s.dmem);
    if (s.hmem) (void)hipHostFree(s.hmem);
    s = ServeSlot();
}

int serve_dispatch(peos_server* sv);

// copy the results of a finished batch out to its requests
void serve_complete(peos_server* sv, ServeSlot& s)
{
    const int ks = sv->cfg.max_k;
    int64_t off = 0;
    for (const ServeRequest& r : s.reqs) {
        for (int32_t i = 0; i < r.nq; ++i) {
            std::memcpy(r.ids + (int64_t)i * r.k, s.h_ids + (off + i) * ks, sizeof(int64_t) * r.k);
            std::memcpy(r.dists + (int64_t)i * r.k, s.h_dists + (off + i) * ks, sizeof(float) * r.k);
        }
        off += r.nq;
        sv->finished.push_back(r.ticket);
        ++sv->n_requests;
    }
    sv->n_queries += off;
    sv->lds_inflight -= s.lds;
    s.reqs.clear();
    s.lds = 0;
    s.busy = false;
}

int serve_reap(peos_server* sv, bool* any)
{
    *any = false;
    for (ServeSlot& s : sv->slots) {
        if (!s.busy) continue;
        hipError_t e = hipEventQuery(s.done);
        if (e == hipErrorNotReady) continue;
        if (e != hipSuccess) return fail(PEOS_EHIP, "hipEventQuery: %s", hipGetErrorString(e));
        serve_complete(sv, s);
        *any = true;
    }
    return PEOS_OK;
}

// enqueue one packed batch on its slot's stream: copy in, tables, search,
// copy out, completion event
int serve_issue(peos_server* sv, ServeSlot& sl, int64_t nqb, int kmax, int efmax, int waves)
{
    const peos_index* ix = sv->ix;
    const peos_serve_config& c = sv->cfg;
    ServeSlot* s = &sl;
    const int d = ix->d;
    hipStream_t st = s->stream;
    HIP_TRY(hipMemcpyAsync(s->d_q, s->h_q, sizeof(float) * nqb * d, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->d_k, s->h_k, sizeof(int32_t) * nqb, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(s->d_ef, s->h_ef, sizeof(int32_t) * nqb, hipMemcpyHostToDevice, st));
    WsLayout w = ws_layout(ix, nqb, spill_words_of(ix));
    float* tables = (float*)((char*)s->d_ws + w.tables_off);
    float* qnorms = (float*)((char*)s->d_ws + w.qnorm_off);
    int rc = peos_query_tables(ix, s->d_q, nqb, tables, qnorms, st);
    if (rc) return rc;
    rc = search_impl(ix, s->d_q, tables, qnorms, nqb, s->d_k, s->d_ef, kmax, efmax, c.max_k,
                     c.pool, c.eps, c.mode, s->d_ids, s->d_dists, nullptr, s->d_ws, s->ws_bytes,
                     st, waves);
    if (rc) return rc;
    HIP_TRY(hipMemcpyAsync(s->h_ids, s->d_ids, sizeof(int64_t) * nqb * c.max_k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(s->h_dists, s->d_dists, sizeof(float) * nqb * c.max_k, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(s->done, st));
    return PEOS_OK;
}

int serve_dispatch(peos_server* sv)
{
    const peos_index* ix = sv->ix;
    const peos_serve_config& c = sv->cfg;
    while (!sv->pending.empty()) {
        ServeSlot* s = nullptr;
        for (ServeSlot& t : sv->slots)
            if (!t.busy) {
                s = &t;
                break;
            }
        if (!s) return PEOS_OK;
        // the longest FIFO prefix that fits one launch
        int64_t nqb = 0;
        int kmax = 1, efmax = 1;
        size_t take = 0;
        for (const ServeRequest& r : sv->pending) {
            if (nqb + r.nq > c.max_batch) break;
            nqb += r.nq;
            kmax = r.k > kmax ? r.k : kmax;
            efmax = r.ef > efmax ? r.ef : efmax;
            ++take;
        }
        const int listmax = efmax > kmax ? efmax : kmax;
        SearchPlan p = plan_search(ix, nqb, listmax, c.pool, true);
        int64_t waves = p.slots < sv->launch_waves ? p.slots : sv->launch_waves;
        const int64_t lds = p.lds * waves;
        if (sv->lds_inflight > 0 && sv->lds_inflight + lds > sv->lds_budget) return PEOS_OK;
        // pack the batch into the slot's pinned staging
        const int d = ix->d;
        int64_t off = 0;
        s->reqs.clear();
        for (size_t i = 0; i < take; ++i) {
            ServeRequest r = sv->pending.front();
            sv->pending.pop_front();
            std::memcpy(s->h_q + off * d, r.q, sizeof(float) * (size_t)r.nq * d);
            for (int32_t j = 0; j < r.nq; ++j) {
                s->h_k[off + j] = r.k;
                s->h_ef[off + j] = r.ef;
            }
            off += r.nq;
            s->reqs.push_back(r);
        }
        sv->pending_q -= nqb;
        int rc = serve_issue(sv, *s, nqb, kmax, efmax, (int)waves);
        if (rc) {
            // nothing of this batch will complete: its requests go back to
            // the head of the queue, in order, and the slot stays free once
            // what was already enqueued on its stream has drained
            (void)hipStreamSynchronize(s->stream);
            for (size_t i = s->reqs.size(); i-- > 0;) sv->pending.push_front(s->reqs[i]);
            sv->pending_q += nqb;
            s->reqs.clear();
            return rc;
        }
        s->busy = true;
        s->lds = lds;
        sv->lds_inflight += lds;
        ++sv->n_launches;
        sv->max_batch_seen = nqb > sv->max_batch_seen ? nqb : sv->max_batch_seen;
    }
    return PEOS_OK;
}

}  // namespace

extern "C" {

int peos_serve_open(const peos_index* ix, const peos_serve_config* cfg, peos_server** out)
{
    if (!out) return fail(PEOS_EINVAL, "null output handle");
    *out = nullptr;
    if (!ix || !cfg) return fail(PEOS_EINVAL, "null pointer");
    const peos_serve_config& c = *cfg;
    if (c.max_batch < 1 || c.max_batch > (1 << 20)) return fail(PEOS_EINVAL, "max_batch=%d", c.max_batch);
    if (c.max_k < 1 || c.max_k > kMaxEf) return fail(PEOS_EINVAL, "max_k=%d", c.max_k);
    if (c.max_ef < 1 || c.max_ef > kMaxEf) return fail(PEOS_EINVAL, "max_ef=%d", c.max_ef);
    if (c.max_inflight < 1 || c.max_inflight > 16) return fail(PEOS_EINVAL, "max_inflight=%d", c.max_inflight);
    if (c.max_pending < c.max_batch) return fail(PEOS_EINVAL, "max_pending=%d < max_batch", c.max_pending);
    if (c.pool < -16 || c.pool > 2 * kMaxEf || (c.pool < 0 && -c.pool * c.max_ef > 2 * kMaxEf))
        return fail(PEOS_EINVAL, "pool=%d", c.pool);
    if (c.mode != PEOS_MODE_PEOS && c.mode != PEOS_MODE_EXHAUSTIVE && c.mode != PEOS_MODE_SIMHASH) return fail(PEOS_EINVAL, "mode=%d", c.mode);
    if (c.mode != PEOS_MODE_EXHAUSTIVE && !(c.eps > 0.f && c.eps <= 0.5f)) return fail(PEOS_EINVAL, "eps=%g", (double)c.eps);
    if (c.mode == PEOS_MODE_SIMHASH && !(ix->flags & PEOS_FLAG_SIMHASH)) return fail(PEOS_EINVAL, "SimHash mode needs PEOS_FLAG_SIMHASH");
    if (c.launch_waves < 0 || c.launch_waves > kMaxSlots) return fail(PEOS_EINVAL, "launch_waves=%d", c.launch_waves);
    int dev;
    int rc = check_device(&dev);
    if (rc) return rc;
    if (dev != ix->device) return fail(PEOS_EINVAL, "current device %d is not the index's %d", dev, ix->device);
    // the largest request must have a launch plan that fits a workgroup's
    // LDS (every ef class of a batch plans within it), else every batch
    // holding one would fail at dispatch
    {
        const int listmax = c.max_ef > c.max_k ? c.max_ef : c.max_k;
        SearchPlan p = plan_search(ix, c.max_batch, listmax, c.pool, true, num_classes(listmax) - 1);
        if (p.lds + kStaticLds > 64 * 1024)
            return fail(PEOS_EINVAL, "max_ef=%d with pool=%d needs %lld bytes of LDS per wave (64 KB at most)",
                        c.max_ef, c.pool, (long long)p.lds);
    }
    // memory of one slot
    const int64_t B = c.max_batch, K = c.max_k, d = ix->d;
    WsLayout w = ws_layout(ix, B, spill_words_of(ix));
    const int64_t o_q = 0, o_k = align256(o_q + 4 * B * d), o_ef = align256(o_k + 4 * B),
                  o_ids = align256(o_ef + 4 * B), o_dist = align256(o_ids + 8 * B * K),
                  o_ws = align256(o_dist + 4 * B * K), dbytes = o_ws + w.total;
    const int64_t h_q = 0, h_k = align256(4 * B * d), h_ef = align256(h_k + 4 * B),
                  h_ids = align256(h_ef + 4 * B), h_dist = align256(h_ids + 8 * B * K),
                  hbytes = align256(h_dist + 4 * B * K);
    int nslots = c.max_inflight;
    if (c.hbm_budget > 0) {
        const int64_t fit = (int64_t)c.hbm_budget / dbytes;
        if (fit < 1) return fail(PEOS_ENOSPACE, "one launch slot needs %lld device bytes, budget %zu", (long long)dbytes, c.hbm_budget);
        if (fit < nslots) nslots = (int)fit;
    }
    peos_server* sv = new (std::nothrow) peos_server();
    if (!sv) return fail(PEOS_EINVAL, "out of host memory");
    sv->ix = ix;
    sv->cfg = c;
    sv->lds_budget = c.lds_budget > 0 ? (int64_t)c.lds_budget : ix->lds_per_cu * ix->num_cu;
    sv->lds_inflight = 0;
    sv->launch_waves = c.launch_waves > 0 ? c.launch_waves : kMaxSlots;
    sv->pending_q = 0;
    sv->next_ticket = 1;
    sv->n_launches = sv->n_queries = sv->n_requests = sv->max_batch_seen = 0;
    sv->slots.resize(nslots);
    hipError_t e = hipSuccess;
    for (ServeSlot& s : sv->slots) {
        if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipMalloc(&s.dmem, (size_t)dbytes)) != hipSuccess) break;
        if ((e = hipHostMalloc(&s.hmem, (size_t)hbytes, hipHostMallocDefault)) != hipSuccess) break;
        char* dm = (char*)s.dmem;
        char* hm = (char*)s.hmem;
        s.d_q = (float*)(dm + o_q);
        s.d_k = (int32_t*)(dm + o_k);
        s.d_ef = (int32_t*)(dm + o_ef);
        s.d_ids = (int64_t*)(dm + o_ids);
        s.d_dists = (float*)(dm + o_dist);
        s.d_ws = dm + o_ws;
        s.ws_bytes = (size_t)w.total;
        s.h_q = (float*)(hm + h_q);
        s.h_k = (int32_t*)(hm + h_k);
        s.h_ef = (int32_t*)(hm + h_ef);
        s.h_ids = (int64_t*)(hm + h_ids);
        s.h_dists = (float*)(hm + h_dist);
    }
    if (e != hipSuccess) {
        for (ServeSlot& s : sv->slots) release_slot(s);
        delete sv;
        return fail(PEOS_EHIP, "serve_open: %s", hipGetErrorString(e));
    }
    *out = sv;
    return PEOS_OK;
}

int peos_serve_submit(peos_server* sv, const float* queries, int32_t nq, int32_t k, int32_t ef,
                      int64_t* ids, float* dists, uint64_t* ticket)
{
    if (!sv || !queries || !ids || !dists || !ticket) return fail(PEOS_EINVAL, "null pointer");
    const peos_serve_config& c = sv->cfg;
    if (nq < 1 || nq > c.max_batch) return fail(PEOS_EINVAL, "nq=%d not in [1, max_batch=%d]", nq, c.max_batch);
    if (k < 1 || k > c.max_k) return fail(PEOS_EINVAL, "k=%d not in [1, max_k=%d]", k, c.max_k);
    if (ef < 1 || ef > c.max_ef) return fail(PEOS_EINVAL, "ef=%d not in [1, max_ef=%d]", ef, c.max_ef);
    if (sv->pending_q + nq > c.max_pending) return fail(PEOS_EBUSY, "%lld queries waiting", (long long)sv->pending_q);
    ServeRequest r;
    r.ticket = sv->next_ticket++;
    r.q = queries;
    r.nq = nq;
    r.k = k;
    r.ef = ef;
    r.ids = ids;
    r.dists = dists;
    sv->pending.push_back(r);
    sv->pending_q += nq;
    const int rc = serve_dispatch(sv);
    if (rc) {
        // a failed dispatch put its batch back at the head of the queue; this
        // request is then still the last one queued: take it out, so that an
        // error means nothing of this call was queued
        if (!sv->pending.empty() && sv->pending.back().ticket == r.ticket) {
            sv->pending.pop_back();
            sv->pending_q -= nq;
        }
        return rc;
    }
    *ticket = r.ticket;
    return PEOS_OK;
}

int peos_serve_poll(peos_server* sv, int32_t wait, uint64_t* done, int32_t max_done, int32_t* n_done)
{
    if (!sv || !n_done || (max_done > 0 && !done) || max_done < 0) return fail(PEOS_EINVAL, "bad poll arguments");
    *n_done = 0;
    bool any = false;
    int rc = serve_reap(sv, &any);
    if (rc) return rc;
    if (wait && !any && sv->finished.empty()) {
        // block on the batch issued first among those in flight
        ServeSlot* first = nullptr;
        for (ServeSlot& s : sv->slots)
            if (s.busy) {
                first = &s;
                break;
            }
        if (first) {
            HIP_TRY(hipEventSynchronize(first->done));
            rc = serve_reap(sv, &any);
            if (rc) return rc;
        }
    }
    rc = serve_dispatch(sv);
    if (rc) return rc;
    int32_t n = 0;
    while (n < max_done && !sv->finished.empty()) {
        done[n++] = sv->finished.front();
        sv->finished.pop_front();
    }
    *n_done = n;
    return PEOS_OK;
}

int peos_serve_counters(const peos_server* sv, int64_t* out)
{
    if (!sv || !out) return fail(PEOS_EINVAL, "null pointer");
    int64_t inflight = 0;
    for (const ServeSlot& s : sv->slots) inflight += s.busy ? 1 : 0;
    out[0] = sv->n_launches;
    out[1] = sv->n_requests;
    out[2] = sv->n_queries;
    out[3] = sv->max_batch_seen;
    out[4] = inflight;
    out[5] = sv->pending_q;
    out[6] = (int64_t)sv->slots.size();
    out[7] = sv->lds_inflight;
    return PEOS_OK;
}

void peos_serve_close(peos_server* sv)
{
    if (!sv) return;
    for (ServeSlot& s : sv->slots) release_slot(s);
    delete sv;
}

}  // extern "C"
