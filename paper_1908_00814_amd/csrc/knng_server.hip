// knng_server.hip -- J-Merge serving: a resident point set with its k-NN
// graph absorbs requests of raw rows (Section 3.2: a built graph takes in
// raw data without being rebuilt).
//
// Every request is one balanced-append J-Merge of the current base (rows and
// lists frozen until the next rebase) with the request's rows, seeded from
// the request's own id, so its result does not depend on which requests run
// beside it.  Requests run in slots -- a stream, a host thread and a merge
// workspace each -- so several are on the device at once and a waiting
// request starts as soon as a slot frees up.  When a request finishes, its
// new entries are folded into the resident graph with the lock-free set-form
// insert; the commits of different requests commute.  With batching on, a
// slot that frees up merges all queued requests (up to max_request rows) as
// one raw set instead: better bridges into the base for small requests, at
// the price of results that depend on the batch.
//
// Device memory is allocated once at creation: the row store for the full
// capacity (request rows are packed at submission into their final place and
// never move), the base lists, the resident lists, and one workspace per
// slot.  A request's merge sees base rows [0, m) and its own rows, which the
// row view maps onto their place in the store.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <set>
#include <mutex>
#include <shared_mutex>
#include <thread>

#include "knng_host.h"

#include <new>

using namespace knng;
using namespace knng::host;

namespace {

enum ReqState { Q_PENDING = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    int64_t first = 0, n = 0;
    uint64_t seed = 0, req_id = 0;
    int state = Q_PENDING;
    knng_status rc = KNNG_OK;
    std::string err;
    std::vector<uint64_t> keys;  // n x k result keys (global ids), filled at the end
    knng_request_info info{};
};

double now_us(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
        .count();
}


struct Slot {
    int idx = 0;
    hipStream_t st = nullptr;
    Layout w{};               // per-request merge state; row arrays point at the store
    uint64_t *out = nullptr;  // capacity x gstride final keys of the request
    std::thread th;
    // Merge state kept between requests: after a merge, only rows it changed
    // (dtag >= prev_tag0) differ from the initial state of an unselected base
    // row, and every tag it wrote is below tag0.  fresh: the state must be
    // initialised in full (first merge, after a rebase or a failed merge).
    int32_t tag0 = 0, prev_tag0 = 0;
    bool fresh = true;
    // the repeat loop as a launch graph of one round, captured on the first
    // request, and its device round state
    RoundGraph graph{};
    DevRound *dev = nullptr;
};

} // namespace

struct knng_server {
    int device = 0;
    int d = 0, k = 0, gstride = 0;
    knng_metric metric = KNNG_L2;
    knng_opts opts{};
    bool bf16 = false, manual = false, batching = false;
    bool host_rounds = false;  // rounds driven by the host instead of the slot graphs
    int64_t capacity = 0, max_request = 0;
    void *mem = nullptr;
    Layout store{};           // x, norm, xb, se for all rows; gin = base lists
    uint64_t *res = nullptr;  // capacity x k resident lists
    float *stage = nullptr;   // max_request x d: host rows on their way in
    uint64_t *sub_ctr = nullptr;
    // reverse index of the base lists (rebuilt by a rebase)
    int64_t *ri_off = nullptr, *ri_part = nullptr;
    int32_t *ri_src = nullptr, *ri_deg = nullptr;
    hipStream_t sub_st = nullptr;
    std::vector<Slot> slots;
    std::chrono::steady_clock::time_point t0;

    std::shared_mutex state_mu;  // shared: a request in a slot; exclusive: snapshot, rebase
    std::mutex mu;               // queue, counters and records below
    std::mutex sub_mu;           // one submission at a time
    std::condition_variable cv_work, cv_done;
    int64_t m_base = 0;     // rows of the base the requests merge with
    int64_t reserved = 0;   // rows taken by accepted submissions
    int64_t committed = 0;  // request rows folded into the resident graph since the rebase
    int64_t dropped = 0;    // rows of failed requests since the rebase (empty lists)
    std::set<uint64_t> fail_ids;  // test hook: request ids made to fail before their commit
    int64_t running = 0;
    uint64_t next_ticket = 1;
    std::deque<uint64_t> pending;
    std::map<uint64_t, Request> reqs;
    bool stop = false, failed = false;
    std::string fail_text;
};

namespace {

// device layout shared by the requests; with base == nullptr it only measures
void carve_store(Carve &c, knng_server &s)
{
    Layout &w = s.store;
    w.dp = pad4(s.d);
    w.db = (s.d + 31) / 32 * 32;
    w.gstride = s.gstride;
    w.x = c.take<float>((size_t)s.capacity * w.dp);
    w.norm = s.metric == KNNG_COSINE ? c.take<float>(s.capacity) : nullptr;
    w.xb = s.bf16 ? c.take<uint16_t>((size_t)s.capacity * w.db) : nullptr;
    w.se = s.bf16 ? c.take<float2>(s.capacity) : nullptr;
    w.gin = c.take<uint64_t>((size_t)s.capacity * s.gstride);
    w.ctr = c.take<uint64_t>(C_WORDS);
    s.res = c.take<uint64_t>((size_t)s.capacity * s.k);
    s.stage = c.take<float>((size_t)s.max_request * s.d);
    s.sub_ctr = c.take<uint64_t>(C_WORDS);
    s.ri_off = c.take<int64_t>((size_t)s.capacity + 1);
    s.ri_src = c.take<int32_t>((size_t)s.capacity * s.k);
    s.ri_deg = c.take<int32_t>(s.capacity);
    s.ri_part = c.take<int64_t>(rindex_parts(s.capacity));
    w.rev_off = s.ri_off;
    w.rev_src = s.ri_src;
}

// the reverse index of the first k entries of the m base lists (those an
// unselected base row starts a request with)
knng_status build_rindex(knng_server *s, int64_t m)
{
    HIP_TRY(launch_zero_counters(s->sub_ctr, C_WORDS, s->sub_st));
    HIP_TRY(launch_build_rindex(s->store.gin, s->gstride, s->k, m, s->ri_off, s->ri_src,
                                s->ri_deg, s->ri_part, s->sub_ctr, s->sub_st));
    uint64_t h[C_WORDS];
    knng_status r = read_ctr(s->sub_ctr, h, s->sub_st);
    if (r != KNNG_OK)
        return r;
    if (h[C_ERR])
        return fail(KNNG_EDEVICE, "reverse index of the base lists: %s", err_text(h[C_ERR]));
    return KNNG_OK;
}

// one slot's merge state for a problem of up to `capacity` rows
void carve_slot(Carve &c, const knng_server &s, Slot &sl)
{
    const int64_t n = s.capacity;
    const int k = s.k, sm = s.opts.sample;
    Layout &w = sl.w;
    w = s.store;  // row arrays and base lists are shared
    w.ctr = c.take<uint64_t>(C_WORDS);
    w.L = c.take<uint64_t>((size_t)n * k);
    w.worst = c.take<uint64_t>(n);
    w.new_f = c.take<int32_t>((size_t)n * sm);
    w.old_f = c.take<int32_t>((size_t)n * k);
    w.cnt_f = c.take<int32_t>((size_t)n * 2);
    w.rnew = c.take<uint64_t>((size_t)n * sm);
    w.rold = c.take<uint64_t>((size_t)n * sm);
    w.dtag = c.take<int32_t>(n);
    w.atag = c.take<int32_t>(n);
    w.rfill = c.take<int32_t>((size_t)n * 2);
    w.alist = c.take<int32_t>(n);  // active rows of a round: a request touches few rows
    sl.out = c.take<uint64_t>((size_t)n * s.gstride);
    sl.dev = c.take<DevRound>(1);
}

size_t store_bytes(knng_server &s)
{
    Carve c(nullptr);
    carve_store(c, s);
    return c.off + 256;
}

size_t slot_bytes(const knng_server &s)
{
    Carve c(nullptr);
    Slot sl;
    carve_slot(c, s, sl);
    return c.off + 256;
}

// One merge in one slot: a single request, or (batching) several queued
// requests whose rows are consecutive (the caller holds the state lock shared).
knng_status run_request(knng_server *s, Slot &sl, const std::vector<uint64_t> &tickets)
{
    int64_t m, first = 0, nr = 0;
    uint64_t seed = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        m = s->m_base;
        for (size_t i = 0; i < tickets.size(); i++) {
            Request &r = s->reqs[tickets[i]];
            if (i == 0) {
                first = r.first;
                seed = r.seed;
            }
            nr += r.n;
            r.state = Q_RUNNING;
            r.info.start_us = now_us(s->t0);
            r.info.slot = sl.idx;
            r.info.merged_rows = 0;
        }
    }
    knng_opts o = s->opts;
    o.flags |= KNNG_FLAG_BALANCED_APPEND;
    o.seed = seed;
    knng_stats st;
    memset(&st, 0, sizeof st);
    Prof prof{(o.flags & KNNG_FLAG_PROFILE) != 0, sl.st};
    std::vector<uint64_t> keys((size_t)nr * s->gstride);
    bool inject = false, committing = false;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t t : tickets)
            inject |= s->fail_ids.erase(s->reqs[t].req_id) > 0;
    }
    const knng_status rc = [&]() -> knng_status {
        Rows R;
        R.x = sl.w.x;
        R.norm = sl.w.norm;
        R.xb = sl.w.xb;
        R.se = sl.w.se;
        R.n = m + nr;
        R.d = s->d;
        R.dp = sl.w.dp;
        R.db = sl.w.db;
        R.split = m;  // the request's rows m .. m+nr-1 are stored at first ..
        R.off2 = first - m;
        HIP_TRY(launch_zero_counters(sl.w.ctr, C_WORDS, sl.st));
        Layout w = sl.w;
        w.rev_m = m;  // rows 0 .. m-1 start from their base lists unless selected
        if (!s->host_rounds) {
            sl.graph.rows_cap = s->capacity;
            w.dev = sl.dev;
            w.graph = &sl.graph;
        }
        if (!sl.fresh)
            HIP_TRY(launch_restore(sl.w.L, sl.w.worst, sl.w.dtag, sl.w.gin, s->gstride, s->k, m,
                                   sl.prev_tag0, sl.st));
        w.tag0 = sl.tag0;
        w.incremental = !sl.fresh;
        sl.fresh = true;  // until this merge ends cleanly
        knng_status r = run_merge(R, w, s->metric, s->bf16, &o, m + nr, m, s->k,
                                  keep_count(&o, s->k), 1, m, nullptr, sl.st, &st, prof, sl.out,
                                  true);
        if (r != KNNG_OK)
            return r;
        if (inject)
            return fail(KNNG_EDEVICE, "request failed on purpose (knng_server_fail_request)");
        committing = true;
        CommitArgs ca;
        ca.out = sl.out;
        ca.gs = s->gstride;
        ca.k = s->k;
        ca.touched = sl.w.dtag;
        ca.tag0 = sl.tag0;
        ca.m_base = m;
        ca.n_req = nr;
        ca.first = first;
        ca.res = s->res;
        ca.ctr = sl.w.ctr;
        HIP_TRY(launch_commit(ca, sl.st));
        HIP_TRY(hipMemcpyAsync(keys.data(), sl.out + m * s->gstride,
                               keys.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, sl.st));
        uint64_t h[C_WORDS];
        r = read_ctr(sl.w.ctr, h, sl.st);
        if (r != KNNG_OK)
            return r;
        if (h[C_ERR])
            return fail(KNNG_EDEVICE, "%s", err_text(h[C_ERR]));
        // every tag this merge wrote is below tag0 + rounds + 2
        sl.prev_tag0 = sl.tag0;
        sl.tag0 += st.rounds + 2;
        sl.fresh = sl.tag0 > (1 << 30);
        if (sl.fresh)
            sl.tag0 = 0;
        return KNNG_OK;
    }();
    const std::string err = rc == KNNG_OK ? std::string() : g_err;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t_done = now_us(s->t0);
        for (uint64_t ticket : tickets) {
            Request &r = s->reqs[ticket];
            r.state = Q_DONE;
            r.rc = rc;
            r.err = err;
            r.info.done_us = t_done;
            r.info.rounds = st.rounds;
            r.info.evals = st.evals;
            r.info.merged_rows = nr;
            r.info.merged_first = first;
            if (rc != KNNG_OK)
                continue;
            // the request's rows, renumbered to their global ids
            const int64_t lo = r.first - first;
            r.keys.resize((size_t)r.n * s->k);
            for (int64_t i = 0; i < r.n; i++)
                for (int j = 0; j < s->k; j++) {
                    uint64_t v = keys[(size_t)(lo + i) * s->gstride + j];
                    const uint32_t id = (uint32_t)v >> 2;
                    if ((uint32_t)(v >> 32) != 0xFFFFFFFFu && id >= (uint64_t)m)
                        v = (v & 0xFFFFFFFF00000003ull) | ((uint64_t)(first + (id - m)) << 2);
                    r.keys[(size_t)i * s->k + j] = v;
                }
        }
        if (rc == KNNG_OK) {
            s->committed += nr;
        } else if (committing) {
            // the resident graph may hold part of this commit: stop serving
            s->failed = true;
            s->fail_text = err;
        } else {
            // failed before its commit: the resident graph and the base are
            // untouched; the request's rows keep their ids with empty lists
            s->dropped += nr;
        }
    }
    if (rc != KNNG_OK && !committing) {
        sl.fresh = true;  // the slot's kept state is unknown: initialise it in full
        const knng_status fr = [&]() -> knng_status {
            HIP_TRY(launch_fill_empty(s->res + first * s->k, nr, s->k, sl.st));
            HIP_TRY(hipStreamSynchronize(sl.st));
            return KNNG_OK;
        }();
        if (fr != KNNG_OK) {
            std::lock_guard<std::mutex> lk(s->mu);
            s->failed = true;
            s->fail_text = g_err;
        }
    }
    s->cv_done.notify_all();
    return rc;
}

// pops the next request -- with batching, every queued request that fits in
// max_request rows (at least one) -- waiting for one when asked; false when
// the server stops, has failed, or (without waiting) nothing is queued
bool next_request(knng_server *s, std::unique_lock<std::mutex> &lk, bool wait,
                  std::vector<uint64_t> *t)
{
    if (wait)
        s->cv_work.wait(lk, [&] { return s->stop || s->failed || !s->pending.empty(); });
    if (s->stop || s->failed || s->pending.empty())
        return false;
    t->clear();
    int64_t rows = 0;
    while (!s->pending.empty()) {
        const Request &r = s->reqs[s->pending.front()];
        if (!t->empty() && (!s->batching || rows + r.n > s->max_request))
            break;
        rows += r.n;
        t->push_back(s->pending.front());
        s->pending.pop_front();
    }
    s->running++;
    return true;
}

void finish_request(knng_server *s)
{
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->running--;
    }
    s->cv_done.notify_all();
}

// run_request, with a host exception (an allocation that failed) turned into
// a failed result for every ticket of the merge instead of leaving them running
knng_status run_request_guarded(knng_server *s, Slot &sl, const std::vector<uint64_t> &t)
{
    try {
        return run_request(s, sl, t);
    } catch (...) {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t_done = now_us(s->t0);
        for (uint64_t ticket : t) {
            auto it = s->reqs.find(ticket);
            if (it == s->reqs.end() || it->second.state == Q_DONE)
                continue;
            it->second.state = Q_DONE;
            it->second.rc = KNNG_ENOMEM;
            it->second.err = "host memory exhausted while merging the request";
            it->second.info.done_us = t_done;
        }
        sl.fresh = true;  // the slot state is unknown: initialise it in full next time
        // whether its commit ran is unknown: stop serving
        s->failed = true;
        s->fail_text = "host memory exhausted while merging a request";
        return fail(KNNG_ENOMEM, "host memory exhausted while merging a request");
    }
}

void slot_main(knng_server *s, Slot *sl)
{
    (void)hipSetDevice(s->device);
    for (;;) {
        std::vector<uint64_t> t;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            if (!next_request(s, lk, true, &t)) {
                if (s->stop)
                    return;
                // failed: leave the queue to the waiters below
                s->cv_done.notify_all();
                return;
            }
        }
        {
            std::shared_lock<std::shared_mutex> state(s->state_mu);
            (void)run_request_guarded(s, *sl, t);
        }
        finish_request(s);
    }
}

// waits until no request is queued or running (caller holds no lock)
knng_status drain(knng_server *s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->manual)
        return s->pending.empty() ? KNNG_OK
                                  : fail(KNNG_EBUSY, "manual server: run the queued requests "
                                                     "with knng_server_step first");
    s->cv_done.wait(lk, [&] { return s->failed || (s->pending.empty() && s->running == 0); });
    return s->failed ? fail(KNNG_EDEVICE, "server failed: %s", s->fail_text.c_str()) : KNNG_OK;
}

} // namespace

extern "C" {

static size_t knng_server_bytes_impl(int64_t capacity, int64_t max_request, int32_t d, int32_t k,
                                     int32_t kin, knng_metric metric, const knng_opts *opts,
                                     int32_t slots)
{
    if (capacity < 2 || max_request < 1 || d < 1 || k < 1 || !opts || slots < 1)
        return 0;
    knng_server probe;
    probe.capacity = capacity;
    probe.max_request = max_request;
    probe.d = d;
    probe.k = k;
    probe.gstride = kin > k ? kin : k;
    probe.metric = metric;
    probe.opts = *opts;
    probe.bf16 = uses_bf16(metric, opts);
    return store_bytes(probe) + (size_t)slots * slot_bytes(probe);
}

size_t knng_server_bytes(int64_t capacity, int64_t max_request, int32_t d, int32_t k, int32_t kin,
                         knng_metric metric, const knng_opts *opts, int32_t slots)
{
    try {
        return knng_server_bytes_impl(capacity, max_request, d, k, kin, metric, opts, slots);
    } catch (const std::bad_alloc &) {
        return 0;
    } catch (...) {
        return 0;
    }
}

static knng_status knng_server_create_impl(const knng_set *base, const knng_graph *G, int32_t k,
                                           knng_metric metric, const knng_opts *opts,
                                           const knng_server_config *cfg, knng_server **out)
{
    knng_status rc;
    if (!out)
        return fail(KNNG_EINVAL, "out is NULL");
    *out = nullptr;
    if ((rc = check_metric(metric)) || (rc = check_set(base, "base")) ||
        (rc = check_opts(opts, k)))
        return rc;
    if (!cfg)
        return fail(KNNG_EINVAL, "cfg is NULL");
    const int64_t m = base->n;
    if (k < 1 || k > MAX_K || k > m - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n_base-1)]", k);
    const int k1 = keep_count(opts, k);
    if ((rc = check_graph_in(G, m, "G", k1)))
        return rc;
    if (cfg->capacity < m || cfg->capacity >= (1ll << 30) - 64)
        return fail(KNNG_EINVAL,
                    "capacity %lld must hold the base (%lld rows) and stay below 2^30 - 64",
                    (long long)cfg->capacity, (long long)m);
    if (cfg->max_request < 1)
        return fail(KNNG_EINVAL, "max_request must be >= 1");
    if (cfg->slots < 0 || cfg->slots > 64)
        return fail(KNNG_EINVAL, "slots %d not in [0, 64]", cfg->slots);
    knng_server *s = new knng_server();
    s->d = base->d;
    s->k = k;
    s->gstride = G->k > k ? G->k : k;
    s->metric = metric;
    s->opts = *opts;
    s->bf16 = uses_bf16(metric, opts);
    s->capacity = cfg->capacity;
    s->max_request = cfg->max_request;
    s->manual = cfg->slots == 0;
    s->batching = cfg->batching != 0;
    s->host_rounds = cfg->host_rounds != 0;
    const size_t gbytes = store_bytes(*s), sbytes = slot_bytes(*s);
    int nslots = s->manual ? 1 : cfg->slots;
    if (cfg->hbm_budget) {
        // as many of the asked-for slots as the budget holds, at least one
        const int64_t fit = cfg->hbm_budget > gbytes
                                ? (int64_t)((cfg->hbm_budget - gbytes) / sbytes)
                                : 0;
        if (fit < 1) {
            delete s;
            return fail(KNNG_ENOMEM, "budget %llu bytes holds no slot (store %zu + slot %zu)",
                        (unsigned long long)cfg->hbm_budget, gbytes, sbytes);
        }
        nslots = fit < nslots ? (int)fit : nslots;
    }
    s->slots.resize(nslots);
    rc = [&]() -> knng_status {
        HIP_TRY(hipGetDevice(&s->device));
        HIP_TRY(hipMalloc(&s->mem, gbytes + (size_t)nslots * sbytes));
        HIP_TRY(hipStreamCreateWithFlags(&s->sub_st, hipStreamNonBlocking));
        Carve c(s->mem);
        carve_store(c, *s);
        for (int i = 0; i < nslots; i++) {
            s->slots[i].idx = i;
            HIP_TRY(hipStreamCreateWithFlags(&s->slots[i].st, hipStreamNonBlocking));
            carve_slot(c, *s, s->slots[i]);
        }
        // base rows and lists into the store (validated, sorted keys); the
        // resident lists start as the base lists.  They are read on the
        // server's own (non-blocking) stream: first let the work the caller
        // queued on the null stream finish.
        HIP_TRY(hipStreamSynchronize(nullptr));
        knng_set none{0, base->d, nullptr};
        Rows R;
        knng_status r =
            prepare(base, G, &none, nullptr, metric, s->bf16, s->store, m, m, s->sub_st, R);
        if (r != KNNG_OK)
            return r;
        HIP_TRY(launch_sort_rows(s->store.gin, s->gstride, m, k, s->res, k, nullptr, nullptr,
                                 s->sub_st));
        return build_rindex(s, m);
    }();
    if (rc != KNNG_OK) {
        const std::string e = g_err;
        for (Slot &sl : s->slots)
            if (sl.st)
                (void)hipStreamDestroy(sl.st);
        if (s->sub_st)
            (void)hipStreamDestroy(s->sub_st);
        if (s->mem)
            (void)hipFree(s->mem);
        delete s;
        return fail(rc, "%s", e.c_str());
    }
    s->m_base = s->reserved = m;
    s->t0 = std::chrono::steady_clock::now();
    if (!s->manual) {
        try {
            for (Slot &sl : s->slots)
                sl.th = std::thread(slot_main, s, &sl);
        } catch (...) {
            knng_server_destroy(s);  // stops and joins the slots that did start
            return fail(KNNG_EDEVICE, "could not start the slot threads");
        }
    }
    *out = s;
    return ok();
}

knng_status knng_server_create(const knng_set *base, const knng_graph *G, int32_t k,
                               knng_metric metric, const knng_opts *opts,
                               const knng_server_config *cfg, knng_server **out)
{
    try {
        return knng_server_create_impl(base, G, k, metric, opts, cfg, out);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

static knng_status knng_server_submit_impl(knng_server *s, const float *raw, int64_t n_raw,
                                           uint64_t req_id, uint64_t *ticket)
{
    if (!s || !ticket)
        return fail(KNNG_EINVAL, "server or ticket is NULL");
    if (!raw || n_raw < 1)
        return fail(KNNG_EINVAL, "a request needs at least one row");
    const double t_submit = now_us(s->t0);
    std::lock_guard<std::mutex> sub_lock(s->sub_mu);
    int64_t row;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed)
            return fail(KNNG_EDEVICE, "server failed earlier: %s", s->fail_text.c_str());
        if (n_raw > s->max_request)
            return fail(KNNG_EINVAL, "request of %lld rows exceeds max_request %lld",
                        (long long)n_raw, (long long)s->max_request);
        if (s->reserved + n_raw > s->capacity)
            return fail(KNNG_ENOMEM, "capacity %lld rows reached", (long long)s->capacity);
        row = s->reserved;
    }
    // pack the rows into their place in the store (no running request reads
    // it), validate them and compute their norms
    const bool on_device = is_device_ptr(raw);
    const knng_status rc = [&]() -> knng_status {
        const Layout &w = s->store;
        const float *src = raw;
        // the rows are read on the server's own (non-blocking) stream: first
        // let the work the caller queued on the null stream finish
        if (on_device)
            HIP_TRY(hipStreamSynchronize(nullptr));
        if (!on_device) {
            HIP_TRY(hipMemcpyAsync(s->stage, raw, (size_t)n_raw * s->d * sizeof(float),
                                   hipMemcpyHostToDevice, s->sub_st));
            src = s->stage;
        }
        HIP_TRY(launch_zero_counters(s->sub_ctr, C_WORDS, s->sub_st));
        HIP_TRY(launch_pack(nullptr, 0, src, n_raw, s->d, w.dp, w.x + row * w.dp,
                            s->bf16 ? w.db : 0, s->bf16 ? w.xb + row * w.db : nullptr,
                            s->bf16 ? w.se + row : nullptr, 1, s->sub_ctr, s->sub_st));
        if (w.norm)
            HIP_TRY(launch_norms(w.x + row * w.dp, n_raw, w.dp, w.norm + row,
                                 s->metric == KNNG_COSINE, s->sub_ctr, s->sub_st));
        uint64_t h[C_WORDS];
        knng_status r = read_ctr(s->sub_ctr, h, s->sub_st);
        if (r != KNNG_OK)
            return r;
        if (h[C_ERR])
            return fail(KNNG_EINVAL, "%s", err_text(h[C_ERR]));
        return KNNG_OK;
    }();
    if (rc != KNNG_OK)
        return rc;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const uint64_t t = s->next_ticket++;
        Request &r = s->reqs[t];
        r.first = row;
        r.n = n_raw;
        r.seed = sm64_host(s->opts.seed ^ sm64_host(req_id));
        r.req_id = req_id;
        r.info.first_id = row;
        r.info.rows = n_raw;
        r.info.submit_us = t_submit;
        r.info.slot = -1;
        s->reserved += n_raw;
        s->pending.push_back(t);
        *ticket = t;
    }
    s->cv_work.notify_one();
    return ok();
}

knng_status knng_server_submit(knng_server *s, const float *raw, int64_t n_raw, uint64_t req_id,
                               uint64_t *ticket)
{
    try {
        return knng_server_submit_impl(s, raw, n_raw, req_id, ticket);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

static knng_status knng_server_step_impl(knng_server *s, int32_t *ran)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    if (!s->manual)
        return fail(KNNG_EINVAL, "knng_server_step needs a server created with slots = 0");
    std::vector<uint64_t> t;
    bool got;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->failed)
            return fail(KNNG_EDEVICE, "server failed earlier: %s", s->fail_text.c_str());
        got = next_request(s, lk, false, &t);
    }
    if (ran)
        *ran = got ? 1 : 0;
    if (!got)
        return ok();
    {
        std::shared_lock<std::shared_mutex> state(s->state_mu);
        (void)run_request_guarded(s, s->slots[0], t);
    }
    finish_request(s);
    // the request's own result goes to knng_server_wait; step fails only
    // when the server itself has failed
    std::lock_guard<std::mutex> lk(s->mu);
    return s->failed ? fail(KNNG_EDEVICE, "server failed: %s", s->fail_text.c_str()) : ok();
}

knng_status knng_server_step(knng_server *s, int32_t *ran)
{
    try {
        return knng_server_step_impl(s, ran);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

static knng_status knng_server_wait_impl(knng_server *s, uint64_t ticket, int64_t timeout_us,
                                         int32_t *ids, float *dist, knng_request_info *info)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return fail(KNNG_EINVAL, "unknown or already collected ticket %llu",
                    (unsigned long long)ticket);
    auto done = [&] { return it->second.state == Q_DONE || (s->failed && it->second.state ==
                                                                          Q_PENDING); };
    if (timeout_us < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
        return fail(KNNG_EBUSY, "request %llu not finished yet", (unsigned long long)ticket);
    if (it->second.state == Q_PENDING) {
        // the server failed before this request ran
        knng_request_info inf = it->second.info;
        s->reqs.erase(it);
        if (info)
            *info = inf;
        return fail(KNNG_EDEVICE, "server failed before the request ran: %s",
                    s->fail_text.c_str());
    }
    Request r = std::move(it->second);
    s->reqs.erase(it);
    lk.unlock();
    if (info)
        *info = r.info;
    if (r.rc != KNNG_OK)
        return fail(r.rc, "%s", r.err.c_str());
    if (ids || dist) {
        const size_t cnt = (size_t)r.n * s->k;
        std::vector<int32_t> hi(cnt);
        std::vector<float> hd(cnt);
        for (size_t e = 0; e < cnt; e++) {
            const uint64_t v = r.keys[e];
            const bool empty = (uint32_t)(v >> 32) == 0xFFFFFFFFu;
            hi[e] = empty ? -1 : (int32_t)((uint32_t)v >> 2);
            uint32_t bits = empty ? 0x7F800000u : (uint32_t)(v >> 32);
            memcpy(&hd[e], &bits, 4);
        }
        if (ids)
            HIP_TRY(hipMemcpy(ids, hi.data(), cnt * sizeof(int32_t), hipMemcpyDefault));
        if (dist)
            HIP_TRY(hipMemcpy(dist, hd.data(), cnt * sizeof(float), hipMemcpyDefault));
    }
    return ok();
}

knng_status knng_server_wait(knng_server *s, uint64_t ticket, int64_t timeout_us, int32_t *ids,
                             float *dist, knng_request_info *info)
{
    try {
        return knng_server_wait_impl(s, ticket, timeout_us, ids, dist, info);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

static knng_status knng_server_snapshot_impl(knng_server *s, knng_graph *out, int64_t *n_rows)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    knng_status rc = drain(s);
    if (rc != KNNG_OK)
        return rc;
    std::unique_lock<std::shared_mutex> state(s->state_mu);  // no request in a slot
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->m_base + s->committed + s->dropped != s->reserved)
            return fail(KNNG_EBUSY, "requests were submitted during the snapshot");
        n = s->reserved;
    }
    if (n_rows)
        *n_rows = n;
    if (!out)
        return ok();
    if (out->n < n || out->k != s->k)
        return fail(KNNG_EINVAL, "out is %lld x %d, needs at least %lld x %d",
                    (long long)out->n, out->k, (long long)n, s->k);
    if (!is_device_ptr(out->ids) || !is_device_ptr(out->dist))
        return fail(KNNG_EINVAL, "out->ids / out->dist must be device memory");
    HIP_TRY(launch_sort_rows(s->res, s->k, n, s->k, nullptr, 0, out->ids, out->dist, s->sub_st));
    HIP_TRY(hipStreamSynchronize(s->sub_st));
    return ok();
}

knng_status knng_server_snapshot(knng_server *s, knng_graph *out, int64_t *n_rows)
{
    try {
        return knng_server_snapshot_impl(s, out, n_rows);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

static knng_status knng_server_rebase_impl(knng_server *s)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    knng_status rc = drain(s);
    if (rc != KNNG_OK)
        return rc;
    std::unique_lock<std::shared_mutex> state(s->state_mu);
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->m_base + s->committed + s->dropped != s->reserved)
            return fail(KNNG_EBUSY, "requests were submitted during the rebase");
        n = s->reserved;
    }
    // the resident graph, sorted, becomes the base lists
    HIP_TRY(launch_sort_rows(s->res, s->k, n, s->k, s->store.gin, s->gstride, nullptr, nullptr,
                             s->sub_st));
    rc = build_rindex(s, n);
    if (rc != KNNG_OK)
        return rc;
    for (Slot &sl : s->slots)
        sl.fresh = true;  // new base lists: the kept merge state is stale
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->m_base = n;
        s->committed = 0;
        s->dropped = 0;
    }
    return ok();
}

knng_status knng_server_rebase(knng_server *s)
{
    try {
        return knng_server_rebase_impl(s);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

knng_status knng_server_status(knng_server *s, int64_t *base_rows, int64_t *committed_rows,
                               int64_t *pending_rows)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (base_rows)
        *base_rows = s->m_base;
    if (committed_rows)
        *committed_rows = s->committed;
    if (pending_rows)
        *pending_rows = s->reserved - s->m_base - s->committed - s->dropped;
    return s->failed ? fail(KNNG_EDEVICE, "server failed: %s", s->fail_text.c_str()) : ok();
}

int32_t knng_server_slots(const knng_server *s) { return s ? (int32_t)s->slots.size() : 0; }

knng_status knng_server_fail_request(knng_server *s, uint64_t req_id)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    try {
        std::lock_guard<std::mutex> lk(s->mu);
        s->fail_ids.insert(req_id);
    } catch (...) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    }
    return ok();
}

void knng_server_destroy(knng_server *s)
{
    if (!s)
        return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    for (Slot &sl : s->slots)
        if (sl.th.joinable())
            sl.th.join();  // a request in a slot finishes first
    for (Slot &sl : s->slots) {
        (void)hipStreamSynchronize(sl.st);
        if (sl.graph.exec)
            (void)hipGraphExecDestroy(sl.graph.exec);
        if (sl.graph.graph)
            (void)hipGraphDestroy(sl.graph.graph);
        (void)hipStreamDestroy(sl.st);
    }
    (void)hipStreamSynchronize(s->sub_st);
    (void)hipStreamDestroy(s->sub_st);
    (void)hipFree(s->mem);
    delete s;
}

} // extern "C"
