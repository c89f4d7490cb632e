// knng_server.hip -- J-Merge serving: a resident point set with its k-NN
// graph absorbs requests of raw rows (Section 3.2: a built graph takes in
// raw data without being rebuilt).  Requests are merged in batches: every
// request waiting when the device turns free joins the next batch
// (continuous batching), and a batch is one joint merge of the resident rows
// with the batch's rows under balanced append.
//
// Device memory is allocated once at creation (the merge state for the full
// capacity, the resident graph as sorted keys, a staging buffer) and rows
// are never moved: request rows are packed at submission into their final
// place, so a batch reads them where they are and its Merge and Sort writes
// the new resident graph in place.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>

#include "knng_host.h"

using namespace knng;
using namespace knng::host;

namespace {

enum ReqState { Q_PENDING = 0, Q_RUNNING = 1, Q_DONE = 2 };

struct Request {
    int64_t first = 0, n = 0;
    int state = Q_PENDING;
    knng_status rc = KNNG_OK;
    std::string err;
    std::vector<uint64_t> keys;  // n x k result keys, filled at batch end
    knng_request_info info{};
};

double now_us(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0)
        .count();
}

} // namespace

struct knng_server {
    int device = 0;
    int d = 0, k = 0, gstride = 0;
    knng_metric metric = KNNG_L2;
    knng_opts opts{};
    bool bf16 = false;
    int64_t capacity = 0, max_batch = 0;
    void *mem = nullptr;
    Layout w{};
    float *stage = nullptr;     // max_batch x d: host rows on their way in
    uint64_t *sub_ctr = nullptr;
    hipStream_t run_st = nullptr, sub_st = nullptr;
    std::chrono::steady_clock::time_point t0;

    std::mutex mu;        // everything below
    std::mutex run_mu;    // held while a batch runs or the graph is read out
    std::mutex sub_mu;    // one submission at a time
    std::condition_variable cv_work, cv_done;
    int64_t resident = 0;  // rows merged (base + finished batches)
    int64_t reserved = 0;  // rows taken by accepted submissions
    uint64_t next_ticket = 1;
    int64_t batches = 0;
    std::deque<uint64_t> pending;
    std::map<uint64_t, Request> reqs;
    bool stop = false, manual = false, failed = false;
    std::string fail_text;
    std::thread worker;
};

namespace {

// the device layout of a server; with base == nullptr it only measures
void carve_server(Carve &c, knng_server &s, int s_sample)
{
    carve_merge(c, s.w, s.capacity, s.capacity, s.d, s.k, s.gstride, s_sample, s.metric,
                s.bf16);
    s.stage = c.take<float>((size_t)s.max_batch * s.d);
    s.sub_ctr = c.take<uint64_t>(C_WORDS);
}

Rows rows_of(const knng_server &s, int64_t n)
{
    Rows R;
    R.x = s.w.x;
    R.norm = s.w.norm;
    R.xb = s.w.xb;
    R.sq = s.w.sq;
    R.eb = s.w.eb;
    R.n = n;
    R.d = s.d;
    R.dp = s.w.dp;
    R.db = s.w.db;
    return R;
}

// One batch: every pending request that fits in max_batch rows (at least
// one), merged into the resident graph.  Caller holds no lock.
knng_status run_batch(knng_server *s, bool *ran)
{
    std::lock_guard<std::mutex> run_lock(s->run_mu);
    std::vector<uint64_t> tickets;
    int64_t rows = 0, m = 0, batch = 0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->failed)
            return fail(KNNG_EDEVICE, "server failed earlier: %s", s->fail_text.c_str());
        while (!s->pending.empty()) {
            Request &r = s->reqs[s->pending.front()];
            if (rows > 0 && rows + r.n > s->max_batch)
                break;
            rows += r.n;
            tickets.push_back(s->pending.front());
            s->pending.pop_front();
            r.state = Q_RUNNING;
            r.info.start_us = now_us(s->t0);
        }
        m = s->resident;
        if (!tickets.empty())
            batch = s->batches++;
    }
    *ran = !tickets.empty();
    if (tickets.empty())
        return ok();
    knng_opts o = s->opts;
    o.flags |= KNNG_FLAG_BALANCED_APPEND;
    o.seed = s->opts.seed + (uint64_t)batch;
    const int64_t n = m + rows;
    knng_stats st;
    memset(&st, 0, sizeof st);
    Prof prof{(o.flags & KNNG_FLAG_PROFILE) != 0, s->run_st};
    std::vector<uint64_t> keys((size_t)rows * s->gstride);
    knng_status rc = [&]() -> knng_status {
        HIP_TRY(launch_zero_counters(s->w.ctr, C_WORDS, s->run_st));
        const Rows R = rows_of(*s, n);
        knng_status r = run_merge(R, s->w, s->metric, s->bf16, &o, n, m, s->k,
                                  keep_count(&o, s->k), 1, m, nullptr, s->run_st, &st, prof,
                                  s->w.gin);
        if (r != KNNG_OK)
            return r;
        HIP_TRY(hipMemcpyAsync(keys.data(), s->w.gin + m * s->gstride,
                               keys.size() * sizeof(uint64_t), hipMemcpyDeviceToHost,
                               s->run_st));
        HIP_TRY(hipStreamSynchronize(s->run_st));
        return KNNG_OK;
    }();
    const std::string err = rc == KNNG_OK ? std::string() : g_err;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const double t = now_us(s->t0);
        if (rc == KNNG_OK) {
            s->resident = n;
        } else {
            // the resident graph may be half written: nothing more runs
            s->failed = true;
            s->fail_text = err;
        }
        for (uint64_t tk : tickets) {
            Request &r = s->reqs[tk];
            r.state = Q_DONE;
            r.rc = rc;
            r.err = err;
            r.info.done_us = t;
            r.info.batch = batch;
            r.info.batch_rows = rows;
            r.info.rounds = st.rounds;
            r.info.evals = st.evals;
            if (rc == KNNG_OK) {
                r.keys.resize((size_t)r.n * s->k);
                for (int64_t i = 0; i < r.n; i++)
                    for (int j = 0; j < s->k; j++)
                        r.keys[i * s->k + j] = keys[(r.first - m + i) * s->gstride + j];
            }
        }
        if (s->failed) {
            // requests still queued cannot run any more
            for (uint64_t tk : s->pending) {
                Request &r = s->reqs[tk];
                r.state = Q_DONE;
                r.rc = KNNG_EDEVICE;
                r.err = "server failed: " + err;
                r.info.done_us = t;
            }
            s->pending.clear();
        }
    }
    s->cv_done.notify_all();
    return rc;
}

void worker_main(knng_server *s)
{
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        s->cv_work.wait(lk, [&] { return s->stop || (!s->pending.empty() && !s->failed); });
        if (s->stop)
            return;
        lk.unlock();
        bool ran = false;
        (void)run_batch(s, &ran);
        lk.lock();
    }
}

size_t server_bytes(knng_server &probe, int sample)
{
    Carve c(nullptr);
    carve_server(c, probe, sample);
    return c.off + 256;
}

} // namespace

extern "C" {

size_t knng_server_bytes(int64_t capacity, int64_t max_batch, int32_t d, int32_t k, int32_t kin,
                         knng_metric metric, const knng_opts *opts)
{
    if (capacity < 2 || max_batch < 1 || d < 1 || k < 1 || !opts)
        return 0;
    knng_server probe;
    probe.capacity = capacity;
    probe.max_batch = max_batch;
    probe.d = d;
    probe.k = k;
    probe.gstride = kin > k ? kin : k;
    probe.metric = metric;
    probe.bf16 = uses_bf16(metric, opts);
    return server_bytes(probe, opts->sample);
}

knng_status knng_server_create(const knng_set *base, const knng_graph *G, int32_t k,
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
        return fail(KNNG_EINVAL, "capacity %lld must hold the base (%lld rows) and stay below 2^30",
                    (long long)cfg->capacity, (long long)m);
    if (cfg->max_batch < 1)
        return fail(KNNG_EINVAL, "max_batch must be >= 1");
    knng_server *s = new knng_server();
    s->d = base->d;
    s->k = k;
    s->gstride = G->k > k ? G->k : k;
    s->metric = metric;
    s->opts = *opts;
    s->bf16 = uses_bf16(metric, opts);
    s->capacity = cfg->capacity;
    s->max_batch = cfg->max_batch < cfg->capacity - m ? cfg->max_batch : cfg->capacity - m;
    if (s->max_batch < 1)
        s->max_batch = 1;
    s->manual = cfg->manual != 0;
    const size_t bytes = server_bytes(*s, opts->sample);
    if (cfg->hbm_budget && bytes > cfg->hbm_budget) {
        delete s;
        return fail(KNNG_ENOMEM, "server needs %zu device bytes, budget %zu", bytes,
                    (size_t)cfg->hbm_budget);
    }
    rc = [&]() -> knng_status {
        HIP_TRY(hipGetDevice(&s->device));
        HIP_TRY(hipMalloc(&s->mem, bytes));
        HIP_TRY(hipStreamCreateWithFlags(&s->run_st, hipStreamNonBlocking));
        HIP_TRY(hipStreamCreateWithFlags(&s->sub_st, hipStreamNonBlocking));
        Carve c(s->mem);
        carve_server(c, *s, opts->sample);
        HIP_TRY(launch_zero_counters(s->sub_ctr, C_WORDS, s->run_st));
        // base rows and their lists (validated, sorted keys) into the layout
        knng_set none{0, base->d, nullptr};
        Rows R;
        knng_status r = prepare(base, G, &none, nullptr, metric, s->bf16, s->w, m, m, s->run_st, R);
        if (r != KNNG_OK)
            return r;
        HIP_TRY(hipStreamSynchronize(s->run_st));
        return KNNG_OK;
    }();
    if (rc != KNNG_OK) {
        const std::string e = g_err;
        if (s->run_st)
            (void)hipStreamDestroy(s->run_st);
        if (s->sub_st)
            (void)hipStreamDestroy(s->sub_st);
        if (s->mem)
            (void)hipFree(s->mem);
        delete s;
        return fail(rc, "%s", e.c_str());
    }
    s->resident = s->reserved = m;
    s->t0 = std::chrono::steady_clock::now();
    if (!s->manual)
        s->worker = std::thread(worker_main, s);
    *out = s;
    return ok();
}

knng_status knng_server_submit(knng_server *s, const float *raw, int64_t n_raw,
                               uint64_t *ticket)
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
        if (n_raw > s->max_batch)
            return fail(KNNG_EINVAL, "request of %lld rows exceeds max_batch %lld",
                        (long long)n_raw, (long long)s->max_batch);
        if (s->reserved + n_raw > s->capacity)
            return fail(KNNG_ENOMEM, "capacity %lld rows reached", (long long)s->capacity);
        row = s->reserved;
    }
    // pack the rows into their final place (disjoint from every row a running
    // batch reads), validate them, and compute their norms
    const bool on_device = is_device_ptr(raw);
    const knng_status rc = [&]() -> knng_status {
        const float *src = raw;
        if (!on_device) {
            HIP_TRY(hipMemcpyAsync(s->stage, raw, (size_t)n_raw * s->d * sizeof(float),
                                   hipMemcpyHostToDevice, s->sub_st));
            src = s->stage;
        }
        HIP_TRY(launch_zero_counters(s->sub_ctr, C_WORDS, s->sub_st));
        HIP_TRY(launch_pack(nullptr, 0, src, n_raw, s->d, s->w.dp, s->w.x + row * s->w.dp,
                            s->bf16 ? s->w.db : 0, s->bf16 ? s->w.xb + row * s->w.db : nullptr,
                            s->sub_ctr, s->sub_st));
        if (s->w.norm || s->w.sq)
            HIP_TRY(launch_norms(s->w.x + row * s->w.dp, n_raw, s->w.dp,
                                 s->w.norm ? s->w.norm + row : nullptr,
                                 s->w.sq ? s->w.sq + row : nullptr,
                                 s->w.eb ? s->w.eb + row : nullptr, s->metric == KNNG_COSINE,
                                 s->sub_ctr, s->sub_st));
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
        r.info.first_id = row;
        r.info.submit_us = t_submit;
        r.info.batch = -1;
        s->reserved += n_raw;
        s->pending.push_back(t);
        *ticket = t;
    }
    s->cv_work.notify_one();
    return ok();
}

knng_status knng_server_step(knng_server *s, int32_t *ran)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    if (!s->manual)
        return fail(KNNG_EINVAL, "knng_server_step needs a server created with manual = 1");
    bool r = false;
    const knng_status rc = run_batch(s, &r);
    if (ran)
        *ran = r ? 1 : 0;
    return rc;
}

knng_status knng_server_wait(knng_server *s, uint64_t ticket, int64_t timeout_us, int32_t *ids,
                             float *dist, knng_request_info *info)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end())
        return fail(KNNG_EINVAL, "unknown or already collected ticket %llu",
                    (unsigned long long)ticket);
    auto done = [&] { return it->second.state == Q_DONE; };
    if (timeout_us < 0)
        s->cv_done.wait(lk, done);
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), done))
        return fail(KNNG_EBUSY, "request %llu not finished yet", (unsigned long long)ticket);
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

knng_status knng_server_snapshot(knng_server *s, knng_graph *out, int64_t *n_rows)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> run_lock(s->run_mu);
    int64_t n;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        n = s->resident;
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
    HIP_TRY(launch_keys_to_graph(s->w.gin, s->gstride, n, s->k, out->ids, out->dist, s->run_st));
    HIP_TRY(hipStreamSynchronize(s->run_st));
    return ok();
}

knng_status knng_server_status(knng_server *s, int64_t *resident_rows, int64_t *pending_rows,
                               int64_t *batches)
{
    if (!s)
        return fail(KNNG_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (resident_rows)
        *resident_rows = s->resident;
    if (pending_rows)
        *pending_rows = s->reserved - s->resident;
    if (batches)
        *batches = s->batches;
    return s->failed ? fail(KNNG_EDEVICE, "server failed: %s", s->fail_text.c_str()) : ok();
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
    if (s->worker.joinable())
        s->worker.join();  // a batch in flight finishes first
    (void)hipStreamSynchronize(s->run_st);
    (void)hipStreamSynchronize(s->sub_st);
    (void)hipStreamDestroy(s->run_st);
    (void)hipStreamDestroy(s->sub_st);
    (void)hipFree(s->mem);
    delete s;
}

} // extern "C"
