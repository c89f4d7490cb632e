// knng_api.hip -- the C ABI of libknngmerge (declared in include/knng_merge.h):
// argument checking, workspace carving and the host side of the merges.
//
// Host orchestration of Algorithms 1 and 2 (Zhao et al., "On the Merge of
// k-NN Graph", Sections 3.1-3.2): Divide/Append (or Initialize), then the
// repeat loop -- per round: sampling, Reverse(G), local join -- until the
// number of surviving insertions c drops to delta*n*k, then Merge and Sort.
#include <chrono>

#include "knng_host.h"

#include <new>

#include <thread>

using namespace knng;
using namespace knng::host;

namespace knng {
namespace host {

// layout + input preparation shared by both merges.  Rows [0, n1) come from
// set A (input lists of A on rows [0, n1)), rows [n1, n) from set B (input
// lists only when listsB).
knng_status prepare(const knng_set *A, const knng_graph *GA, const knng_set *B,
                    const knng_graph *GB, knng_metric metric, bool bf16, const Layout &w,
                    int64_t n1, int64_t n, hipStream_t st, Rows &R)
{
    const int d = B->d;
    HIP_TRY(launch_zero_counters(w.ctr, C_WORDS, st));
    HIP_TRY(launch_pack(A->n ? A->x : nullptr, n1, B->x, n - n1, d, w.dp, w.x,
                        bf16 ? w.db : 0, bf16 ? w.xb : nullptr, bf16 ? w.se : nullptr, w.ws,
                        w.ctr, st));
    R.x = w.x;
    R.xb = bf16 ? w.xb : nullptr;
    R.db = w.db;
    R.norm = w.norm;
    R.se = w.se;
    R.se_stride = w.ws;
    R.n = n;
    R.d = d;
    R.dp = w.dp;
    if (w.norm)
        HIP_TRY(launch_norms(w.x, n, w.dp, w.norm, metric == KNNG_COSINE, w.ctr, st));
    uint64_t h[C_WORDS];
    knng_status s = read_ctr(w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EINVAL, "%s", err_text(h[C_ERR]));
    if (GA && n1 > 0)
        HIP_TRY(launch_prep_input(R, metric, 0, n1, 0, n1, GA->ids, GA->dist, GA->k, w.gstride,
                                  w.gin, w.ctr, st));
    if (GB)
        HIP_TRY(launch_prep_input(R, metric, n1, n - n1, n1, n - n1, GB->ids, GB->dist, GB->k,
                                  w.gstride, w.gin, w.ctr, st));
    s = read_ctr(w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EINVAL, "%s", err_text(h[C_ERR]));
    return KNNG_OK;
}

// Graph mode: capture the slot's round once (sampling, the last round's
// count, the loop control, Reverse(G), the local join, the round advance),
// then per merge set the device round state and replay the round until the
// device has ended the loop.
static knng_status replay_rounds(const Rows &R, const Layout &w, knng_metric metric, bool bf16,
                                 const knng_opts *o, const RoundArgs &a0, int64_t n, int64_t n1,
                                 hipStream_t st, int *rounds)
{
    RoundGraph &G = *w.graph;
    if (!G.exec) {
        // grids of the captured launches are sized for the slot's largest merge
        RoundArgs ag = a0;
        ag.dev = w.dev;
        ag.n = G.rows_cap;
        ag.n_active = G.rows_cap;
        ag.rev_m = G.rows_cap;
        Rows Rg = R;
        Rg.n = G.rows_cap;
        HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        hipError_t e = launch_sample(ag, st);
        if (e == hipSuccess)
            e = launch_count_fresh(ag, st);
        if (e == hipSuccess)
            e = launch_round_ctl(ag, a0.k, st);
        if (e == hipSuccess)
            e = launch_prep_active(ag, st);
        if (e == hipSuccess)
            e = launch_reverse_indexed(ag, st);
        if (e == hipSuccess)
            e = launch_join(Rg, (int)metric, bf16 ? 1 : 0, ag, st);
        if (e == hipSuccess)
            e = launch_round_next(ag, st);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(st, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g)
                (void)hipGraphDestroy(g);
            return fail(KNNG_EDEVICE, "capturing the round graph failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        }
        G.graph = g;
        HIP_TRY(hipGraphInstantiate(&G.exec, G.graph, nullptr, nullptr, 0));
    }
    DevRound v{};
    v.round = 0;
    v.done = 0;
    v.rounds = 0;
    v.tag0 = a0.tag0;
    v.max_rounds = o->max_rounds;
    v.n = n;
    v.n1 = n1;
    v.n_active = 0;
    v.rev_m = a0.rev_m;
    v.split = R.split;
    v.off2 = R.off2;
    v.seed = o->seed;
    v.delta = (double)o->delta;
    HIP_TRY(launch_set_round(w.dev, v, st));
    // round t ends the loop in replay t + 1; most merges take 6-12 rounds
    int replays = 0;
    for (int block = 8;; block = 4) {
        for (int b = 0; b < block; b++)
            HIP_TRY(hipGraphLaunch(G.exec, st));
        replays += block;
        DevRound hd;
        HIP_TRY(hipMemcpyAsync(&hd, w.dev, sizeof hd, hipMemcpyDeviceToHost, st));
        uint64_t h[C_WORDS];
        knng_status s = read_ctr(w.ctr, h, st);
        if (s != KNNG_OK)
            return s;
        if (h[C_ERR])
            return fail(KNNG_EDEVICE, "%s", err_text(h[C_ERR]));
        if (hd.done) {
            *rounds = hd.rounds;
            return KNNG_OK;
        }
        if (replays > o->max_rounds + 1)
            return fail(KNNG_EDEVICE, "the round graph did not end the loop in %d replays",
                        replays);
    }
}

// the repeat loop and Merge and Sort, shared by S-Merge and J-Merge
knng_status run_merge(const Rows &R, const Layout &w, knng_metric metric, bool bf16,
                      const knng_opts *o, int64_t n, int64_t n1, int k, int k1, int joint,
                      int64_t rows_with_rear, knng_graph *out, hipStream_t st, knng_stats *stats,
                      Prof &prof, uint64_t *out_keys, bool touched_only)
{
    const int balanced = joint && (o->flags & KNNG_FLAG_BALANCED_APPEND) ? 1 : 0;
    InitArgs ia;
    ia.L = w.L;
    ia.worst = w.worst;
    ia.ws = w.ws;
    ia.dtag = w.dtag;
    ia.atag = w.atag;
    ia.balanced = balanced;
    ia.gin = w.gin;
    ia.kin = w.gstride;
    ia.k = k;
    ia.k1 = k1;
    ia.n = n;
    ia.n1 = n1;
    ia.joint = joint;
    ia.seed = o->seed;
    ia.ctr = w.ctr;
    ia.tag0 = w.tag0;
    ia.incremental = w.incremental ? 1 : 0;
    prof.begin(PH_INIT);
    HIP_TRY(launch_init(R, (int)metric, ia, st));
    prof.end();

    RoundArgs a;
    a.L = w.L;
    a.worst = w.worst;
    a.ws = w.ws;
    a.new_f = w.new_f;
    a.old_f = w.old_f;
    a.cnt_f = w.cnt_f;
    a.rnew = w.rnew;
    a.rold = w.rold;
    a.dtag = w.dtag;
    a.atag = w.atag;
    a.rfill = w.rfill;
    a.ctr = w.ctr;
    a.rev_off = w.rev_off;
    a.rev_src = w.rev_src;
    a.rev_m = w.rev_m;
    a.tag0 = w.tag0;
    a.alist = w.alist;
    a.n_active = 0;
    a.n = n;
    a.n1 = n1;
    a.k = k;
    a.s = o->sample;
    a.joint = joint;
    a.seed = o->seed;
    uint64_t h[C_WORDS];
    int rounds = 0;
    if (w.graph) {
        // graph mode: the round is a captured launch graph, replayed in blocks
        // with one read-back per block; the device ends the loop itself
        knng_status gs = replay_rounds(R, w, metric, bf16, o, a, n, n1, st, &rounds);
        if (gs != KNNG_OK)
            return gs;
    }
    for (int t = 0; !w.graph; t++) {
        const bool last = t == o->max_rounds;
        a.round = t;
        prof.begin(PH_SAMPLE);
        if (!last)
            HIP_TRY(launch_sample(a, st));  // also counts the FRESH entries of round t-1
        else
            HIP_TRY(launch_count_fresh(a, st));
        prof.end();
        if (t > 0 || a.alist) {
            knng_status s = read_ctr(w.ctr, h, st);
            if (s != KNNG_OK)
                return s;
            if (h[C_ERR])
                return fail(KNNG_EDEVICE, "%s", err_text(h[C_ERR]));
            a.n_active = (int64_t)h[C_ACTIVE];  // list mode: the round's active rows
        }
        if (t > 0) {
            if (stats && t - 1 < KNNG_STATS_ROUNDS) {
                stats->updates[t - 1] = (int64_t)h[C_FRESH];
                stats->pairs[t - 1] = (int64_t)h[C_PAIRS];
                stats->gathered[t - 1] = (int64_t)h[C_GATHER];
            }
            rounds = t;
            // delta is relative to the rows that started the loop with NEW
            // entries (all rows, except under balanced append)
            if ((double)h[C_FRESH] <= (double)o->delta * (double)h[C_N0] * (double)k)
                break;
        }
        if (last)
            break;
        HIP_TRY(launch_zero_counters(w.ctr, C_ROUND_WORDS, st));
        prof.begin(PH_REVERSE);
        HIP_TRY(launch_prep_active(a, st));
        if (a.rev_off)
            HIP_TRY(launch_reverse_indexed(a, st));
        else
            HIP_TRY(launch_reverse(a, st));
        prof.end();
        prof.begin(PH_JOIN);
        HIP_TRY(launch_join(R, (int)metric, bf16 ? 1 : 0, a, st));
        prof.end();
    }
    prof.begin(PH_FINAL);
    FinalArgs fa;
    fa.L = w.L;
    fa.gin = w.gin;
    fa.k = k;
    fa.kin = w.gstride;
    fa.k1 = k1;
    fa.rows_with_rear = rows_with_rear;
    fa.n = n;
    fa.balanced = balanced;
    fa.n_raw = n - n1;
    fa.seed = o->seed;
    fa.out_ids = out ? out->ids : nullptr;
    fa.out_dist = out ? out->dist : nullptr;
    fa.out_keys = out_keys;
    fa.touched = touched_only ? w.dtag : nullptr;
    fa.tag0 = w.tag0;
    HIP_TRY(launch_final(fa, st));
    prof.end();
    knng_status s = read_ctr(w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EDEVICE, "%s", err_text(h[C_ERR]));
    if (stats) {
        stats->rounds = rounds;
        stats->evals = (int64_t)h[C_EVALS];
        stats->rescored = (int64_t)h[C_RESCORE];
        stats->insert_attempts = (int64_t)h[C_ATTEMPT];
        stats->screen_violations = (int64_t)h[C_VIOL];
        stats->max_group = (int32_t)h[C_MAXG];
    }
    prof.collect(stats);
    // A rescored pair whose bf16 distance left the proven margin means the
    // bound failed, and a pair it screened out may have been lost: the
    // result is not trusted (the count is in stats->screen_violations).
    if (h[C_VIOL])
        return fail(KNNG_EDEVICE, "BF16 screen: %llu rescored pairs left the error margin",
                    (unsigned long long)h[C_VIOL]);
    return ok();
}


} // namespace host
} // namespace knng

extern "C" {

void knng_opts_default(knng_opts *o)
{
    if (!o)
        return;
    o->keep_ratio = 0.5f;
    o->sample = 10;
    o->delta = 0.0f;
    o->max_rounds = 30;
    o->seed = 0;
    o->precision = KNNG_FP32;
    o->flags = 0;
}

const char *knng_last_error(void) { return g_err.c_str(); }

int knng_version(void) { return KNNG_VERSION; }

size_t knng_merge_workspace_size(int64_t n1, int64_t n2, int32_t d, int32_t k, int32_t kin1,
                                 int32_t kin2, knng_metric metric, const knng_opts *opts)
{
    if (n1 < 1 || n2 < 1 || d < 1 || k < 1 || !opts)
        return 0;
    Carve c(nullptr);
    Layout w;
    carve_merge(c, w, n1 + n2, n1 + n2, d, k, kin1 > kin2 ? kin1 : kin2, opts->sample, metric,
                uses_bf16(metric, opts));
    return c.off + 256;
}

size_t knng_expand_workspace_size(int64_t n_base, int64_t n_raw, int32_t d, int32_t k,
                                  int32_t kin, knng_metric metric, const knng_opts *opts)
{
    if (n_base < 0 || n_raw < 1 || d < 1 || k < 1 || !opts)
        return 0;
    Carve c(nullptr);
    Layout w;
    carve_merge(c, w, n_base + n_raw, n_base, d, k, n_base > 0 ? kin : 0, opts->sample, metric,
                uses_bf16(metric, opts));
    return c.off + 256;
}

// ws_is_device: the workspace is known to be device memory (the library's
// own static scratch, which hipPointerGetAttributes need not know)
static knng_status knng_merge_impl(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                                   const knng_graph *G2, int32_t k, knng_metric metric,
                                   const knng_opts *opts, knng_graph *out, void *workspace,
                                   size_t workspace_bytes, void *stream, knng_stats *stats,
                                   bool ws_is_device = false)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(S1, "S1")) || (s = check_set(S2, "S2")) ||
        (s = check_opts(opts, k)))
        return s;
    if (S1->d != S2->d)
        return fail(KNNG_EINVAL, "S1->d = %d differs from S2->d = %d", S1->d, S2->d);
    const int64_t n1 = S1->n, n2 = S2->n, n = n1 + n2;
    // a list entry holds a row id in 30 bits
    if (n >= (1ll << 30) - 64)
        return fail(KNNG_EINVAL, "n1 + n2 = %lld rows out of range", (long long)n);
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n1+n2-1)]", k);
    const int k1 = keep_count(opts, k);
    if ((s = check_graph_in(G1, n1, "G1", k1)) || (s = check_graph_in(G2, n2, "G2", k1)) ||
        (s = check_out(out, n, k)))
        return s;
    const bool bf16 = uses_bf16(metric, opts);
    const int gstride = G1->k > G2->k ? G1->k : G2->k;
    const size_t need = knng_merge_workspace_size(n1, n2, S1->d, k, G1->k, G2->k, metric, opts);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!ws_is_device && !is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    if (stats)
        memset(stats, 0, sizeof *stats);
    Carve c(workspace);
    Layout w;
    carve_merge(c, w, n, n, S1->d, k, gstride, opts->sample, metric, bf16);
    Prof prof{(opts->flags & KNNG_FLAG_PROFILE) != 0, st};
    Rows R;
    prof.begin(PH_PREP);
    s = prepare(S1, G1, S2, G2, metric, bf16, w, n1, n, st, R);
    prof.end();
    if (s != KNNG_OK)
        return s;
    return run_merge(R, w, metric, bf16, opts, n, n1, k, k1, 0, n, out, st, stats, prof);
}

knng_status knng_merge(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                       const knng_graph *G2, int32_t k, knng_metric metric,
                       const knng_opts *opts, knng_graph *out, void *workspace,
                       size_t workspace_bytes, void *stream, knng_stats *stats)
{
    try {
        return knng_merge_impl(S1, G1, S2, G2, k, metric, opts, out, workspace, workspace_bytes,
                               stream, stats);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

} // extern "C"

namespace knng {
namespace host {
// knng_merge on device memory the caller vouches for (the no-allocation
// entry point's static scratch)
knng_status merge_on_scratch(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                             const knng_graph *G2, int32_t k, knng_metric metric,
                             const knng_opts *opts, knng_graph *out, void *scratch,
                             size_t scratch_bytes, void *stream, knng_stats *stats)
{
    try {
        return knng_merge_impl(S1, G1, S2, G2, k, metric, opts, out, scratch, scratch_bytes,
                               stream, stats, true);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}
} // namespace host
} // namespace knng

extern "C" {

static knng_status knng_expand_impl(const knng_set *S, const knng_graph *G, const knng_set *raw,
                                    int32_t k, knng_metric metric, const knng_opts *opts,
                                    knng_graph *out, void *workspace, size_t workspace_bytes,
                                    void *stream, knng_stats *stats)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(S, "S", true)) ||
        (s = check_set(raw, "raw")) || (s = check_opts(opts, k)))
        return s;
    if (S->n > 0 && S->d != raw->d)
        return fail(KNNG_EINVAL, "S->d = %d differs from raw->d = %d", S->d, raw->d);
    const int64_t nb = S->n, nr = raw->n, n = nb + nr;
    if (n >= (1ll << 30) - 64)
        return fail(KNNG_EINVAL, "S->n + raw->n = %lld rows out of range", (long long)n);
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n-1)]", k);
    const int k1 = keep_count(opts, k);
    if (nb > 0 && (s = check_graph_in(G, nb, "G", k1)))
        return s;
    if ((s = check_out(out, n, k)))
        return s;
    const bool bf16 = uses_bf16(metric, opts);
    const int kin = nb > 0 ? G->k : 0;
    const size_t need = knng_expand_workspace_size(nb, nr, raw->d, k, kin, metric, opts);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    if (stats)
        memset(stats, 0, sizeof *stats);
    Carve c(workspace);
    Layout w;
    carve_merge(c, w, n, nb, raw->d, k, kin, opts->sample, metric, bf16);
    Prof prof{(opts->flags & KNNG_FLAG_PROFILE) != 0, st};
    Rows R;
    prof.begin(PH_PREP);
    s = prepare(S, nb > 0 ? G : nullptr, raw, nullptr, metric, bf16, w, nb, n, st, R);
    prof.end();
    if (s != KNNG_OK)
        return s;
    return run_merge(R, w, metric, bf16, opts, n, nb, k, nb > 0 ? k1 : 0, 1, nb, out, st, stats,
                     prof);
}

knng_status knng_expand(const knng_set *S, const knng_graph *G, const knng_set *raw, int32_t k,
                        knng_metric metric, const knng_opts *opts, knng_graph *out,
                        void *workspace, size_t workspace_bytes, void *stream,
                        knng_stats *stats)
{
    try {
        return knng_expand_impl(S, G, raw, k, metric, opts, out, workspace, workspace_bytes, stream,
                                stats);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

// ---------------------------------------------------------------- merge tree
namespace {

struct Seg {
    int64_t a, c;  // rows [a, c) of X
    int32_t *ids;  // local ids (row - a)
    float *dist;
    int32_t kk;
};

// two ping-pong levels of ids and distances, then the merge workspace at the
// next 256-byte boundary (the same carve sizes and places them)
struct TreeBufs {
    int32_t *ids[2];
    float *dist[2];
};

void carve_tree(Carve &c, TreeBufs &t, int64_t n, int k)
{
    t.ids[0] = c.take<int32_t>((size_t)n * k);
    t.ids[1] = c.take<int32_t>((size_t)n * k);
    t.dist[0] = c.take<float>((size_t)n * k);
    t.dist[1] = c.take<float>((size_t)n * k);
    c.off = (c.off + 255) / 256 * 256;
}

// Workspace slices of the merges of every level (the merges of a level run
// at the same time, each in a 256-byte aligned slice of its own); the tree
// needs the largest per-level sum.
std::vector<std::vector<size_t>> tree_plan(const int64_t *starts, int nb, int d, int k,
                                           int kin_max, knng_metric m, const knng_opts *o)
{
    std::vector<int64_t> b(starts, starts + nb + 1);
    std::vector<std::vector<size_t>> plan;
    int kin = kin_max;
    while (b.size() > 2) {
        std::vector<int64_t> nxt;
        std::vector<size_t> lvl;
        nxt.push_back(b[0]);
        for (size_t i = 0; i + 2 < b.size(); i += 2) {
            const size_t w = knng_merge_workspace_size(b[i + 1] - b[i], b[i + 2] - b[i + 1], d, k,
                                                       kin, kin, m, o);
            lvl.push_back((w + 255) / 256 * 256);
            nxt.push_back(b[i + 2]);
        }
        if ((b.size() - 1) % 2 == 1)
            nxt.push_back(b.back());
        b.swap(nxt);
        plan.push_back(lvl);
        kin = kin > k ? kin : k;
    }
    return plan;
}

size_t tree_merge_ws(const int64_t *starts, int nb, int d, int k, int kin_max, knng_metric m,
                     const knng_opts *o)
{
    size_t best = 0;
    for (const auto &lvl : tree_plan(starts, nb, d, k, kin_max, m, o)) {
        size_t sum = 0;
        for (size_t w : lvl)
            sum += w;
        best = sum > best ? sum : best;
    }
    return best;
}

} // namespace

static size_t knng_merge_tree_workspace_size_impl(int64_t n, int32_t d, int32_t nblocks,
                                                  const int64_t *starts, int32_t k, int32_t kin_max,
                                                  knng_metric metric, const knng_opts *opts)
{
    if (!starts || nblocks < 2 || n < 2 || d < 1 || k < 1 || !opts || starts[nblocks] != n)
        return 0;
    Carve c(nullptr);
    TreeBufs t;
    carve_tree(c, t, n, k);
    const int kin = kin_max > k ? kin_max : k;
    return c.off + 256 + tree_merge_ws(starts, nblocks, d, k, kin, metric, opts);
}

extern "C" size_t knng_merge_tree_workspace_size(int64_t n, int32_t d, int32_t nblocks,
                                                 const int64_t *starts, int32_t k,
                                                 int32_t kin_max, knng_metric metric,
                                                 const knng_opts *opts)
{
    try {
        return knng_merge_tree_workspace_size_impl(n, d, nblocks, starts, k, kin_max, metric, opts);
    } catch (const std::bad_alloc &) {
        return 0;
    } catch (...) {
        return 0;
    }
}

static knng_status knng_merge_tree_impl(const knng_set *X, const int64_t *starts,
                                        const knng_graph *G, int32_t nblocks, int32_t k,
                                        knng_metric metric, const knng_opts *opts, knng_graph *out,
                                        void *workspace, size_t workspace_bytes, void *stream,
                                        knng_stats *stats)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(X, "X")) || (s = check_opts(opts, k)))
        return s;
    if (!starts || !G || nblocks < 2)
        return fail(KNNG_EINVAL, "merge tree needs at least 2 blocks");
    const int64_t n = X->n;
    if (starts[0] != 0 || starts[nblocks] != n)
        return fail(KNNG_EINVAL, "block starts must run from 0 to X->n");
    int kin_max = 0;
    for (int b = 0; b < nblocks; b++) {
        if (starts[b + 1] - starts[b] < 2)
            return fail(KNNG_EINVAL, "block %d has fewer than 2 rows", b);
        kin_max = G[b].k > kin_max ? G[b].k : kin_max;
    }
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range", k);
    if ((s = check_out(out, n, k)))
        return s;
    const size_t need =
        knng_merge_tree_workspace_size(n, X->d, nblocks, starts, k, kin_max, metric, opts);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    TreeBufs t;
    carve_tree(c, t, n, k);
    int32_t *const *ids = t.ids;
    float *const *dist = t.dist;
    uint8_t *mws = static_cast<uint8_t *>(workspace) + c.off;
    const int kin_plan = kin_max > k ? kin_max : k;
    const auto plan = tree_plan(starts, nblocks, X->d, k, kin_plan, metric, opts);
    knng_stats total;
    memset(&total, 0, sizeof total);
    std::vector<Seg> segs;
    for (int b = 0; b < nblocks; b++)
        segs.push_back({starts[b], starts[b + 1], G[b].ids, G[b].dist, G[b].k});
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    HIP_TRY(hipStreamSynchronize(st));  // inputs written on the caller's stream are complete
    // one stream per merge of a level (the first level has the most)
    std::vector<hipStream_t> streams(plan.empty() ? 0 : plan[0].size(), nullptr);
    auto destroy = [&]() {
        for (hipStream_t x : streams)
            if (x)
                (void)hipStreamDestroy(x);
    };
    for (hipStream_t &x : streams)
        if (hipStreamCreateWithFlags(&x, hipStreamNonBlocking) != hipSuccess) {
            destroy();
            return fail(KNNG_EDEVICE, "stream creation failed");
        }
    int level = 0;
    while (segs.size() > 1) {
        const bool last = segs.size() == 2;
        const auto t_level = std::chrono::steady_clock::now();
        int32_t *li = last ? out->ids : ids[level & 1];
        float *ld = last ? out->dist : dist[level & 1];
        const size_t npairs = segs.size() / 2;
        std::vector<knng_stats> one(npairs);
        std::vector<knng_status> rc(npairs, KNNG_OK);
        std::vector<std::string> msg(npairs);
        std::vector<std::thread> workers;
        size_t off = 0;
        // the merges of a level are independent: each runs in a host thread
        // of its own, on its own stream and workspace slice
        for (size_t i = 0; i < npairs; i++) {
            const Seg p = segs[2 * i], q = segs[2 * i + 1];
            uint8_t *ws = mws + off;
            const size_t ws_bytes = plan[level][i];
            off += ws_bytes;
            hipStream_t sx = streams[i];
            auto work = [=, &one, &rc, &msg]() {
                if (hipSetDevice(device) != hipSuccess) {
                    rc[i] = KNNG_EDEVICE;
                    msg[i] = "hipSetDevice failed in a merge-tree worker";
                    return;
                }
                knng_set s1{p.c - p.a, X->d, X->x + p.a * X->d};
                knng_set s2{q.c - q.a, X->d, X->x + q.a * X->d};
                knng_graph g1{p.c - p.a, p.kk, p.ids, p.dist};
                knng_graph g2{q.c - q.a, q.kk, q.ids, q.dist};
                knng_graph o{q.c - p.a, k, li + p.a * k, ld + p.a * k};
                memset(&one[i], 0, sizeof one[i]);
                rc[i] = knng_merge(&s1, &g1, &s2, &g2, k, metric, opts, &o, ws, ws_bytes, sx,
                                   &one[i]);
                if (rc[i] != KNNG_OK)
                    msg[i] = g_err;
            };
            // a thread that cannot be started: the merge runs here instead
            try {
                workers.emplace_back(work);
            } catch (...) {
                work();
            }
        }
        for (std::thread &w : workers)
            w.join();
        for (size_t i = 0; i < npairs; i++) {
            if (rc[i] != KNNG_OK) {
                destroy();
                return fail(rc[i], "merge %zu of level %d: %s", i, level, msg[i].c_str());
            }
        }
        std::vector<Seg> nxt;
        for (size_t i = 0; i < npairs; i++) {
            const Seg &p = segs[2 * i], &q = segs[2 * i + 1];
            const knng_stats &o1 = one[i];
            total.rounds += o1.rounds;
            total.evals += o1.evals;
            total.rescored += o1.rescored;
            total.insert_attempts += o1.insert_attempts;
            total.screen_violations += o1.screen_violations;
            total.max_group = o1.max_group > total.max_group ? o1.max_group : total.max_group;
            total.ms_prep += o1.ms_prep;
            total.ms_init += o1.ms_init;
            total.ms_sample += o1.ms_sample;
            total.ms_reverse += o1.ms_reverse;
            total.ms_join += o1.ms_join;
            total.ms_final += o1.ms_final;
            total.join_launches += o1.join_launches;
            if (level < KNNG_STATS_ROUNDS) {
                total.updates[level] += o1.evals;  // distance evaluations per level
                total.pairs[level] += o1.rounds;   // rounds per level
            }
            nxt.push_back({p.a, q.c, li + p.a * k, ld + p.a * k, k});
        }
        if (segs.size() % 2 == 1) {
            // an odd last block moves up unchanged (copied: the next level
            // writes into the buffer it lives in)
            const Seg &r = segs.back();
            const int64_t rows = r.c - r.a;
            if (r.kk < k || !r.dist) {
                destroy();
                return fail(KNNG_EINVAL, "a block carried up unmerged needs k_in >= k and "
                                         "distances");
            }
            if (hipMemcpy2DAsync(li + r.a * k, (size_t)k * 4, r.ids, (size_t)r.kk * 4,
                                 (size_t)k * 4, (size_t)rows, hipMemcpyDeviceToDevice,
                                 st) != hipSuccess ||
                hipMemcpy2DAsync(ld + r.a * k, (size_t)k * 4, r.dist, (size_t)r.kk * 4,
                                 (size_t)k * 4, (size_t)rows, hipMemcpyDeviceToDevice,
                                 st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                destroy();
                return fail(KNNG_EDEVICE, "copy of an unmerged block failed");
            }
            nxt.push_back({r.a, r.c, li + r.a * k, ld + r.a * k, k});
        }
        if (level < KNNG_STATS_ROUNDS)
            total.gathered[level] = (int64_t)std::chrono::duration<double, std::micro>(
                                        std::chrono::steady_clock::now() - t_level)
                                        .count();
        segs.swap(nxt);
        level++;
    }
    destroy();
    if (stats)
        *stats = total;
    return ok();
}

extern "C" knng_status knng_merge_tree(const knng_set *X, const int64_t *starts,
                                       const knng_graph *G, int32_t nblocks, int32_t k,
                                       knng_metric metric, const knng_opts *opts,
                                       knng_graph *out, void *workspace, size_t workspace_bytes,
                                       void *stream, knng_stats *stats)
{
    try {
        return knng_merge_tree_impl(X, starts, G, nblocks, k, metric, opts, out, workspace,
                                    workspace_bytes, stream, stats);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

// ---------------------------------------------------------------- H-Merge
namespace {

// Layers of H-Merge (Section 3.3): NN-Descent on the first n_top positions,
// then J-Merges that double the rows until all n are in.  Lists hold k/2
// entries on the layers above the bottom one and k on the bottom layer, never
// more than the layer's rows - 1.
struct HPlan {
    std::vector<int64_t> rows;
    std::vector<int> kk;
};

HPlan hmerge_plan(int64_t n, int64_t n_top, int k)
{
    HPlan p;
    const int kh = k / 2;
    auto list = [&](int64_t rows) {
        const int v = rows == n ? k : kh;
        return (int64_t)v > rows - 1 ? (int)(rows - 1) : v;
    };
    int64_t m = n_top < n ? n_top : n;
    p.rows.push_back(m);
    p.kk.push_back(list(m));
    while (m < n) {
        m = 2 * m < n ? 2 * m : n;
        p.rows.push_back(m);
        p.kk.push_back(list(m));
    }
    return p;
}

// bits of each Feistel half: 2 * half >= bits of n - 1
int perm_half(int64_t n)
{
    int b = 2;
    while (b < 62 && ((int64_t)1 << b) < n)
        b++;
    return (b + 1) / 2;
}

struct HBufs {
    int32_t *perm, *ids[2];
    float *xp, *dist[2];
};

void carve_hmerge(Carve &c, HBufs &h, int64_t n, int d, int k)
{
    h.perm = c.take<int32_t>(n);
    h.xp = c.take<float>((size_t)n * d);
    for (int i = 0; i < 2; i++) {
        h.ids[i] = c.take<int32_t>((size_t)n * k);
        h.dist[i] = c.take<float>((size_t)n * k);
    }
    c.off = (c.off + 255) / 256 * 256;
}

knng_opts layer_opts(const knng_opts *o, int level)
{
    knng_opts lo = *o;
    lo.seed = sm64_host(o->seed ^ sm64_host((uint64_t)level));
    return lo;
}

} // namespace

static size_t knng_hmerge_workspace_size_impl(int64_t n, int32_t d, int32_t k, int64_t n_top,
                                              knng_metric metric, const knng_opts *opts)
{
    if (n < 2 || d < 1 || k < 1 || n_top < 2 || !opts)
        return 0;
    Carve c(nullptr);
    HBufs h;
    carve_hmerge(c, h, n, d, k);
    const HPlan p = hmerge_plan(n, n_top, k);
    size_t best = 0;
    for (size_t l = 0; l < p.rows.size(); l++) {
        const int64_t nb = l ? p.rows[l - 1] : 0, nr = p.rows[l] - nb;
        const knng_opts lo = layer_opts(opts, (int)l);
        const size_t w =
            knng_expand_workspace_size(nb, nr, d, p.kk[l], l ? p.kk[l - 1] : 0, metric, &lo);
        best = w > best ? w : best;
    }
    return c.off + best + 256;
}

extern "C" size_t knng_hmerge_workspace_size(int64_t n, int32_t d, int32_t k, int64_t n_top,
                                            knng_metric metric, const knng_opts *opts)
{
    try {
        return knng_hmerge_workspace_size_impl(n, d, k, n_top, metric, opts);
    } catch (const std::bad_alloc &) {
        return 0;
    } catch (...) {
        return 0;
    }
}

// Optional outputs of the hierarchy (knng_hmerge_hierarchy): the random
// order, the permuted rows and every layer's graph over positions.
struct HOut {
    int32_t *perm = nullptr;
    float *xp = nullptr;
    knng_graph *layers = nullptr;
    int32_t nlayers = 0;
};

static knng_status knng_hmerge_impl(const knng_set *X, int32_t k, int64_t n_top, knng_metric metric,
                                    const knng_opts *opts, knng_graph *out, void *workspace,
                                    size_t workspace_bytes, void *stream, knng_stats *stats,
                                    const HOut *ho = nullptr)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(X, "X")) || (s = check_opts(opts, k)))
        return s;
    const int64_t n = X->n;
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n-1)]", k);
    if (n_top < 2)
        return fail(KNNG_EINVAL, "n_top = %lld: the top layer needs at least 2 rows",
                    (long long)n_top);
    const HPlan p = hmerge_plan(n, n_top, k);
    for (size_t l = 0; l < p.rows.size(); l++) {
        if (p.kk[l] < 1)
            return fail(KNNG_EINVAL, "layer %zu would hold empty lists (k = %d)", l, k);
        if (l && keep_count(opts, p.kk[l]) > p.kk[l - 1])
            return fail(KNNG_EINVAL, "keep_ratio keeps %d entries of a layer with %d-entry lists",
                        keep_count(opts, p.kk[l]), p.kk[l - 1]);
    }
    if (ho) {
        if ((int)p.rows.size() != ho->nlayers || !ho->layers)
            return fail(KNNG_EINVAL, "the hierarchy has %zu layers, %d given", p.rows.size(),
                        ho->nlayers);
        for (size_t l = 0; l < p.rows.size(); l++) {
            const knng_graph &g = ho->layers[l];
            if (g.n != p.rows[l] || g.k != p.kk[l] || !is_device_ptr(g.ids) ||
                !is_device_ptr(g.dist))
                return fail(KNNG_EINVAL, "layer %zu must be %lld x %d device arrays", l,
                            (long long)p.rows[l], p.kk[l]);
        }
        if ((ho->perm && !is_device_ptr(ho->perm)) || (ho->xp && !is_device_ptr(ho->xp)))
            return fail(KNNG_EINVAL, "perm / xp must be device memory");
    }
    if ((out || !ho) && (s = check_out(out, n, k)))
        return s;
    const size_t need = knng_hmerge_workspace_size(n, X->d, k, n_top, metric, opts);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    HBufs h;
    carve_hmerge(c, h, n, X->d, k);
    uint8_t *mws = static_cast<uint8_t *>(workspace) + c.off;
    const size_t mws_bytes = workspace_bytes - c.off;
    // random order of the rows: the blocks joined in are random subsets
    HIP_TRY(launch_permute_rows(X->x, n, X->d, opts->seed, perm_half(n), h.perm, h.xp, st));
    knng_stats total;
    memset(&total, 0, sizeof total);
    int cur = 0;
    for (size_t l = 0; l < p.rows.size(); l++) {
        const auto t_level = std::chrono::steady_clock::now();
        const int64_t nb = l ? p.rows[l - 1] : 0, nr = p.rows[l] - nb;
        const knng_opts lo = layer_opts(opts, (int)l);
        knng_set base{nb, X->d, nb ? h.xp : nullptr};
        knng_graph g{nb, l ? p.kk[l - 1] : 0, l ? h.ids[cur] : nullptr,
                     l ? h.dist[cur] : nullptr};
        knng_set raw{nr, X->d, h.xp + nb * X->d};
        const int nxt = l ? 1 - cur : cur;
        knng_graph o{p.rows[l], p.kk[l], h.ids[nxt], h.dist[nxt]};
        knng_stats one;
        s = knng_expand(&base, &g, &raw, p.kk[l], metric, &lo, &o, mws, mws_bytes, stream, &one);
        if (s != KNNG_OK)
            return s;
        if (ho) {
            const size_t cells = (size_t)p.rows[l] * p.kk[l];
            HIP_TRY(hipMemcpyAsync(ho->layers[l].ids, o.ids, cells * sizeof(int32_t),
                                   hipMemcpyDeviceToDevice, st));
            HIP_TRY(hipMemcpyAsync(ho->layers[l].dist, o.dist, cells * sizeof(float),
                                   hipMemcpyDeviceToDevice, st));
        }
        cur = nxt;
        total.rounds += one.rounds;
        total.evals += one.evals;
        total.rescored += one.rescored;
        total.insert_attempts += one.insert_attempts;
        total.screen_violations += one.screen_violations;
        total.max_group = one.max_group > total.max_group ? one.max_group : total.max_group;
        total.ms_prep += one.ms_prep;
        total.ms_init += one.ms_init;
        total.ms_sample += one.ms_sample;
        total.ms_reverse += one.ms_reverse;
        total.ms_join += one.ms_join;
        total.ms_final += one.ms_final;
        total.join_launches += one.join_launches;
        if (l < KNNG_STATS_ROUNDS) {
            total.updates[l] = one.evals;  // distance evaluations of the layer
            total.pairs[l] = one.rounds;   // its rounds
            total.gathered[l] = (int64_t)std::chrono::duration<double, std::micro>(
                                    std::chrono::steady_clock::now() - t_level)
                                    .count();
        }
    }
    // back to the caller's row numbering
    if (out)
        HIP_TRY(launch_unpermute_graph(h.ids[cur], h.dist[cur], n, k, h.perm, out->ids,
                                       out->dist, st));
    if (ho && ho->perm)
        HIP_TRY(hipMemcpyAsync(ho->perm, h.perm, (size_t)n * sizeof(int32_t),
                               hipMemcpyDeviceToDevice, st));
    if (ho && ho->xp)
        HIP_TRY(hipMemcpyAsync(ho->xp, h.xp, (size_t)n * X->d * sizeof(float),
                               hipMemcpyDeviceToDevice, st));
    if (ho)
        HIP_TRY(hipStreamSynchronize(st));
    if (stats)
        *stats = total;
    return ok();
}

extern "C" int32_t knng_hierarchy_shape(int64_t n, int64_t n_top, int32_t k, int64_t *rows,
                                        int32_t *lists, int32_t cap)
{
    if (n < 2 || n_top < 2 || k < 1)
        return 0;
    try {
        const HPlan p = hmerge_plan(n, n_top, k);
        for (size_t l = 0; l < p.rows.size() && (int32_t)l < cap; l++) {
            if (rows)
                rows[l] = p.rows[l];
            if (lists)
                lists[l] = p.kk[l];
        }
        return (int32_t)p.rows.size();
    } catch (...) {
        return 0;
    }
}

extern "C" knng_status knng_hmerge_hierarchy(const knng_set *X, int32_t k, int64_t n_top,
                                             knng_metric metric, const knng_opts *opts,
                                             int32_t *perm, float *xp, knng_graph *layers,
                                             int32_t nlayers, void *workspace,
                                             size_t workspace_bytes, void *stream,
                                             knng_stats *stats)
{
    try {
        HOut ho;
        ho.perm = perm;
        ho.xp = xp;
        ho.layers = layers;
        ho.nlayers = nlayers;
        return knng_hmerge_impl(X, k, n_top, metric, opts, nullptr, workspace, workspace_bytes,
                                stream, stats, &ho);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

extern "C" knng_status knng_hmerge(const knng_set *X, int32_t k, int64_t n_top,
                                   knng_metric metric, const knng_opts *opts, knng_graph *out,
                                   void *workspace, size_t workspace_bytes, void *stream,
                                   knng_stats *stats)
{
    try {
        return knng_hmerge_impl(X, k, n_top, metric, opts, out, workspace, workspace_bytes, stream,
                                stats);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

size_t knng_bruteforce_workspace_size(int64_t n1, int64_t n2, int32_t d, int32_t k,
                                      int32_t kin1, int32_t kin2, knng_metric metric)
{
    if (n1 < 1 || n2 < 1 || d < 1 || k < 1)
        return 0;
    Carve c(nullptr);
    const int64_t n = n1 + n2;
    c.take<uint64_t>(C_WORDS);
    c.take<float>((size_t)n * pad4(d));
    if (metric == KNNG_COSINE)
        c.take<float>(n);
    c.take<uint64_t>((size_t)n * (kin1 > kin2 ? kin1 : kin2));
    return c.off + 256;
}

static knng_status knng_merge_bruteforce_impl(const knng_set *S1, const knng_graph *G1,
                                              const knng_set *S2, const knng_graph *G2, int32_t k,
                                              knng_metric metric, knng_graph *out, void *workspace,
                                              size_t workspace_bytes, void *stream)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(S1, "S1")) || (s = check_set(S2, "S2")))
        return s;
    if (S1->d != S2->d)
        return fail(KNNG_EINVAL, "S1->d = %d differs from S2->d = %d", S1->d, S2->d);
    const int64_t n1 = S1->n, n2 = S2->n, n = n1 + n2;
    // a list entry holds a row id in 30 bits
    if (n >= (1ll << 30) - 64)
        return fail(KNNG_EINVAL, "n1 + n2 = %lld rows out of range", (long long)n);
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n1+n2-1)]", k);
    if ((s = check_graph_in(G1, n1, "G1", 0)) || (s = check_graph_in(G2, n2, "G2", 0)) ||
        (s = check_out(out, n, k)))
        return s;
    const size_t need = knng_bruteforce_workspace_size(n1, n2, S1->d, k, G1->k, G2->k, metric);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    Layout w{};
    w.dp = pad4(S1->d);
    w.gstride = G1->k > G2->k ? G1->k : G2->k;
    w.ctr = c.take<uint64_t>(C_WORDS);
    w.x = c.take<float>((size_t)n * w.dp);
    w.norm = metric == KNNG_COSINE ? c.take<float>(n) : nullptr;
    w.gin = c.take<uint64_t>((size_t)n * w.gstride);
    Rows R;
    s = prepare(S1, G1, S2, G2, metric, false, w, n1, n, st, R);
    if (s != KNNG_OK)
        return s;
    HIP_TRY(launch_brute(R, metric, 0, n1, n1, n, w.gin, w.gstride, k, 0, 0, 0, out->ids,
                         out->dist, st));
    HIP_TRY(launch_brute(R, metric, n1, n, 0, n1, w.gin + n1 * w.gstride, w.gstride, k, 0, 0, 0,
                         out->ids, out->dist, st));
    HIP_TRY(hipStreamSynchronize(st));
    return ok();
}

knng_status knng_merge_bruteforce(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                                  const knng_graph *G2, int32_t k, knng_metric metric,
                                  knng_graph *out, void *workspace, size_t workspace_bytes,
                                  void *stream)
{
    try {
        return knng_merge_bruteforce_impl(S1, G1, S2, G2, k, metric, out, workspace,
                                          workspace_bytes, stream);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

size_t knng_exact_graph_workspace_size(int64_t n, int32_t d, int32_t k, knng_metric metric)
{
    if (n < 2 || d < 1 || k < 1)
        return 0;
    Carve c(nullptr);
    c.take<uint64_t>(C_WORDS);
    c.take<float>((size_t)n * pad4(d));
    if (metric == KNNG_COSINE)
        c.take<float>(n);
    return c.off + 256;
}

static knng_status knng_exact_graph_impl(const knng_set *S, int32_t k, knng_metric metric,
                                         knng_graph *out, void *workspace, size_t workspace_bytes,
                                         void *stream)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(S, "S")))
        return s;
    const int64_t n = S->n;
    if (k < 1 || k > MAX_K || k > n - 1)
        return fail(KNNG_EINVAL, "k = %d out of range [1, min(64, n-1)]", k);
    if ((s = check_out(out, n, k)))
        return s;
    const size_t need = knng_exact_graph_workspace_size(n, S->d, k, metric);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    Layout w{};
    w.dp = pad4(S->d);
    w.ctr = c.take<uint64_t>(C_WORDS);
    w.x = c.take<float>((size_t)n * w.dp);
    w.norm = metric == KNNG_COSINE ? c.take<float>(n) : nullptr;
    knng_set empty{0, S->d, nullptr};
    Rows R;
    s = prepare(&empty, nullptr, S, nullptr, metric, false, w, 0, n, st, R);
    if (s != KNNG_OK)
        return s;
    HIP_TRY(launch_brute(R, metric, 0, n, 0, n, nullptr, 0, k, 1, 0, 0, out->ids, out->dist,
                         st));
    HIP_TRY(hipStreamSynchronize(st));
    return ok();
}

knng_status knng_exact_graph(const knng_set *S, int32_t k, knng_metric metric, knng_graph *out,
                             void *workspace, size_t workspace_bytes, void *stream)
{
    try {
        return knng_exact_graph_impl(S, k, metric, out, workspace, workspace_bytes, stream);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

} // extern "C"
