// knng_host.h -- host-side helpers shared by the C ABI entry points:
// error reporting, argument checks, the workspace carve of a merge, counter
// read-back, phase timing, and the two halves of a merge call (input
// preparation and the repeat loop of Algorithms 1 and 2 with Merge and Sort).
#pragma once

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/knng_merge.h"
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {
namespace host {

inline thread_local std::string g_err;

inline knng_status fail(knng_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

inline knng_status ok()
{
    g_err.clear();
    return KNNG_OK;
}

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(KNNG_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

inline int pad4(int d) { return (d + 3) / 4 * 4; }

// bump allocator over the caller's workspace; with base == nullptr it only
// measures
struct Carve {
    uint8_t *base;
    size_t off = 0;
    explicit Carve(void *b) : base((uint8_t *)b) {}
    template <class T> T *take(size_t count)
    {
        off = (off + 255) / 256 * 256;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// A slot's repeat loop captured once as a launch graph of one round (graph
// mode, see DevRound); replayed for every round of every request.
struct RoundGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t rows_cap = 0;   // most rows a merge of the slot has (grid sizes)
};

struct Layout {
    uint64_t *ctr;
    float *x, *norm;
    float2 *se;
    uint16_t *xb;
    uint64_t *gin, *L, *worst, *rnew, *rold;
    int32_t *new_f, *old_f, *cnt_f, *dtag, *atag, *rfill;
    int dp, db, gstride;
    // u64 words from one row's `worst` word to the next: 2 when each is
    // followed by the row's `se` pair (merges on the BF16 path), else 1
    int ws = 1;
    // reverse index of the base lists (server only; see RoundArgs)
    const int64_t *rev_off = nullptr;
    const int32_t *rev_src = nullptr;
    int64_t rev_m = 0;
    // tag of the merge's round 0, and whether the state already holds the
    // initial lists of unselected base rows (server slots; see RoundArgs)
    int32_t tag0 = 0;
    bool incremental = false;
    int32_t *alist = nullptr;  // n words: the round's active rows (list mode)
    // graph mode (server slots): the device round state and the slot's graph
    DevRound *dev = nullptr;
    RoundGraph *graph = nullptr;
};

// SplitMix64 (one step of the published generator), for seeds derived on the host
inline uint64_t sm64_host(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline bool uses_bf16(knng_metric m, const knng_opts *o)
{
    return o && o->precision == KNNG_BF16_RESCORE && m != KNNG_L1;
}

// one layout for S-Merge and J-Merge: n rows, input lists on `n_list` rows
inline void carve_merge(Carve &c, Layout &w, int64_t n, int64_t n_list, int d, int k,
                        int gstride, int s, knng_metric m, bool bf16)
{
    w.dp = pad4(d);
    w.db = (d + 31) / 32 * 32;
    w.gstride = gstride;
    w.ctr = c.take<uint64_t>(C_WORDS);
    w.x = c.take<float>((size_t)n * w.dp);
    w.norm = m == KNNG_COSINE ? c.take<float>(n) : nullptr;
    w.xb = bf16 ? c.take<uint16_t>((size_t)n * w.db) : nullptr;
    w.gin = c.take<uint64_t>((size_t)(n_list > 0 ? n_list : 1) * (gstride > 0 ? gstride : 1));
    w.L = c.take<uint64_t>((size_t)n * k);
    // BF16 path: a row's bound and its (norm, error bound) pair share one
    // 16-byte record, which forming a neighbourhood reads per member
    w.ws = bf16 ? 2 : 1;
    w.worst = c.take<uint64_t>((size_t)n * w.ws);
    w.se = bf16 ? reinterpret_cast<float2 *>(w.worst + 1) : nullptr;
    w.new_f = c.take<int32_t>((size_t)n * s);
    w.old_f = c.take<int32_t>((size_t)n * k);
    w.cnt_f = c.take<int32_t>((size_t)n * 2);
    w.rnew = c.take<uint64_t>((size_t)n * s);
    w.rold = c.take<uint64_t>((size_t)n * s);
    w.dtag = c.take<int32_t>((size_t)n);
    w.atag = c.take<int32_t>((size_t)n);
    w.rfill = c.take<int32_t>((size_t)n * 2);
}

inline bool is_device_ptr(const void *p)
{
    if (!p)
        return false;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

inline knng_status check_set(const knng_set *S, const char *name, bool allow_empty = false)
{
    if (!S)
        return fail(KNNG_EINVAL, "%s is NULL", name);
    if (S->n < (allow_empty ? 0 : 1) || S->n >= (1ll << 30) - 64)
        return fail(KNNG_EINVAL, "%s->n = %lld out of range", name, (long long)S->n);
    if (S->d < 1 || S->d > 65536)
        return fail(KNNG_EINVAL, "%s->d = %d out of range", name, S->d);
    if (S->n > 0 && !is_device_ptr(S->x))
        return fail(KNNG_EINVAL, "%s->x is not device memory", name);
    return KNNG_OK;
}

inline knng_status check_graph_in(const knng_graph *G, int64_t n, const char *name, int kmin)
{
    if (!G)
        return fail(KNNG_EINVAL, "%s is NULL", name);
    if (G->n != n)
        return fail(KNNG_EINVAL, "%s->n = %lld, expected %lld", name, (long long)G->n,
                    (long long)n);
    if (G->k < kmin || G->k > MAX_K || G->k > n - 1)
        return fail(KNNG_EINVAL, "%s->k = %d out of range [%d, min(64, n-1)]", name, G->k, kmin);
    if (G->k > 0 && !is_device_ptr(G->ids))
        return fail(KNNG_EINVAL, "%s->ids is not device memory", name);
    if (G->dist && !is_device_ptr(G->dist))
        return fail(KNNG_EINVAL, "%s->dist is not device memory", name);
    return KNNG_OK;
}

inline knng_status check_out(const knng_graph *out, int64_t n, int k)
{
    if (!out)
        return fail(KNNG_EINVAL, "out is NULL");
    if (out->n != n || out->k != k)
        return fail(KNNG_EINVAL, "out is %lld x %d, expected %lld x %d", (long long)out->n,
                    out->k, (long long)n, k);
    if (!is_device_ptr(out->ids) || !is_device_ptr(out->dist))
        return fail(KNNG_EINVAL, "out->ids / out->dist must be device memory");
    return KNNG_OK;
}

inline knng_status check_opts(const knng_opts *o, int k)
{
    if (!o)
        return fail(KNNG_EINVAL, "opts is NULL");
    if (!(o->keep_ratio >= 0.0f && o->keep_ratio <= 1.0f))
        return fail(KNNG_EINVAL, "keep_ratio %g not in [0, 1]", (double)o->keep_ratio);
    if (o->sample < 1 || o->sample > MAX_S)
        return fail(KNNG_EINVAL, "sample %d not in [1, %d]", o->sample, MAX_S);
    if (!(o->delta >= 0.0f))
        return fail(KNNG_EINVAL, "delta must be >= 0");
    if (o->max_rounds < 0)
        return fail(KNNG_EINVAL, "max_rounds must be >= 0");
    if (o->precision != KNNG_FP32 && o->precision != KNNG_BF16_RESCORE)
        return fail(KNNG_EINVAL, "unknown precision %d", o->precision);
    if (3 * o->sample + k > MAX_G)
        return fail(KNNG_EINVAL, "3*sample + k = %d exceeds %d", 3 * o->sample + k, MAX_G);
    if (o->flags & ~(KNNG_FLAG_PROFILE | KNNG_FLAG_BALANCED_APPEND))
        return fail(KNNG_EINVAL, "unknown flags 0x%x", o->flags);
    return KNNG_OK;
}

inline knng_status check_metric(knng_metric m)
{
    if (m != KNNG_L2 && m != KNNG_COSINE && m != KNNG_L1)
        return fail(KNNG_EINVAL, "unknown metric %d", (int)m);
    return KNNG_OK;
}

inline const char *err_text(uint64_t bits)
{
    if (bits & ERR_NONFINITE)
        return "input rows hold a non-finite value";
    if (bits & ERR_ZERO_NORM)
        return "cosine metric: an input row has zero norm";
    if (bits & ERR_ID_RANGE)
        return "input graph id out of range";
    if (bits & ERR_SELF)
        return "input graph row lists itself";
    if (bits & ERR_DUP)
        return "input graph row holds a duplicate id";
    if (bits & ERR_UNSORTED)
        return "input graph row not sorted by (distance, id)";
    if (bits & ERR_BAD_DIST)
        return "input graph distance negative or not finite";
    if (bits & ERR_SPIN)
        return "internal: list insert exceeded its retry budget";
    if (bits & ERR_ROW_REVERSE)
        return "internal: a sampled edge names a row out of range";
    if (bits & ERR_ROW_GROUP)
        return "internal: a neighbourhood member is out of range";
    if (bits & ERR_ROW_SAMPLE)
        return "internal: a list entry names a row out of range";
    if (bits & ERR_ROW_COMMIT)
        return "internal: a committed entry names a row out of range";
    if (bits & ERR_GROUP)
        return "internal: neighbourhood exceeded the kernel bound";
    return "unknown device error";
}

// reads the counter block; returns the error bits
inline knng_status read_ctr(const uint64_t *dctr, uint64_t *h, hipStream_t st)
{
    HIP_TRY(hipMemcpyAsync(h, dctr, sizeof(uint64_t) * C_WORDS, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return KNNG_OK;
}

// phase timing with HIP events (KNNG_FLAG_PROFILE)
struct Prof {
    bool on;
    hipStream_t st;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
    hipEvent_t cur = nullptr;
    int cur_phase = -1;
    void begin(int phase)
    {
        if (!on)
            return;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return;
        (void)hipEventRecord(e, st);
        cur = e;
        cur_phase = phase;
    }
    void end()
    {
        if (!on || !cur)
            return;
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return;
        (void)hipEventRecord(e, st);
        ev.push_back({cur_phase, {cur, e}});
        cur = nullptr;
    }
    void collect(knng_stats *s)
    {
        if (!on)
            return;
        (void)hipStreamSynchronize(st);
        for (auto &p : ev) {
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, p.second.first, p.second.second);
            if (s) {
                double *slot[] = {&s->ms_prep, &s->ms_init, &s->ms_sample, &s->ms_reverse,
                                  &s->ms_join, &s->ms_final};
                *slot[p.first] += ms;
                if (p.first == 4)
                    s->join_launches++;
            }
            (void)hipEventDestroy(p.second.first);
            (void)hipEventDestroy(p.second.second);
        }
        ev.clear();
    }
    ~Prof()
    {
        for (auto &p : ev) {
            (void)hipEventDestroy(p.second.first);
            (void)hipEventDestroy(p.second.second);
        }
        if (cur)
            (void)hipEventDestroy(cur);
    }
};
enum { PH_PREP = 0, PH_INIT, PH_SAMPLE, PH_REVERSE, PH_JOIN, PH_FINAL };

// Input preparation of a merge: rows of A then B packed into the layout,
// norms, validation, and the input lists as sorted keys.
knng_status prepare(const knng_set *A, const knng_graph *GA, const knng_set *B,
                    const knng_graph *GB, knng_metric metric, bool bf16, const Layout &w,
                    int64_t n1, int64_t n, hipStream_t st, Rows &R);

// Divide/Append (or Initialize), the repeat loop, and Merge and Sort into out.
knng_status run_merge(const Rows &R, const Layout &w, knng_metric metric, bool bf16,
                      const knng_opts *o, int64_t n, int64_t n1, int k, int k1, int joint,
                      int64_t rows_with_rear, knng_graph *out, hipStream_t st, knng_stats *stats,
                      Prof &prof, uint64_t *out_keys = nullptr, bool touched_only = false);

inline int keep_count(const knng_opts *o, int k) { return (int)floorf(o->keep_ratio * (float)k); }

} // namespace host
} // namespace knng
