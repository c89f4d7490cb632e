// knng_internal.h -- host-side launchers of the kernels (one per .hip file
// family) and the layout shared between the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knng {

// Device view of the rows of a merge: the two input sets concatenated into one
// padded fp32 array (rows of the first set first), plus per-row canonical norms.
// Row i of the merge is stored at row phys(i) of the arrays: rows below
// `split` in place, the others `off2` rows further on (a server keeps each
// request's rows apart from the base rows they are merged with).
struct Rows {
    const float *x;  // rows x dp fp32, zero-padded
    const float *norm;  // canonical norms (cosine) or nullptr
    const uint16_t *xb; // BF16 path: bf16 copy (round to nearest even, stride db), or nullptr
    // BF16 path, per row: the squared norm of the bf16-rounded row and an
    // upper bound of |x - bf16(x)| (read together), or nullptr
    const float2 *se;
    int se_stride = 1;  // float2 units from one row's pair to the next
    int64_t n;
    int d, dp, db;  // db: bf16 row stride, d rounded up to 32
    int64_t split = INT64_MAX, off2 = 0;
    __host__ __device__ int64_t phys(int64_t i) const { return i < split ? i : i + off2; }
};

// Round state of a merge whose repeat loop runs as a replayed launch graph
// (a server slot): the scalars that change between requests and rounds live
// here, on the device, and every kernel of the round reads them at entry
// instead of its by-value arguments; `done` makes the rest of a replay, and
// every later replay, return at once.
struct DevRound {
    int32_t round;      // t, advanced at the end of each round
    int32_t done;       // the loop has ended
    int32_t rounds;     // rounds run (valid once done)
    int32_t tag0;
    int32_t max_rounds;
    int32_t pad;
    int64_t n, n1, n_active, rev_m;
    int64_t split, off2;  // row view of the merge (Rows::phys)
    uint64_t seed;
    double delta;
};

// Parameters of one iteration of the merge loop.
struct RoundArgs {
    uint64_t *L;        // n x k list words
    uint64_t *worst;    // n: upper bound of each list's maximum word (set by the
                        // sampling step, lowered by the join's inserts), row u at
                        // worst[u * ws]
    int ws;
    int32_t *new_f;     // n x s
    int32_t *old_f;     // n x k
    int32_t *cnt_f;     // n x 2: (#new_f, #old_f)
    uint64_t *rnew;     // n x s reverse NEW reservoirs
    uint64_t *rold;     // n x s reverse OLD reservoirs
    int32_t *rfill;     // n x 2 offers made to each reservoir (NEW, OLD) this round
    // Row tags.  Round t of this merge has tag T(t) = tag0 + t (tag0 = 0 for
    // a merge on fresh state; a server slot starts each merge above every tag
    // its previous merges wrote, so old tags read as "never"):
    //   dtag[u] = T(t): u holds NEW entries to sample in round t (set by
    //            Divide/Append/Initialize for t = 0, by an insert during round
    //            t-1, or by round t-1's sampling when more than s NEW entries
    //            were left).  Before round t's join, u is sampled in round t
    //            iff dtag[u] >= T(t); dtag[u] < tag0 iff u still holds the list
    //            it started the merge with.
    //   atag[u] = T(t): u's round-t neighbourhood has a NEW member (u sampled
    //            NEW entries, or a row sampled u as a NEW entry).
    // Rows outside both sets hold only OLD entries: their neighbourhood has no
    // NEW member and joins nothing, and their whole list is their OLD sample.
    int32_t *dtag;
    int32_t *atag;
    int32_t tag0;
    // List mode (alist != nullptr): the sampling step also appends every row it
    // makes active to alist (each row once per round, counted in C_ACTIVE),
    // and the active-row kernels of the round take their n_active rows from
    // there instead of walking atag over all n rows.
    int32_t *alist;
    int64_t n_active;
    uint64_t *ctr;      // counter words
    // Reverse index of the initial lists of rows 0 .. rev_m-1 (or rev_off ==
    // nullptr): the rows u whose initial list holds v are
    // rev_src[rev_off[v] .. rev_off[v+1]).  With it, Reverse(G) reads the
    // lists only of rows with dtag >= 0; every other row still holds its
    // initial list, all OLD.
    const int64_t *rev_off;
    const int32_t *rev_src;
    int64_t rev_m;
    int64_t n;
    int64_t n1;         // first row of the second set
    int k, s;
    int joint;          // 0: S-Merge predicate, 1: J-Merge predicate
    uint64_t seed;
    int round;
    // graph mode: the round state on the device (nullptr: host-driven loop,
    // every scalar above is valid as passed)
    const DevRound *dev = nullptr;
};

// Graph mode: a kernel's by-value arguments updated from the device round
// state; false when the loop has ended (the kernel returns at once).
__device__ inline bool take_round(RoundArgs &a)
{
    if (!a.dev)
        return true;
    const DevRound *d = a.dev;
    if (d->done)
        return false;
    a.round = d->round;
    a.tag0 = d->tag0;
    a.n = d->n;
    a.n1 = d->n1;
    a.n_active = d->n_active;
    a.rev_m = d->rev_m;
    a.seed = d->seed;
    return true;
}
__device__ inline bool take_round(RoundArgs &a, Rows &R)
{
    if (!take_round(a))
        return false;
    if (a.dev) {
        R.n = a.dev->n;
        R.split = a.dev->split;
        R.off2 = a.dev->off2;
    }
    return true;
}

// ---- knng_prep.hip
// se (BF16 path, or nullptr): per row the squared norm of the bf16-rounded row
// and the bound of |x - bf16(x)|, at se[r * se_stride]
hipError_t launch_pack(const float *x1, int64_t n1, const float *x2, int64_t n2, int d, int dp,
                       float *x, int db, uint16_t *xb, float2 *se, int se_stride, uint64_t *ctr,
                       hipStream_t st);
hipError_t launch_norms(const float *x, int64_t n, int dp, float *norm, int check_zero,
                        uint64_t *ctr, hipStream_t st);
// Input graph rows [row0, row0+nrows) of the concatenated set: local ids +
// offset -> sorted keys (kin per row) in `gin`.
hipError_t launch_prep_input(const Rows &R, int metric, int64_t row0, int64_t nrows,
                             int64_t id_offset, int64_t n_local, const int32_t *ids,
                             const float *dist, int kin, int gstride, uint64_t *gin,
                             uint64_t *ctr, hipStream_t st);
// Divide + Append (rows with an input list) and Initialize (raw rows).
struct InitArgs {
    uint64_t *L;
    uint64_t *worst;    // n: maximum word of each list, row u at worst[u * ws]
    int ws;
    int32_t *dtag, *atag;
    const uint64_t *gin;
    int kin, k, k1;
    int64_t n, n1;      // n1: rows of the first set (S1 or base)
    int joint;          // J-Merge: rows >= n1 are raw
    int balanced;       // J-Merge: balanced append (base rows selected by hash)
    uint64_t seed;
    uint64_t *ctr;
    int32_t tag0;       // dtag = tag0 for rows holding NEW entries, tag0 - 1 otherwise
    int incremental;    // only rows >= n1 and selected base rows are written; the
                        // others already hold their initial state with tags < tag0
};
hipError_t launch_init(const Rows &R, int metric, const InitArgs &a, hipStream_t st);
// Rows u < m with dtag[u] >= since (changed by an earlier merge) get back their
// initial state as an unselected base row: the first min(kin, k) entries of
// gin as OLD, the list maximum in worst; their tags stay (below the next tag0).
hipError_t launch_restore(uint64_t *L, uint64_t *worst, const int32_t *dtag, const uint64_t *gin,
                          int kin, int k, int64_t m, int32_t since, hipStream_t st);
// Merge and Sort: list + set-aside rear part -> output rows.  Rows below
// rows_with_rear have a rear part: gin entries from k1 on (or, for base rows
// that balanced append leaves unselected, from min(kin, k) on).
struct FinalArgs {
    const uint64_t *L;
    const uint64_t *gin;
    int k, kin, k1;
    int64_t rows_with_rear, n;
    int balanced;
    int64_t n_raw;
    uint64_t seed;
    int32_t *out_ids;    // n x k, or nullptr
    float *out_dist;     // n x k, or nullptr
    uint64_t *out_keys;  // n x kin sorted keys (may be gin itself), or nullptr
    const int32_t *touched;  // when set, rows below rows_with_rear with touched[i] < tag0
                             // (never held a NEW entry) are left out
    int32_t tag0;
};
hipError_t launch_final(const FinalArgs &a, hipStream_t st);

// ---- serving (knng_prep.hip)
// Folds one request's merge into the resident graph: for base rows that held
// a NEW entry, its entries of request rows (local ids >= m_base, renumbered
// to first + id - m_base) are offered to the resident list (UpdateNN, set
// form, so commits of different requests commute); the request's own rows
// are copied, renumbered, to resident rows first .. first + n_req - 1.
struct CommitArgs {
    const uint64_t *out;     // (m_base + n_req) x gs final keys of the request
    int gs, k;
    const int32_t *touched;  // dtag of the request's merge (rows below tag0 untouched)
    int32_t tag0;
    int64_t m_base, n_req, first;
    uint64_t *res;           // resident lists, k per row
    uint64_t *ctr;
};
hipError_t launch_commit(const CommitArgs &a, hipStream_t st);
// rows of keys (stride src_stride, k used) sorted by (distance, id), empty
// slots last; written as keys (dst, stride dst_stride, padded with empty
// slots) and/or as ids / distances (n x k, -1 / +inf for empty slots)
hipError_t launch_sort_rows(const uint64_t *src, int src_stride, int64_t n, int k,
                            uint64_t *dst, int dst_stride, int32_t *ids, float *dist,
                            hipStream_t st);
hipError_t launch_zero_counters(uint64_t *ctr, int words, hipStream_t st);
hipError_t launch_fill_empty(uint64_t *p, int64_t rows, int k, hipStream_t st);

// ---- H-Merge (knng_prep.hip)
// Random order of n rows (the blocks H-Merge joins in are random subsets):
// perm[i] = the row placed at position i, from a 4-round Feistel network on
// 2*half bits (2^(2*half) >= n) walked until the value falls below n; then
// xp[i] = x[perm[i]] (rows of d floats).
hipError_t launch_permute_rows(const float *x, int64_t n, int d, uint64_t seed, int half,
                               int32_t *perm, float *xp, hipStream_t st);
// Graph over positions (ids and distances, n x k) back to row numbering: row
// perm[i] of out gets row i with every id j replaced by perm[j], sorted by
// (distance, id).
hipError_t launch_unpermute_graph(const int32_t *ids, const float *dist, int64_t n, int k,
                                  const int32_t *perm, int32_t *out_ids, float *out_dist,
                                  hipStream_t st);

// ---- knng_round.hip
hipError_t launch_sample(const RoundArgs &a, hipStream_t st);
hipError_t launch_prep_active(const RoundArgs &a, hipStream_t st);
hipError_t launch_reverse(const RoundArgs &a, hipStream_t st);
hipError_t launch_reverse_indexed(const RoundArgs &a, hipStream_t st);
// Reverse index of the first kk entries of each of the m lists of gin (row
// stride gs): off (m+1 words), src (up to m*kk), deg (m words) and part
// (rindex_parts(m) words) are caller-provided scratch/outputs; an id outside
// [0, m) sets ERR_ROW_REVERSE in ctr.
int64_t rindex_parts(int64_t m);
hipError_t launch_build_rindex(const uint64_t *gin, int gs, int kk, int64_t m, int64_t *off,
                               int32_t *src, int32_t *deg, int64_t *part, uint64_t *ctr,
                               hipStream_t st);
hipError_t launch_count_fresh(const RoundArgs &a, hipStream_t st);
// Graph mode.  set_round: the state at the start of a merge's loop (round 0).
// round_ctl, after the round's sampling: ends the loop when round t > 0 left
// c <= delta*n0*k entries, when t = max_rounds, or on an error bit (rounds =
// t); otherwise copies the round's active-row count and clears the per-round
// counters.  round_next, after the join: t += 1.  Grids of the graph-mode
// launches are fixed by `rows_cap` (the most rows a merge of the slot has).
hipError_t launch_set_round(DevRound *d, const DevRound &v, hipStream_t st);
hipError_t launch_round_ctl(const RoundArgs &a, int k, hipStream_t st);
hipError_t launch_round_next(const RoundArgs &a, hipStream_t st);

// ---- knng_join.hip
hipError_t launch_join(const Rows &R, int metric, int bf16, const RoundArgs &a, hipStream_t st);

// ---- knng_brute.hip
// Rows [a_lo,a_hi) against rows [b_lo,b_hi) of R; optional sorted initial
// keys per A row (kin each, indexed from a_lo); writes out rows a (global
// index a - out_base).  exclude_self skips a == b.
hipError_t launch_brute(const Rows &R, int metric, int64_t a_lo, int64_t a_hi, int64_t b_lo,
                        int64_t b_hi, const uint64_t *init, int kin, int k, int exclude_self,
                        int64_t out_base, int64_t id_base, int32_t *out_ids, float *out_dist,
                        hipStream_t st);

} // namespace knng
