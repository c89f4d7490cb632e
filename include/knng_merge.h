/*
 * knng_merge.h -- C ABI of libknngmerge.so, k-NN graph merge on one MI355X.
 *
 * Implements the two merge problems of Zhao, Wang, Lin and Ngo, "On the Merge
 * of k-NN Graph":
 *   knng_merge   symmetric merge, S-Merge (Section 3.1, Algorithm 1): two
 *                built graphs G1 of S1 and G2 of S2 become the graph of
 *                S1 u S2;
 *   knng_expand  joint merge, J-Merge (Section 3.2, Algorithm 2): a built
 *                graph G of S absorbs a raw set that has no graph yet;
 *   knng_merge_bruteforce   the exhaustive cross comparison that Section 1
 *                describes as the naive way to merge (deterministic);
 *   knng_exact_graph        the exact k-NN graph by brute force (Section 1's
 *                definition of G[i]), used to build inputs.
 *
 * Conventions shared by every entry point:
 *   - Pointers inside knng_set / knng_graph are DEVICE pointers (HIP device
 *     memory of the current device).  A host pointer is rejected with
 *     KNNG_EINVAL.  Row-major layouts: set rows are n x d fp32; graph rows are
 *     n x k int32 ids and n x k fp32 distances.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *     The merges read a 4-byte counter back to the host once per round and
 *     therefore synchronise the stream; results are valid on return.
 *   - The caller owns every buffer.  Inputs are never written.  Device
 *     scratch memory is the caller's `workspace` of at least the bytes that
 *     the matching *_workspace_size call returns; nothing is allocated on
 *     the device by these calls.  Outputs must not alias inputs.
 *   - Distances: l2 is the SQUARED Euclidean distance, l1 the sum of
 *     absolute differences, cosine is 1 - cos.  Smaller is closer.  Stored
 *     distances are canonical FP32 values (ascending-coordinate
 *     accumulation with fused multiply-add; see the design notes).
 *   - Output rows are sorted by (distance, id) ascending, hold no self and
 *     no duplicate ids; ids are global (rows of the first set first, then
 *     rows of the second).  When fewer than k neighbours exist a row is
 *     padded with id -1 and distance +inf.
 *   - Errors: no exception or abort crosses the ABI.  The return code says
 *     what failed and knng_last_error() (thread-local, valid until the next
 *     call on the same thread) says why.  On error the output content is
 *     unspecified and inputs are untouched.
 */
#ifndef KNNG_MERGE_H
#define KNNG_MERGE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KNNG_VERSION 10000 /* major*10000 + minor*100 + patch */

typedef enum {
    KNNG_OK = 0,
    KNNG_EINVAL = 1,  /* bad argument or invalid input data */
    KNNG_ENOMEM = 2,  /* workspace smaller than required, or host memory exhausted */
    KNNG_EDEVICE = 3, /* a HIP call failed; see knng_last_error() */
    KNNG_EBUSY = 4,   /* knng_server_wait: the request has not finished in time */
} knng_status;

typedef enum {
    KNNG_L2 = 0,     /* squared Euclidean */
    KNNG_COSINE = 1, /* 1 - cos; zero rows are rejected */
    KNNG_L1 = 2,     /* sum of |a_t - b_t| */
} knng_metric;

typedef enum {
    /* every joined pair evaluated in canonical FP32 */
    KNNG_FP32 = 0,
    /* block distances in BF16 on MFMA with FP32 accumulation, screened with a
     * bound that never drops a pair the FP32 path would insert; pairs that
     * pass are rescored in canonical FP32 before insertion (l2 and cosine;
     * l1 has no MFMA form and runs the FP32 path) */
    KNNG_BF16_RESCORE = 1,
} knng_precision;

/* opts.flags */
#define KNNG_FLAG_PROFILE 1u /* time each phase with HIP events (stats.ms_*) */
/* knng_expand only -- balanced append, for a raw set much smaller than the
 * base (a case Section 5.2's size-ratio study stops short of): a base row
 * takes part in Divide and Append only when a hash draw selects it, with
 * probability min(1, n_raw/n_base); the other base rows keep their whole
 * list, all OLD, and receive no samples.  Every raw row then meets about
 * k - k1 base rows through Append, as in the balanced case.  With
 * n_raw >= n_base every row is selected and the call is Algorithm 2 as
 * printed.  Rows that never hold a NEW entry are skipped by the rounds'
 * sampling and local join (they join nothing), so small raw sets cost little
 * beyond one pass over the lists per round. */
#define KNNG_FLAG_BALANCED_APPEND 2u

/*
 * Parameters of the merges.
 *   keep_ratio  r = k1/k, the share of each input list kept by Divide
 *               (Section 5.2 ablation; Sections 3.1-3.2 use 1/2).
 *               k1 = floor(r*k); the other k-k1 slots receive random samples.
 *   sample      s: NEW entries sampled per list per round, and the size of
 *               each sampled reverse list (NN-Descent sampling, which
 *               Section 3.1 invokes by citation).  1..32.
 *   delta       the repeat loop of Algorithms 1-2 stops when the number of
 *               entries inserted in a round (and still present at its end)
 *               is <= delta*n0*k, n0 = rows holding a NEW entry when the
 *               loop starts: every row of the call, except under balanced
 *               append (0 = until no update, as the paper states).
 *   max_rounds  cap on rounds (the paper has none).
 *   seed        seed of the counter-based random stream (SplitMix64).
 *   precision   knng_precision.  Under KNNG_BF16_RESCORE a rescored pair
 *               whose bf16 distance lies outside the proven screening margin
 *               (the bound failed; never observed) makes the call return
 *               KNNG_EDEVICE, with the count in stats->screen_violations.
 *   flags       KNNG_FLAG_*.
 * Constraints: 3*sample + k <= 160, 1 <= k <= 64.
 */
typedef struct {
    float keep_ratio;
    int32_t sample;
    float delta;
    int32_t max_rounds;
    uint64_t seed;
    int32_t precision;
    uint32_t flags;
} knng_opts;

/* a point set: n rows of d fp32 values, row-major, on the device; a set and
 * the union of the sets one call merges hold fewer than 2^30 - 64 rows (a
 * list entry keeps a row id in 30 bits), 1 <= d <= 65536 */
typedef struct {
    int64_t n;
    int32_t d;
    const float *x;
} knng_set;

/*
 * A k-NN graph: n rows of k entries.  As an INPUT, ids are LOCAL to the
 * graph's own set (0..n-1), rows must be duplicate-free and self-free, and
 * `dist` may be NULL (distances are then computed canonically and each row is
 * sorted) or must hold each row sorted by (distance, id).  Given distances
 * are trusted as they are.  As an OUTPUT, ids are global and both arrays are
 * written.
 */
typedef struct {
    int64_t n;
    int32_t k;
    int32_t *ids;
    float *dist;
} knng_graph;

#define KNNG_STATS_ROUNDS 64

/* Counters of one merge (all counts are exact, taken on the device). */
typedef struct {
    int32_t rounds;              /* rounds of the repeat loop run */
    int32_t max_group;           /* largest neighbourhood seen (|new|+|old|) */
    int64_t evals;               /* C of the scanning rate: distance evaluations
                                    of Append/Initialize and of the local joins */
    int64_t rescored;            /* BF16 path: pairs re-evaluated in FP32 */
    int64_t insert_attempts;     /* list inserts tried after the worst-entry screen */
    int64_t screen_violations;   /* BF16 path: rescored pairs whose bf16 distance left
                                    the proven error margin (0 unless the bound fails) */
    int64_t updates[KNNG_STATS_ROUNDS];  /* c: entries inserted and kept, per round */
    int64_t pairs[KNNG_STATS_ROUNDS];    /* joined pairs per round */
    int64_t gathered[KNNG_STATS_ROUNDS]; /* neighbourhood members staged per round */
    /* device time per phase in ms (KNNG_FLAG_PROFILE only) */
    double ms_prep, ms_init, ms_sample, ms_reverse, ms_join, ms_final;
    int32_t join_launches;
    int32_t reserved;
} knng_stats;

/* fills *o with keep_ratio 0.5, sample 10, delta 0, max_rounds 30, seed 0,
 * precision FP32, flags 0 */
void knng_opts_default(knng_opts *o);

/*
 * S-Merge (Algorithm 1): Divide G1 and G2 (first k1 entries kept, the rear
 * set aside), Append k-k1 distinct random samples of the other set to every
 * list, iterate the cross-set local join (only pairs from different sets are
 * compared), then Merge and Sort each list with its set-aside rear part.
 *   S1, G1: n1 rows; G1->k = kin1 >= k1.   S2, G2: n2 rows; kin2 >= k1.
 *   k: output list size, 1..min(64, n1+n2-1).
 *   out: n1+n2 rows, k columns; S1 rows first, S2 ids offset by n1.
 *   stats: may be NULL.
 * Returns KNNG_EINVAL for bad sizes/options, ids out of range, duplicate or
 * self ids, unsorted given rows, non-finite values or (cosine) zero rows.
 */
knng_status knng_merge(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                       const knng_graph *G2, int32_t k, knng_metric metric,
                       const knng_opts *opts, knng_graph *out, void *workspace,
                       size_t workspace_bytes, void *stream, knng_stats *stats);

size_t knng_merge_workspace_size(int64_t n1, int64_t n2, int32_t d, int32_t k, int32_t kin1,
                                 int32_t kin2, knng_metric metric, const knng_opts *opts);

/*
 * J-Merge (Algorithm 2): Divide G (base set S, n_b rows), Append k-k1 random
 * raw samples to every base list, Initialize every raw row with k random
 * samples of S u raw (self excluded), iterate the local join over pairs that
 * are not both from S (cross pairs and raw-raw pairs), then Merge and Sort
 * the base rows with their set-aside rear parts.
 *   S may have n = 0 (G ignored): the call is then an NN-Descent build of
 *   the raw set.  out: n_b + n_raw rows, base rows first.
 */
knng_status knng_expand(const knng_set *S, const knng_graph *G, const knng_set *raw, int32_t k,
                        knng_metric metric, const knng_opts *opts, knng_graph *out,
                        void *workspace, size_t workspace_bytes, void *stream,
                        knng_stats *stats);

size_t knng_expand_workspace_size(int64_t n_base, int64_t n_raw, int32_t d, int32_t k,
                                  int32_t kin, knng_metric metric, const knng_opts *opts);

/*
 * Merge of many blocks by repeated S-Merge: Section 1 merges more than two
 * graphs by recursive calls of the two-graph merge, and Section 3.1 (last
 * paragraph) merges sub-graphs built in parallel pairwise until one graph
 * remains.  Blocks are consecutive row ranges of X: block b holds rows
 * [starts[b], starts[b+1]) (`starts` is a HOST array of nblocks+1 entries,
 * starts[0] = 0, starts[nblocks] = X->n) and G[b] is its graph with ids local
 * to the block (any G[b].k >= k1; a block carried up unmerged needs >= k).
 * Level by level, neighbouring ranges (0,1), (2,3), ... are merged with
 * knng_merge; an odd last range moves up unchanged.  out: X->n rows, k
 * columns, ids = row indices of X.  stats (may be NULL): totals over all
 * merges; updates[l] holds the distance evaluations of level l, pairs[l] its
 * rounds and gathered[l] its wall time in microseconds.  The merges of one
 * level are independent and run at the same time, each in a host thread and
 * on a stream of its own (default priority) with a slice of the workspace;
 * the call first waits for `stream` and returns when `out` is complete.
 */
knng_status knng_merge_tree(const knng_set *X, const int64_t *starts, const knng_graph *G,
                            int32_t nblocks, int32_t k, knng_metric metric,
                            const knng_opts *opts, knng_graph *out, void *workspace,
                            size_t workspace_bytes, void *stream, knng_stats *stats);

size_t knng_merge_tree_workspace_size(int64_t n, int32_t d, int32_t nblocks,
                                      const int64_t *starts, int32_t k, int32_t kin_max,
                                      knng_metric metric, const knng_opts *opts);

/*
 * H-Merge (Section 3.3): the graph of X built layer by layer.  The rows are
 * taken in a random order (the blocks joined in must be random subsets):
 * position i holds row perm(i), a seeded bijection of [0, n) (a 4-round
 * Feistel network on the counter hash, walked until the value falls below
 * n).  NN-Descent (J-Merge with an empty base) builds the graph of the first
 * n_top positions; each later layer joins a raw block as large as the current
 * graph (the last one: the rows left) with J-Merge, doubling the rows until
 * all n are in.  Lists hold k/2 entries on every layer above the bottom one
 * and k on the bottom layer, at most the layer's rows - 1.  Layer l is seeded
 * SplitMix64(opts->seed ^ SplitMix64(l)); every layer uses opts otherwise
 * (keep_ratio must keep at most the upper layer's list size).
 *   out: X->n rows, k columns, ids = row indices of X, rows sorted by
 *   (distance, id).  stats (may be NULL): totals over the layers;
 *   updates[l], pairs[l] and gathered[l] hold layer l's distance
 *   evaluations, rounds and wall time in microseconds.  The workspace holds
 *   the permuted rows, two layer graphs and one J-Merge's workspace.
 *   Errors as knng_merge; n_top < 2 is EINVAL.
 */
knng_status knng_hmerge(const knng_set *X, int32_t k, int64_t n_top, knng_metric metric,
                        const knng_opts *opts, knng_graph *out, void *workspace,
                        size_t workspace_bytes, void *stream, knng_stats *stats);

size_t knng_hmerge_workspace_size(int64_t n, int32_t d, int32_t k, int64_t n_top,
                                  knng_metric metric, const knng_opts *opts);

/*
 * ------------------------------------------------ hierarchy, diversification, search
 * Section 4: the layers H-Merge builds form a hierarchy for NN search; each
 * layer's graph is diversified (Algorithm 3) and the search descends from the
 * top layer to the bottom one.
 *
 * knng_hierarchy_shape: the layers of knng_hmerge for n rows, top block
 * n_top and list size k: returns the layer count L (0 on bad arguments) and
 * writes the first min(L, cap) layer sizes to rows (host, may be NULL) and
 * list sizes to lists (host, may be NULL).  Layer l holds the first rows[l]
 * positions of the random order; rows[L-1] = n.
 */
int32_t knng_hierarchy_shape(int64_t n, int64_t n_top, int32_t k, int64_t *rows, int32_t *lists,
                             int32_t cap);

/*
 * knng_hmerge keeping its hierarchy (Section 3.3 builds it, Section 4 searches
 * it).  Arguments and workspace as knng_hmerge, and instead of `out`:
 *   perm    (device, n int32, may be NULL): perm[i] = the row of X at position i;
 *   xp      (device, n x d fp32, may be NULL): xp[i] = X[perm[i]];
 *   layers  (host array of nlayers graphs with device arrays): layer l is
 *           rows[l] x lists[l] (knng_hierarchy_shape), ids are positions
 *           (rows of xp), each row sorted by (distance, id), exactly the graph
 *           H-Merge built on that layer.
 * Returns after the outputs are complete.  nlayers must equal the layer count.
 */
knng_status knng_hmerge_hierarchy(const knng_set *X, int32_t k, int64_t n_top, knng_metric metric,
                                  const knng_opts *opts, int32_t *perm, float *xp,
                                  knng_graph *layers, int32_t nlayers, void *workspace,
                                  size_t workspace_bytes, void *stream, knng_stats *stats);

/*
 * Graph diversification (Algorithm 3, Section 4) of G (n = X->n rows of
 * G->k <= 64 entries; ids over the rows of X, -1 = empty; dist REQUIRED, each
 * row's stored distances m(a, s), canonical values as the merges write
 * them).  Per row a, Algorithm 3 keeps the nearest entry of a's list and then
 * every entry s, in (distance, id) order, that no kept entry c occludes
 * (m(s, c) < m(s, a), m(s, c) evaluated canonically); the same rule runs over
 * a's reverse list {b : a in G[b]} (at G[b]'s stored distance); the two kept
 * sets are merged, an id in both taken once, and the max_degree (1..64)
 * nearest by (distance, id) are written to out (n x max_degree, padded with
 * -1 / +inf).  Ids out of range, self ids and negative or non-finite
 * distances are KNNG_EINVAL.  Synchronises the stream before returning.
 */
knng_status knng_diversify(const knng_set *X, const knng_graph *G, int32_t max_degree,
                           knng_metric metric, knng_graph *out, void *workspace,
                           size_t workspace_bytes, void *stream);

size_t knng_diversify_workspace_size(int64_t n, int32_t d, int32_t k, knng_metric metric);

/*
 * NN search over a graph hierarchy (Section 4), one query per row of Q
 * (nq x d, device).  layers[0..nlayers) (host array, device ids; nlayers <=
 * 32): layer l is a graph over the rows 0 .. layers[l].n - 1 of X (each
 * layer a prefix of the next and of X; ids -1 = empty; layers[l].k <= 256),
 * typically the diversified layers of knng_hmerge_hierarchy over xp.
 *   Stage 1: from the vertex draw_below(H(seed, 0xD1, query, 0, 0),
 *     layers[0].n) of the top layer, on each upper layer move to the
 *     nearest neighbour of the current vertex while it is nearer than the
 *     current vertex, by (distance, id);
 *   Stage 2: on the bottom layer, a ranked list of at most ef entries starts
 *     with the vertex reached; the best entry not yet expanded is expanded
 *     (its neighbours not evaluated before are evaluated and the list keeps
 *     the ef best), until every entry is expanded.
 * out_ids / out_dist (device, nq x topk): the first topk entries (ids are
 * rows of X, canonical distances; padded with -1 / +inf).  1 <= topk <= ef <=
 * 256.  evals (host, may be NULL): distances evaluated.  Synchronises the
 * stream before returning.
 */
knng_status knng_search(const knng_set *X, const knng_graph *layers, int32_t nlayers,
                        const knng_set *Q, int32_t topk, int32_t ef, uint64_t seed,
                        knng_metric metric, int32_t *out_ids, float *out_dist, void *workspace,
                        size_t workspace_bytes, void *stream, int64_t *evals);

size_t knng_search_workspace_size(int64_t n, int32_t d, int64_t nq, knng_metric metric);

/*
 * knng_merge without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, semantics and errors as knng_merge, except:
 *   - the scratch is a fixed array of KNNG_NOALLOC_SCRATCH_BYTES bytes held
 *     by the library on every GPU it runs on, until the process ends; a
 *     merge whose knng_merge_workspace_size exceeds it returns KNNG_ENOMEM;
 *   - every call on one GPU shares that GPU's array: calls that overlap on
 *     one GPU (any streams, any threads) race and must not be issued;
 *   - nothing is allocated on the device; KNNG_FLAG_PROFILE (which creates
 *     HIP events) is refused with KNNG_EINVAL.
 */
#define KNNG_NOALLOC_SCRATCH_BYTES (64u << 20)

knng_status knng_merge_noalloc(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                               const knng_graph *G2, int32_t k, knng_metric metric,
                               const knng_opts *opts, knng_graph *out, void *stream,
                               knng_stats *stats);

/* KNNG_NOALLOC_SCRATCH_BYTES of the loaded library */
size_t knng_merge_noalloc_scratch_bytes(void);

/*
 * Brute-force cross merge (Section 1): row i of S1 becomes the top k of
 * G1[i] and every (m(x_i, y_j), n1+j); S2 rows likewise against S1.
 * Deterministic: equal to the exact result in canonical FP32 with ties broken
 * by the smaller id.  Arguments as in knng_merge (no options).
 */
knng_status knng_merge_bruteforce(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                                  const knng_graph *G2, int32_t k, knng_metric metric,
                                  knng_graph *out, void *workspace, size_t workspace_bytes,
                                  void *stream);

size_t knng_bruteforce_workspace_size(int64_t n1, int64_t n2, int32_t d, int32_t k,
                                      int32_t kin1, int32_t kin2, knng_metric metric);

/*
 * Exact k-NN graph of S (Section 1): each row's k smallest (distance, id)
 * over all other rows.  out: S->n rows, k columns, ids local to S.
 */
knng_status knng_exact_graph(const knng_set *S, int32_t k, knng_metric metric, knng_graph *out,
                             void *workspace, size_t workspace_bytes, void *stream);

size_t knng_exact_graph_workspace_size(int64_t n, int32_t d, int32_t k, knng_metric metric);

/*
 * ---------------------------------------------------------------- serving
 * J-Merge as a service (Section 3.2: a built graph absorbs raw data without
 * a rebuild).  A server holds, in device memory it owns, a base -- rows and
 * their k-NN lists, frozen between rebases -- and the resident graph: the
 * base rows, every accepted request's rows, and their lists.
 *
 * A request of raw rows is one knng_expand of the base with the request's
 * rows as the raw set, under KNNG_FLAG_BALANCED_APPEND, with seed
 * SM(opts->seed ^ SM(req_id)) (SM = the SplitMix64 output function of
 * state + 0x9E3779B97F4A7C15).  Its result therefore depends only on the
 * base, its rows and req_id, never on other requests: the same request gives
 * the same result alone and in any mix.  Row ids: base rows 0..m-1, then each
 * accepted request's rows in submission order (knng_request_info.first_id).
 *
 * When a request finishes, its rows' lists enter the resident graph and the
 * new entries of base rows are offered to the resident lists with the
 * set-form UpdateNN (top k of the union, ties by id), so the resident graph
 * does not depend on the order in which requests finish.  Requests merge with
 * the base only; knng_server_rebase makes the whole resident graph the base,
 * so later requests also meet earlier requests' rows.
 *
 * Requests run in slots: each slot is a stream, a host thread and a merge
 * workspace sized for the capacity.  Several requests are on the device at
 * once; a queued request starts as soon as a slot frees up.  The number of
 * slots is cfg->slots, lowered to what cfg->hbm_budget holds (slots = 0: no
 * thread, requests run inside knng_server_step).
 *
 * cfg->batching = 1 trades that independence for quality under load: a slot
 * that frees up takes every queued request that fits in max_request rows and
 * merges them as ONE raw set (seed from the first request's id), so requests
 * meet each other's rows; a request's result then depends on what it was
 * batched with (knng_request_info.merged_rows).
 *
 * Threads: submit, wait, step, snapshot, rebase and status may be called from
 * any threads concurrently; destroy must not overlap any other call on the
 * same server.  Work runs on the device that was current at creation.
 */
typedef struct knng_server knng_server;

typedef struct {
    int64_t capacity;    /* rows the server can ever hold: base + every request row */
    int64_t max_request; /* most rows in one request */
    uint64_t hbm_budget; /* device bytes the server may allocate; 0 = no limit */
    int32_t slots;       /* requests on the device at once; 0 = run in knng_server_step */
    int32_t batching;    /* 1: a slot merges all queued requests that fit as one raw set */
    int32_t host_rounds; /* 0: each slot runs the rounds of its merges as a launch graph of
                            one round, captured once and replayed (the device ends the loop;
                            one read-back per block of rounds); 1: one host round trip per
                            round (the merges' own loop) */
} knng_server_config;

typedef struct {
    int64_t first_id;   /* id of the request's first row */
    int64_t rows;       /* rows of the request */
    int64_t merged_first; /* id of the first raw row of the merge that ran it */
    int64_t merged_rows; /* raw rows of that merge (> rows when batched) */
    int64_t evals;      /* distance evaluations of its merge */
    int32_t rounds;     /* rounds of its repeat loop */
    int32_t slot;       /* slot that ran it (-1: none) */
    /* host steady clock, microseconds since the server was created */
    double submit_us;   /* knng_server_submit entered */
    double start_us;    /* its merge started */
    double done_us;     /* its result is on the host and committed */
} knng_request_info;

/* Device bytes of a server of this shape with `slots` slots (kin: columns of
 * the base graph). */
size_t knng_server_bytes(int64_t capacity, int64_t max_request, int32_t d, int32_t k, int32_t kin,
                         knng_metric metric, const knng_opts *opts, int32_t slots);

/*
 * Copies base (n_base x d, device) and its graph G (as for knng_expand: local
 * ids, rows sorted with distances or dist NULL, G->k >= k1) into server
 * memory, allocated once with hipMalloc.  KNNG_ENOMEM when cfg->hbm_budget
 * holds no slot.  Inputs are not kept.  *srv receives the server (NULL on
 * error).
 * Stream contract (also for device rows given to knng_server_submit): the
 * server reads its inputs on streams of its own, after waiting for the work
 * queued on the null stream; a caller that writes them on another stream
 * must synchronise that stream first.
 */
knng_status knng_server_create(const knng_set *base, const knng_graph *G, int32_t k,
                               knng_metric metric, const knng_opts *opts,
                               const knng_server_config *cfg, knng_server **srv);

/*
 * Queues n_raw rows (n_raw x d fp32, host or device memory; read before
 * return, so the buffer may be reused at once) under the caller's request id
 * req_id (which seeds its merge).  Rows are validated (KNNG_EINVAL:
 * non-finite values, zero rows under cosine; nothing is reserved then);
 * KNNG_ENOMEM when the capacity would be exceeded, KNNG_EINVAL when
 * n_raw > max_request.  *ticket identifies the request for knng_server_wait.
 */
knng_status knng_server_submit(knng_server *srv, const float *raw, int64_t n_raw, uint64_t req_id,
                               uint64_t *ticket);

/* servers without slots: runs the oldest queued request (*ran = 0 when none
 * was queued); the request's own result is collected by knng_server_wait,
 * and step returns an error only when the server has failed */
knng_status knng_server_step(knng_server *srv, int32_t *ran);

/*
 * Waits up to timeout_us (< 0: no limit) for the request; KNNG_EBUSY when it
 * has not finished.  On success ids / dist (n_raw x k, host or device; either
 * may be NULL) receive its rows' lists with global ids, and the ticket is
 * released (a second wait gives KNNG_EINVAL).  info (may be NULL) is filled
 * also when the request failed.
 */
knng_status knng_server_wait(knng_server *srv, uint64_t ticket, int64_t timeout_us,
                             int32_t *ids, float *dist, knng_request_info *info);

/* Waits until no request is queued or running, then writes the resident
 * graph (rows sorted by (distance, id)) to out (device, out->n >= rows,
 * out->k = k) when not NULL; *n_rows receives the row count.  KNNG_EBUSY on
 * a server without slots while requests are queued. */
knng_status knng_server_snapshot(knng_server *srv, knng_graph *out, int64_t *n_rows);

/* Waits like knng_server_snapshot, then makes the resident graph the base. */
knng_status knng_server_rebase(knng_server *srv);

/* rows of the base, request rows committed since the last rebase, request
 * rows accepted but not committed */
knng_status knng_server_status(knng_server *srv, int64_t *base_rows, int64_t *committed_rows,
                               int64_t *pending_rows);

/* slots the server runs (after the budget) */
int32_t knng_server_slots(const knng_server *srv);

/*
 * Failure isolation, test hook: the next request submitted (or queued) with
 * this req_id fails with KNNG_EDEVICE after its merge ran and before its
 * commit, as a request whose merge reported an error would.  A request that
 * fails before its commit fails alone: the base and the resident graph are
 * untouched, its rows keep their ids with empty lists (-1 / +inf), and the
 * server goes on serving.  (A failure during a commit stops the server.)
 */
knng_status knng_server_fail_request(knng_server *srv, uint64_t req_id);

/* Lets the requests in slots finish, then frees everything; queued requests
 * are dropped. */
void knng_server_destroy(knng_server *srv);

/* thread-local text of the last error ("" after success) */
const char *knng_last_error(void);

/* KNNG_VERSION of the loaded library */
int knng_version(void);

#ifdef __cplusplus
}
#endif

#endif /* KNNG_MERGE_H */
