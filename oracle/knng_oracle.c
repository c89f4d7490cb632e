/*
 * knng_oracle.c -- plain, slow CPU oracle for k-NN graph merge.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never calls, links or includes anything from here, and
 * this file includes nothing from the product path.
 *
 * What it computes (Zhao, Wang, Lin, Ngo, "On the Merge of k-NN Graph"):
 *   - metrics l2 (squared), l1 and cosine distance (Table 3 names them; the
 *     paper gives no formulas, so the plain textbook definitions are used);
 *   - the exact k-NN graph by brute force (Section 1, definition of G[i]);
 *   - the brute-force cross merge (Section 1: every cross pair is compared and
 *     inserted into both lists when it ranks in the top k);
 *   - symmetric merge, S-Merge (Algorithm 1, Section 3.1);
 *   - joint merge, J-Merge (Algorithm 2, Section 3.2);
 *   - the per-round statistics used by the tests: the update count c, the
 *     objective phi(G) of Eq. (1) and the number of distance evaluations C
 *     behind the scanning rate of Section 5.1;
 *   - graph diversification (Algorithm 3, Section 4) of a k-NN graph, its
 *     lists and reverse lists merged, and the two-stage top-down NN search
 *     over a hierarchy of graphs (Section 4).
 *
 * Precision: decisions (which id enters a list) are taken on canonical FP32
 * distances, evaluated in one fixed order written out below, because the GPU
 * takes the same decisions in FP32.  FP64 versions of the metrics exist for
 * error checks only.
 *
 * Canonical FP32 evaluation (ascending t, accumulator starts at +0):
 *   l2:     diff = a[t]-b[t];  acc = fmaf(diff, diff, acc)
 *   l1:     acc = acc + fabsf(a[t]-b[t])
 *   norm:   acc = fmaf(a[t], a[t], acc); norm = sqrtf(acc)
 *   cosine: D = l2(a,b); e = na-nb; num = fmaf(-e, e, D);
 *           den = (2*na)*nb; r = num/den; result = r > 0 ? r : +0
 *   The cosine form equals 1 - cos exactly in real arithmetic
 *   (|a-b|^2 = na^2 + nb^2 - 2ab) and avoids cancellation near 0.
 *
 * Random draws use SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the
 * generator with state x returns mix(x + 0x9E3779B97F4A7C15) where mix is its
 * published output function.  Tuples are hashed by chaining it:
 *   H(seed,tag,a,b,c) = sm(sm(sm(sm(seed ^ tag) ^ a) ^ b) ^ c).
 *
 * Readings of the paper where it is silent (each listed with its reason in
 * the design notes of the repository):
 *   - k1 = floor(r*k) entries are kept by Divide, k-k1 are appended;
 *   - appended and initial random samples are distinct, drawn by rejection
 *     from the hash stream, and never include the row itself;
 *   - NN-Descent sampling (cited, not spelled out, in Section 3.1): each round
 *     a row samples up to s NEW entries (smallest hash priority), marks them
 *     OLD, and keeps all previously OLD entries; reverse lists keep the s
 *     smallest-priority sources of each kind; new x new and new x old pairs
 *     are joined;
 *   - UpdateNN rejects self and ids already present, orders entries by
 *     (distance, id) and keeps at most k;
 *   - c is the number of entries present at the end of a round that were
 *     inserted during it; the loop stops when c <= delta*n0*k or after
 *     max_rounds rounds, n0 being the number of rows that hold a NEW entry
 *     when the loop starts (every row in both algorithms as printed);
 *   - Kept (Divide) entries start OLD, appended/initial entries start NEW;
 *   - balanced append (J-Merge of a raw set much smaller than the base, a
 *     case the paper's experiments stop short of): a base row takes part in
 *     Divide and Append only when a hash draw selects it, with probability
 *     min(1, n_raw/n_base); other base rows keep their whole list (OLD) and
 *     receive no samples.  With n_raw >= n_base every row is selected, which
 *     is Algorithm 2 as printed.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_L2 0
#define ORC_COS 1
#define ORC_L1 2

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2

#define TAG_APPEND 0xA1u
#define TAG_INIT 0xA2u
#define TAG_FWD 0xB1u
#define TAG_RNEW 0xB2u
#define TAG_ROLD 0xB3u
#define TAG_SELECT 0xA3u
#define TAG_PERM 0xC1u

/* ------------------------------------------------------------------------ */
/* SplitMix64                                                                */
/* ------------------------------------------------------------------------ */

uint64_t orc_splitmix64(uint64_t state)
{
    uint64_t z = state + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

uint64_t orc_hash(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b, uint64_t c)
{
    uint64_t h = orc_splitmix64(seed ^ tag);
    h = orc_splitmix64(h ^ a);
    h = orc_splitmix64(h ^ b);
    h = orc_splitmix64(h ^ c);
    return h;
}

/* a draw in [0, N) from the top 32 bits of a hash (multiply-shift) */
static uint32_t draw_below(uint64_t h, uint32_t N)
{
    return (uint32_t)(((h >> 32) * (uint64_t)N) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Distances                                                                 */
/* ------------------------------------------------------------------------ */

static float l2_f32(const float *a, const float *b, int d)
{
    float acc = 0.0f;
    for (int t = 0; t < d; t++) {
        float diff = a[t] - b[t];
        acc = fmaf(diff, diff, acc);
    }
    return acc;
}

static float l1_f32(const float *a, const float *b, int d)
{
    float acc = 0.0f;
    for (int t = 0; t < d; t++)
        acc = acc + fabsf(a[t] - b[t]);
    return acc;
}

float orc_norm32(const float *a, int d)
{
    float acc = 0.0f;
    for (int t = 0; t < d; t++)
        acc = fmaf(a[t], a[t], acc);
    return sqrtf(acc);
}

static float cos_f32(const float *a, const float *b, int d)
{
    float D = l2_f32(a, b, d);
    float na = orc_norm32(a, d);
    float nb = orc_norm32(b, d);
    float e = na - nb;
    float num = fmaf(-e, e, D);
    float den = (2.0f * na) * nb;
    float r = num / den;
    return r > 0.0f ? r : 0.0f;
}

float orc_dist32(int metric, const float *a, const float *b, int d)
{
    if (metric == ORC_L2)
        return l2_f32(a, b, d);
    if (metric == ORC_L1)
        return l1_f32(a, b, d);
    return cos_f32(a, b, d);
}

/* FP64 reference distances from the stored FP32 rows (plain definitions). */
double orc_dist64(int metric, const float *a, const float *b, int d)
{
    if (metric == ORC_L2) {
        double s = 0.0;
        for (int t = 0; t < d; t++) {
            double df = (double)a[t] - (double)b[t];
            s += df * df;
        }
        return s;
    }
    if (metric == ORC_L1) {
        double s = 0.0;
        for (int t = 0; t < d; t++)
            s += fabs((double)a[t] - (double)b[t]);
        return s;
    }
    double ab = 0.0, aa = 0.0, bb = 0.0;
    for (int t = 0; t < d; t++) {
        ab += (double)a[t] * (double)b[t];
        aa += (double)a[t] * (double)a[t];
        bb += (double)b[t] * (double)b[t];
    }
    return 1.0 - ab / (sqrt(aa) * sqrt(bb));
}

/* ------------------------------------------------------------------------ */
/* Bounded sorted k-NN list and UpdateNN                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    float dist;
    int32_t id;
    uint8_t isnew; /* NN-Descent flag: not yet used as a NEW sample */
    uint8_t fresh; /* inserted during the current round */
} entry_t;

typedef struct {
    entry_t *e; /* capacity k, sorted ascending by (dist, id) */
    int cnt;
} nnlist_t;

static int key_less(float da, int32_t ia, float db, int32_t ib)
{
    return da < db || (da == db && ia < ib);
}

/*
 * UpdateNN(G[owner], id, dist) of Algorithms 1 and 2: insert the edge unless
 * it is the owner itself, already present, or not among the k best.
 * Returns 1 when the list changed.
 */
static int update_nn(nnlist_t *L, int k, int32_t owner, int32_t id, float dist, uint8_t isnew,
                     uint8_t fresh)
{
    if (id == owner)
        return 0;
    for (int j = 0; j < L->cnt; j++)
        if (L->e[j].id == id)
            return 0;
    if (L->cnt == k && !key_less(dist, id, L->e[k - 1].dist, L->e[k - 1].id))
        return 0;
    int pos = L->cnt < k ? L->cnt : k - 1; /* slot freed (or appended) */
    while (pos > 0 && key_less(dist, id, L->e[pos - 1].dist, L->e[pos - 1].id)) {
        L->e[pos] = L->e[pos - 1];
        pos--;
    }
    L->e[pos].dist = dist;
    L->e[pos].id = id;
    L->e[pos].isnew = isnew;
    L->e[pos].fresh = fresh;
    if (L->cnt < k)
        L->cnt++;
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Small helpers                                                             */
/* ------------------------------------------------------------------------ */

typedef struct {
    uint64_t key; /* (priority << 32) | id  -- ordered by priority, then id */
} prio_t;

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

typedef struct {
    float dist;
    int32_t id;
} pair_t;

static int cmp_pair(const void *a, const void *b)
{
    const pair_t *x = (const pair_t *)a, *y = (const pair_t *)b;
    if (key_less(x->dist, x->id, y->dist, y->id))
        return -1;
    if (key_less(y->dist, y->id, x->dist, x->id))
        return 1;
    return 0;
}

/*
 * m distinct draws from [0, N) excluding 'skip' (skip = -1: none), in draw
 * order.  Draw t is H(seed, tag, row, t, 0).  When m equals the number of
 * admissible values all of them are taken in ascending order; if the draw
 * budget 64*m + 4096 runs out (practically never) the rest is filled with the
 * smallest values not yet taken.
 */
static void distinct_draws(uint64_t seed, uint32_t tag, uint64_t row, uint32_t N, int64_t skip,
                           int m, int32_t *out)
{
    uint32_t avail = N - (skip >= 0 ? 1u : 0u);
    int got = 0;
    if ((uint32_t)m >= avail) {
        for (uint32_t v = 0; v < N && got < m; v++)
            if ((int64_t)v != skip)
                out[got++] = (int32_t)v;
        return;
    }
    int64_t budget = 64 * (int64_t)m + 4096;
    for (int64_t t = 0; t < budget && got < m; t++) {
        uint64_t h = orc_hash(seed, tag, row, (uint64_t)t, 0);
        uint32_t v;
        if (skip >= 0) {
            v = draw_below(h, N - 1);
            if ((int64_t)v >= skip)
                v++;
        } else {
            v = draw_below(h, N);
        }
        int dup = 0;
        for (int j = 0; j < got; j++)
            if (out[j] == (int32_t)v)
                dup = 1;
        if (!dup)
            out[got++] = (int32_t)v;
    }
    for (uint32_t v = 0; v < N && got < m; v++) {
        if ((int64_t)v == skip)
            continue;
        int dup = 0;
        for (int j = 0; j < got; j++)
            if (out[j] == (int32_t)v)
                dup = 1;
        if (!dup)
            out[got++] = (int32_t)v;
    }
}

/* ------------------------------------------------------------------------ */
/* Exact graph and brute-force cross merge                                   */
/* ------------------------------------------------------------------------ */

/*
 * Exact k-NN graph of X (n x d): for each row the k smallest (dist, id) over
 * all other rows.  Rows with fewer than k others are padded with (-1, +inf).
 */
int orc_exact_graph(const float *X, int64_t n, int d, int k, int metric, int32_t *ids, float *dist)
{
    if (n < 1 || d < 1 || k < 1)
        return ORC_EINVAL;
    nnlist_t L;
    L.e = (entry_t *)malloc(sizeof(entry_t) * (size_t)k);
    if (!L.e)
        return ORC_ENOMEM;
    for (int64_t i = 0; i < n; i++) {
        L.cnt = 0;
        for (int64_t j = 0; j < n; j++) {
            if (j == i)
                continue;
            float l = orc_dist32(metric, X + i * d, X + j * d, d);
            update_nn(&L, k, (int32_t)i, (int32_t)j, l, 0, 0);
        }
        for (int j = 0; j < k; j++) {
            ids[i * k + j] = j < L.cnt ? L.e[j].id : -1;
            dist[i * k + j] = j < L.cnt ? L.e[j].dist : INFINITY;
        }
    }
    free(L.e);
    return ORC_OK;
}

/*
 * Read one input graph row into (dist, id) pairs with global ids.  Given
 * distances are trusted; with dist == NULL they are computed canonically and
 * the row is sorted.  Rows must hold distinct in-range non-self ids and, when
 * distances are given, be sorted by (dist, id).
 */
static int load_row(const float *X, int d, int metric, int64_t row_global, int64_t id_offset,
                    int64_t n_local, const int32_t *ids, const float *dist, int kin, pair_t *out)
{
    for (int j = 0; j < kin; j++) {
        int32_t loc = ids[j];
        if (loc < 0 || loc >= n_local)
            return ORC_EINVAL;
        int64_t g = loc + id_offset;
        if (g == row_global)
            return ORC_EINVAL;
        for (int q = 0; q < j; q++)
            if (out[q].id == (int32_t)g)
                return ORC_EINVAL;
        out[j].id = (int32_t)g;
        if (dist) {
            out[j].dist = dist[j];
            if (!(dist[j] >= 0.0f) || isinf(dist[j]))
                return ORC_EINVAL;
        } else {
            out[j].dist = orc_dist32(metric, X + row_global * d, X + g * d, d);
        }
    }
    if (dist) {
        for (int j = 1; j < kin; j++)
            if (key_less(out[j].dist, out[j].id, out[j - 1].dist, out[j - 1].id))
                return ORC_EINVAL;
    } else {
        qsort(out, (size_t)kin, sizeof(pair_t), cmp_pair);
    }
    return ORC_OK;
}

static float *concat_rows(const float *X1, int64_t n1, const float *X2, int64_t n2, int d)
{
    float *X = (float *)malloc(sizeof(float) * (size_t)(n1 + n2) * (size_t)d);
    if (!X)
        return NULL;
    if (n1)
        memcpy(X, X1, sizeof(float) * (size_t)n1 * (size_t)d);
    if (n2)
        memcpy(X + n1 * d, X2, sizeof(float) * (size_t)n2 * (size_t)d);
    return X;
}

static int check_inputs(const float *X, int64_t n, int d, int metric)
{
    for (int64_t i = 0; i < n; i++) {
        for (int t = 0; t < d; t++)
            if (!isfinite(X[i * d + t]))
                return ORC_EINVAL;
        if (metric == ORC_COS && orc_norm32(X + i * d, d) == 0.0f)
            return ORC_EINVAL;
    }
    return ORC_OK;
}

/*
 * Brute-force cross merge: for x_i in S1 the output row is the top k of
 * G1[i] and every (m(x_i, y_j), n1+j); symmetrically for S2 rows.
 * Output ids are global (S1 rows first).
 */
int orc_merge_bruteforce(const float *X1, int64_t n1, const float *X2, int64_t n2, int d,
                         const int32_t *g1_ids, const float *g1_dist, int kin1,
                         const int32_t *g2_ids, const float *g2_dist, int kin2, int k, int metric,
                         int32_t *out_ids, float *out_dist)
{
    if (n1 < 1 || n2 < 1 || d < 1 || k < 1 || kin1 < 0 || kin2 < 0)
        return ORC_EINVAL;
    if (kin1 > n1 - 1 || kin2 > n2 - 1 || k > n1 + n2 - 1)
        return ORC_EINVAL;
    int64_t n = n1 + n2;
    float *X = concat_rows(X1, n1, X2, n2, d);
    if (!X)
        return ORC_ENOMEM;
    int rc = check_inputs(X, n, d, metric);
    int kmax = kin1 > kin2 ? kin1 : kin2;
    pair_t *row = (pair_t *)malloc(sizeof(pair_t) * (size_t)(kmax + 1));
    nnlist_t L;
    L.e = (entry_t *)malloc(sizeof(entry_t) * (size_t)k);
    if (!row || !L.e)
        rc = ORC_ENOMEM;
    for (int64_t i = 0; i < n && rc == ORC_OK; i++) {
        int own1 = i < n1;
        int kin = own1 ? kin1 : kin2;
        const int32_t *gi = own1 ? g1_ids + i * kin1 : g2_ids + (i - n1) * kin2;
        const float *gd = own1 ? (g1_dist ? g1_dist + i * kin1 : NULL)
                               : (g2_dist ? g2_dist + (i - n1) * kin2 : NULL);
        rc = load_row(X, d, metric, i, own1 ? 0 : n1, own1 ? n1 : n2, gi, gd, kin, row);
        if (rc != ORC_OK)
            break;
        L.cnt = 0;
        for (int j = 0; j < kin; j++)
            update_nn(&L, k, (int32_t)i, row[j].id, row[j].dist, 0, 0);
        int64_t lo = own1 ? n1 : 0, hi = own1 ? n : n1;
        for (int64_t j = lo; j < hi; j++) {
            float l = orc_dist32(metric, X + i * d, X + j * d, d);
            update_nn(&L, k, (int32_t)i, (int32_t)j, l, 0, 0);
        }
        for (int j = 0; j < k; j++) {
            out_ids[i * k + j] = j < L.cnt ? L.e[j].id : -1;
            out_dist[i * k + j] = j < L.cnt ? L.e[j].dist : INFINITY;
        }
    }
    free(row);
    free(L.e);
    free(X);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* S-Merge and J-Merge                                                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    float keep_ratio; /* r = k1 / k */
    int32_t sample;   /* s: NEW samples per list and per reverse list */
    float delta;      /* stop when c <= delta * n0 * k */
    int32_t max_rounds;
    uint64_t seed;
} orc_params;

typedef struct {
    int32_t rounds;
    int64_t evals;     /* C: distance evaluations (append/init + joins) */
    int64_t c[256];    /* per-round update count (first min(rounds,256)) */
    double phi[257];   /* phi(U^t), t = 0 (after append) .. rounds */
    int64_t pairs[256]; /* joined pairs per round */
} orc_stats;

typedef struct {
    int64_t n, n1; /* n1: rows of the first set (S1, or the base set) */
    int d, k, metric, joint;
    const float *X;
    nnlist_t *G;
    entry_t *store;
} state_t;

/* the join predicate of Algorithm 1 (cross pairs) or Algorithm 2 (cross or raw-raw) */
static int joinable(const state_t *S, int32_t p, int32_t q)
{
    int p1 = p < S->n1, q1 = q < S->n1;
    if (S->joint)
        return !(p1 && q1);
    return p1 != q1;
}

static double phi_of(const state_t *S)
{
    double s = 0.0;
    for (int64_t i = 0; i < S->n; i++)
        for (int j = 0; j < S->G[i].cnt; j++)
            s += (double)S->G[i].e[j].dist;
    return s;
}

static int add_unique(int32_t *arr, int cnt, int32_t v)
{
    for (int j = 0; j < cnt; j++)
        if (arr[j] == v)
            return cnt;
    arr[cnt] = v;
    return cnt + 1;
}

/*
 * The NN-Descent iteration shared by both merges (the repeat loop of
 * Algorithms 1 and 2).  Returns ORC_OK or ORC_ENOMEM.
 */
static int iterate(state_t *S, const orc_params *P, orc_stats *st)
{
    int64_t n = S->n;
    int k = S->k, s = P->sample;
    int32_t *new_f = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)s);
    int32_t *old_f = (int32_t *)malloc(sizeof(int32_t) * (size_t)n * (size_t)k);
    int *n_new_f = (int *)calloc((size_t)n, sizeof(int));
    int *n_old_f = (int *)calloc((size_t)n, sizeof(int));
    uint64_t **rcand_new = (uint64_t **)calloc((size_t)n, sizeof(uint64_t *));
    uint64_t **rcand_old = (uint64_t **)calloc((size_t)n, sizeof(uint64_t *));
    int *rc_new = (int *)calloc((size_t)n, sizeof(int)), *rc_old = (int *)calloc((size_t)n, sizeof(int));
    int *cap_new = (int *)calloc((size_t)n, sizeof(int)), *cap_old = (int *)calloc((size_t)n, sizeof(int));
    uint64_t *tmp = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(k + 1));
    int32_t *grp_new = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * s));
    int32_t *grp_old = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + s));
    int rc = ORC_OK;
    if (!new_f || !old_f || !n_new_f || !n_old_f || !rcand_new || !rcand_old || !rc_new ||
        !rc_old || !cap_new || !cap_old || !tmp || !grp_new || !grp_old) {
        rc = ORC_ENOMEM;
        goto done;
    }
    st->rounds = 0;
    st->phi[0] = phi_of(S);
    /* n0: rows that start the loop with a NEW entry (normaliser of delta) */
    int64_t n0 = 0;
    for (int64_t u = 0; u < n; u++) {
        int any = 0;
        for (int j = 0; j < S->G[u].cnt; j++)
            any |= S->G[u].e[j].isnew;
        n0 += any;
    }
    for (int t = 0; t < P->max_rounds; t++) {
        /* forward sample: up to s NEW entries by smallest priority become
         * the NEW sample and are marked OLD; previously OLD entries are all
         * kept as the OLD sample.  Fresh marks of the last round are cleared. */
        for (int64_t u = 0; u < n; u++) {
            nnlist_t *L = &S->G[u];
            int nn = 0, no = 0;
            for (int j = 0; j < L->cnt; j++) {
                L->e[j].fresh = 0;
                if (L->e[j].isnew) {
                    uint64_t pr = orc_hash(P->seed, TAG_FWD, (uint64_t)t, (uint64_t)u,
                                           (uint64_t)L->e[j].id) >> 32;
                    tmp[nn++] = (pr << 32) | (uint32_t)L->e[j].id;
                } else {
                    old_f[u * k + no++] = L->e[j].id;
                }
            }
            qsort(tmp, (size_t)nn, sizeof(uint64_t), cmp_u64);
            int take = nn < s ? nn : s;
            for (int j = 0; j < take; j++) {
                int32_t id = (int32_t)(tmp[j] & 0xFFFFFFFFu);
                new_f[u * s + j] = id;
                for (int q = 0; q < L->cnt; q++)
                    if (L->e[q].id == id)
                        L->e[q].isnew = 0;
            }
            n_new_f[u] = take;
            n_old_f[u] = no;
        }
        /* Reverse(G): every sampled edge u -> v offers u to v's reverse list */
        for (int64_t v = 0; v < n; v++)
            rc_new[v] = rc_old[v] = 0;
        for (int pass = 0; pass < 2; pass++) {
            for (int64_t u = 0; u < n; u++) {
                int cnt = pass == 0 ? n_new_f[u] : n_old_f[u];
                const int32_t *src = pass == 0 ? new_f + u * s : old_f + u * k;
                for (int j = 0; j < cnt; j++) {
                    int32_t v = src[j];
                    uint64_t pr = orc_hash(P->seed, pass == 0 ? TAG_RNEW : TAG_ROLD, (uint64_t)t,
                                           (uint64_t)v, (uint64_t)u) >> 32;
                    uint64_t **cand = pass == 0 ? rcand_new : rcand_old;
                    int *cn = pass == 0 ? rc_new : rc_old;
                    int *cap = pass == 0 ? cap_new : cap_old;
                    if (cn[v] == cap[v]) {
                        int nc = cap[v] ? 2 * cap[v] : 8;
                        uint64_t *p = (uint64_t *)realloc(cand[v], sizeof(uint64_t) * (size_t)nc);
                        if (!p) {
                            rc = ORC_ENOMEM;
                            goto done;
                        }
                        cand[v] = p;
                        cap[v] = nc;
                    }
                    cand[v][cn[v]++] = (pr << 32) | (uint32_t)u;
                }
            }
        }
        for (int64_t v = 0; v < n; v++) {
            qsort(rcand_new[v], (size_t)rc_new[v], sizeof(uint64_t), cmp_u64);
            qsort(rcand_old[v], (size_t)rc_old[v], sizeof(uint64_t), cmp_u64);
            if (rc_new[v] > s)
                rc_new[v] = s;
            if (rc_old[v] > s)
                rc_old[v] = s;
        }
        /* local join on every neighbourhood G[u] = reverse(u) + forward(u) */
        int64_t pairs = 0;
        for (int64_t u = 0; u < n; u++) {
            int gn = 0, go = 0;
            for (int j = 0; j < n_new_f[u]; j++)
                gn = add_unique(grp_new, gn, new_f[u * s + j]);
            for (int j = 0; j < rc_new[u]; j++)
                gn = add_unique(grp_new, gn, (int32_t)(rcand_new[u][j] & 0xFFFFFFFFu));
            for (int pass = 0; pass < 2; pass++) {
                int cnt = pass == 0 ? n_old_f[u] : rc_old[u];
                for (int j = 0; j < cnt; j++) {
                    int32_t v = pass == 0 ? old_f[u * k + j]
                                          : (int32_t)(rcand_old[u][j] & 0xFFFFFFFFu);
                    int in_new = 0;
                    for (int q = 0; q < gn; q++)
                        if (grp_new[q] == v)
                            in_new = 1;
                    if (!in_new)
                        go = add_unique(grp_old, go, v);
                }
            }
            for (int a = 0; a < gn; a++) {
                int32_t p = grp_new[a];
                for (int b = a + 1; b < gn + go; b++) {
                    int32_t q = b < gn ? grp_new[b] : grp_old[b - gn];
                    if (!joinable(S, p, q))
                        continue;
                    float l = orc_dist32(S->metric, S->X + (int64_t)p * S->d,
                                         S->X + (int64_t)q * S->d, S->d);
                    pairs++;
                    update_nn(&S->G[p], k, p, q, l, 1, 1);
                    update_nn(&S->G[q], k, q, p, l, 1, 1);
                }
            }
        }
        int64_t c = 0;
        for (int64_t i = 0; i < n; i++)
            for (int j = 0; j < S->G[i].cnt; j++)
                c += S->G[i].e[j].fresh;
        st->evals += pairs;
        if (t < 256) {
            st->c[t] = c;
            st->pairs[t] = pairs;
            st->phi[t + 1] = phi_of(S);
        }
        st->rounds = t + 1;
        if ((double)c <= (double)P->delta * (double)n0 * (double)k)
            break;
    }
done:
    if (rcand_new)
        for (int64_t v = 0; v < n; v++)
            free(rcand_new[v]);
    if (rcand_old)
        for (int64_t v = 0; v < n; v++)
            free(rcand_old[v]);
    free(new_f);
    free(old_f);
    free(n_new_f);
    free(n_old_f);
    free(rcand_new);
    free(rcand_old);
    free(rc_new);
    free(rc_old);
    free(cap_new);
    free(cap_old);
    free(tmp);
    free(grp_new);
    free(grp_old);
    return rc;
}

/* balanced append: base row i joins Divide and Append when
 * floor(hi32(H(seed, SELECT, i, 0, 0)) * nb / 2^32) < nr, i.e. with
 * probability min(1, nr/nb); every row when nr >= nb or when not balanced */
static int selected_base_row(uint64_t seed, int balanced, int64_t i, int64_t nb, int64_t nr)
{
    if (!balanced || nr >= nb)
        return 1;
    uint64_t h = orc_hash(seed, TAG_SELECT, (uint64_t)i, 0, 0);
    return (int64_t)(((h >> 32) * (uint64_t)nb) >> 32) < nr;
}

static int check_params(const orc_params *P, int k)
{
    if (!(P->keep_ratio >= 0.0f && P->keep_ratio <= 1.0f))
        return ORC_EINVAL;
    if (P->sample < 1 || P->max_rounds < 0 || !(P->delta >= 0.0f))
        return ORC_EINVAL;
    if (k < 1 || k > 64)
        return ORC_EINVAL;
    return ORC_OK;
}

/* Merge and Sort: top k of the iterated list and the set-aside rear part. */
static void merge_and_sort(const nnlist_t *L, const pair_t *rear, int nrear, int k, int32_t owner,
                           int32_t *out_ids, float *out_dist, entry_t *scratch)
{
    nnlist_t M;
    M.e = scratch;
    M.cnt = 0;
    for (int j = 0; j < L->cnt; j++)
        update_nn(&M, k, owner, L->e[j].id, L->e[j].dist, 0, 0);
    for (int j = 0; j < nrear; j++)
        update_nn(&M, k, owner, rear[j].id, rear[j].dist, 0, 0);
    for (int j = 0; j < k; j++) {
        out_ids[j] = j < M.cnt ? M.e[j].id : -1;
        out_dist[j] = j < M.cnt ? M.e[j].dist : INFINITY;
    }
}

/*
 * S-Merge (Algorithm 1).  S1 = X1 (n1 rows, graph G1 with kin1 columns of
 * local ids), S2 = X2 (n2 rows, G2 with kin2 columns of local ids).  Output:
 * n1+n2 rows of k global ids (S1 rows first) and canonical distances.
 */
int orc_smerge(const float *X1, int64_t n1, const float *X2, int64_t n2, int d,
               const int32_t *g1_ids, const float *g1_dist, int kin1, const int32_t *g2_ids,
               const float *g2_dist, int kin2, int k, int metric, const orc_params *P,
               int32_t *out_ids, float *out_dist, orc_stats *st)
{
    if (n1 < 1 || n2 < 1 || d < 1 || check_params(P, k) != ORC_OK)
        return ORC_EINVAL;
    int k1 = (int)floorf(P->keep_ratio * (float)k);
    if (kin1 < k1 || kin2 < k1 || kin1 > 64 || kin2 > 64 || kin1 > n1 - 1 || kin2 > n2 - 1)
        return ORC_EINVAL;
    if (k > n1 + n2 - 1)
        return ORC_EINVAL;
    memset(st, 0, sizeof(*st));
    int64_t n = n1 + n2;
    state_t S;
    S.n = n;
    S.n1 = n1;
    S.d = d;
    S.k = k;
    S.metric = metric;
    S.joint = 0;
    float *X = concat_rows(X1, n1, X2, n2, d);
    S.X = X;
    S.G = (nnlist_t *)malloc(sizeof(nnlist_t) * (size_t)n);
    S.store = (entry_t *)malloc(sizeof(entry_t) * (size_t)n * (size_t)k);
    int kinmax = kin1 > kin2 ? kin1 : kin2;
    pair_t *rear = (pair_t *)malloc(sizeof(pair_t) * (size_t)n * (size_t)(kinmax + 1));
    int *nrear = (int *)malloc(sizeof(int) * (size_t)n);
    pair_t *row = (pair_t *)malloc(sizeof(pair_t) * (size_t)(kinmax + 1));
    int32_t *draws = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
    entry_t *scratch = (entry_t *)malloc(sizeof(entry_t) * (size_t)k);
    int rc = ORC_OK;
    if (!X || !S.G || !S.store || !rear || !nrear || !row || !draws || !scratch) {
        rc = ORC_ENOMEM;
        goto out;
    }
    rc = check_inputs(X, n, d, metric);
    /* Divide: the first k1 entries stay (OLD), the rear part is set aside. */
    for (int64_t i = 0; i < n && rc == ORC_OK; i++) {
        int own1 = i < n1;
        int kin = own1 ? kin1 : kin2;
        const int32_t *gi = own1 ? g1_ids + i * kin1 : g2_ids + (i - n1) * kin2;
        const float *gd = own1 ? (g1_dist ? g1_dist + i * kin1 : NULL)
                               : (g2_dist ? g2_dist + (i - n1) * kin2 : NULL);
        rc = load_row(X, d, metric, i, own1 ? 0 : n1, own1 ? n1 : n2, gi, gd, kin, row);
        if (rc != ORC_OK)
            break;
        S.G[i].e = S.store + i * k;
        S.G[i].cnt = 0;
        for (int j = 0; j < k1; j++)
            update_nn(&S.G[i], k, (int32_t)i, row[j].id, row[j].dist, 0, 0);
        nrear[i] = kin - k1;
        for (int j = k1; j < kin; j++)
            rear[i * (kinmax + 1) + (j - k1)] = row[j];
    }
    if (rc != ORC_OK)
        goto out;
    /* Append k - k1 random samples of the other set (NEW). */
    for (int64_t i = 0; i < n; i++) {
        int own1 = i < n1;
        int64_t N = own1 ? n2 : n1;
        int m = (int64_t)(k - k1) < N ? k - k1 : (int)N;
        distinct_draws(P->seed, TAG_APPEND, (uint64_t)i, (uint32_t)N, -1, m, draws);
        for (int j = 0; j < m; j++) {
            int32_t g = own1 ? (int32_t)(n1 + draws[j]) : draws[j];
            float l = orc_dist32(metric, X + i * d, X + (int64_t)g * d, d);
            st->evals++;
            update_nn(&S.G[i], k, (int32_t)i, g, l, 1, 0);
        }
    }
    rc = iterate(&S, P, st);
    if (rc != ORC_OK)
        goto out;
    for (int64_t i = 0; i < n; i++)
        merge_and_sort(&S.G[i], rear + i * (kinmax + 1), nrear[i], k, (int32_t)i,
                       out_ids + i * k, out_dist + i * k, scratch);
out:
    free(X);
    free(S.G);
    free(S.store);
    free(rear);
    free(nrear);
    free(row);
    free(draws);
    free(scratch);
    return rc;
}

/*
 * J-Merge (Algorithm 2).  Base set S1 = Xb (nb rows, graph G with kin
 * columns of local ids) absorbs the raw set S2 = Xr (nr rows, no graph).
 * Output: nb+nr rows of k global ids (base rows first).  nb = 0 is allowed
 * and then the call is a plain NN-Descent build of the raw set.
 */
int orc_jmerge(const float *Xb, int64_t nb, const float *Xr, int64_t nr, int d,
               const int32_t *g_ids, const float *g_dist, int kin, int k, int metric,
               const orc_params *P, int balanced, int32_t *out_ids, float *out_dist,
               orc_stats *st)
{
    if (nb < 0 || nr < 1 || d < 1 || check_params(P, k) != ORC_OK)
        return ORC_EINVAL;
    int k1 = (int)floorf(P->keep_ratio * (float)k);
    if (nb > 0 && (kin < k1 || kin > 64 || kin > nb - 1))
        return ORC_EINVAL;
    if (nb == 0)
        kin = 0;
    if (k > nb + nr - 1)
        return ORC_EINVAL;
    memset(st, 0, sizeof(*st));
    int64_t n = nb + nr;
    state_t S;
    S.n = n;
    S.n1 = nb;
    S.d = d;
    S.k = k;
    S.metric = metric;
    S.joint = 1;
    float *X = concat_rows(Xb, nb, Xr, nr, d);
    S.X = X;
    S.G = (nnlist_t *)malloc(sizeof(nnlist_t) * (size_t)n);
    S.store = (entry_t *)malloc(sizeof(entry_t) * (size_t)n * (size_t)k);
    pair_t *rear = (pair_t *)malloc(sizeof(pair_t) * (size_t)(nb + 1) * (size_t)(kin + 1));
    int *nrear = (int *)malloc(sizeof(int) * (size_t)(nb + 1));
    pair_t *row = (pair_t *)malloc(sizeof(pair_t) * (size_t)(kin + 1));
    int32_t *draws = (int32_t *)malloc(sizeof(int32_t) * (size_t)(k + 1));
    entry_t *scratch = (entry_t *)malloc(sizeof(entry_t) * (size_t)k);
    int rc = ORC_OK;
    if (!X || !S.G || !S.store || !rear || !nrear || !row || !draws || !scratch) {
        rc = ORC_ENOMEM;
        goto out;
    }
    rc = check_inputs(X, n, d, metric);
    for (int64_t i = 0; i < nb && rc == ORC_OK; i++) {
        rc = load_row(X, d, metric, i, 0, nb, g_ids + i * kin, g_dist ? g_dist + i * kin : NULL,
                      kin, row);
        if (rc != ORC_OK)
            break;
        S.G[i].e = S.store + i * k;
        S.G[i].cnt = 0;
        /* Divide keeps k1 entries of a selected row; an unselected row
         * (balanced append only) keeps all it can hold */
        int keep = selected_base_row(P->seed, balanced, i, nb, nr) ? k1 : (kin < k ? kin : k);
        for (int j = 0; j < keep; j++)
            update_nn(&S.G[i], k, (int32_t)i, row[j].id, row[j].dist, 0, 0);
        nrear[i] = kin - keep;
        for (int j = keep; j < kin; j++)
            rear[i * (kin + 1) + (j - keep)] = row[j];
    }
    if (rc != ORC_OK)
        goto out;
    /* selected base rows: Append k - k1 random raw samples (NEW) */
    for (int64_t i = 0; i < nb; i++) {
        if (!selected_base_row(P->seed, balanced, i, nb, nr))
            continue;
        int m = (int64_t)(k - k1) < nr ? k - k1 : (int)nr;
        distinct_draws(P->seed, TAG_APPEND, (uint64_t)i, (uint32_t)nr, -1, m, draws);
        for (int j = 0; j < m; j++) {
            int32_t g = (int32_t)(nb + draws[j]);
            float l = orc_dist32(metric, X + i * d, X + (int64_t)g * d, d);
            st->evals++;
            update_nn(&S.G[i], k, (int32_t)i, g, l, 1, 0);
        }
    }
    /* raw rows: Initialize with k random samples of S1 u S2, self excluded */
    for (int64_t g = nb; g < n; g++) {
        S.G[g].e = S.store + g * k;
        S.G[g].cnt = 0;
        int m = (int64_t)k < n - 1 ? k : (int)(n - 1);
        distinct_draws(P->seed, TAG_INIT, (uint64_t)g, (uint32_t)n, g, m, draws);
        for (int j = 0; j < m; j++) {
            float l = orc_dist32(metric, X + g * d, X + (int64_t)draws[j] * d, d);
            st->evals++;
            update_nn(&S.G[g], k, (int32_t)g, draws[j], l, 1, 0);
        }
    }
    rc = iterate(&S, P, st);
    if (rc != ORC_OK)
        goto out;
    for (int64_t i = 0; i < n; i++)
        merge_and_sort(&S.G[i], i < nb ? rear + i * (kin + 1) : NULL, i < nb ? nrear[i] : 0, k,
                       (int32_t)i, out_ids + i * k, out_dist + i * k, scratch);
out:
    free(X);
    free(S.G);
    free(S.store);
    free(rear);
    free(nrear);
    free(row);
    free(draws);
    free(scratch);
    return rc;
}

/*
 * FP64 distances of query rows to every row of X, for recall ground truth:
 * out[q*n + j] = m64(X[rows[q]], X[j]).
 */
void orc_dist64_rows(const float *X, int64_t n, int d, int metric, const int64_t *rows,
                     int64_t nrows, double *out)
{
    for (int64_t q = 0; q < nrows; q++)
        for (int64_t j = 0; j < n; j++)
            out[q * n + j] = orc_dist64(metric, X + rows[q] * d, X + j * d, d);
}

/* The distinct random draws used by Append and Initialize (exposed for tests). */
void orc_draws(uint64_t seed, uint32_t tag, uint64_t row, uint32_t N, int64_t skip, int m,
               int32_t *out)
{
    distinct_draws(seed, tag, row, N, skip, m, out);
}

/*
 * The order in which H-Merge (Section 3.3) takes the rows; the blocks it
 * joins in must be random subsets of the whole set.  Reading: a seeded
 * bijection of [0, n).  Let h >= 1 be the smallest count with 4^h >= n.  A
 * balanced Feistel network of four rounds on 2h-bit values splits x into a
 * high half L and a low half R (h bits each); round r (0..3) replaces (L, R)
 * with (R, L xor F_r(R)), where F_r(R) is the low h bits of
 * H(seed, PERM, r, R, 0).  Every round is invertible, so the network permutes
 * [0, 4^h); a result >= n is put through the network again until it falls
 * below n ("cycle walking", Black and Rogaway, Ciphers with Arbitrary Finite
 * Domains, 2002), which keeps a bijection on [0, n).  order[i] = the row at
 * position i.
 */
static uint64_t feistel4(uint64_t seed, uint64_t x, int h)
{
    const uint64_t mask = ((uint64_t)1 << h) - 1;
    uint64_t L = x >> h, R = x & mask;
    for (int r = 0; r < 4; r++) {
        uint64_t f = orc_hash(seed, TAG_PERM, (uint64_t)r, R, 0) & mask;
        uint64_t nl = R, nr = L ^ f;
        L = nl;
        R = nr;
    }
    return (L << h) | R;
}

void orc_hmerge_order(uint64_t seed, int64_t n, int32_t *order)
{
    int h = 1;
    while (((uint64_t)1 << (2 * h)) < (uint64_t)n)
        h++;
    for (int64_t i = 0; i < n; i++) {
        uint64_t x = feistel4(seed, (uint64_t)i, h);
        while (x >= (uint64_t)n)
            x = feistel4(seed, x, h);
        order[i] = (int32_t)x;
    }
}

/* one Feistel pass on 2h-bit values (exposed for tests) */
uint64_t orc_feistel4(uint64_t seed, uint64_t x, int h)
{
    return feistel4(seed, x, h);
}

/* ------------------------------------------------------------------------ */
/* Graph diversification (Algorithm 3, Section 4)                            */
/* ------------------------------------------------------------------------ */

/*
 * Algorithm 3 on one neighbourhood of sample a: cand[0..m) sorted ascending
 * by (distance to a, id); cand[0] is kept; every later candidate s is kept
 * unless some already kept c has m(s, c) < m(s, a) (c occludes s).  The
 * distance to a is the one the list stores (canonical FP32, symmetric);
 * m(s, c) is evaluated canonically.  Kept entries go to out (in order);
 * returns how many.
 */
static int gd_select(const float *X, int d, int metric, const pair_t *cand, int m, pair_t *out)
{
    int q = 0;
    for (int i = 0; i < m; i++) {
        int keep = 1;
        for (int j = 0; j < q && keep; j++) {
            float sc = orc_dist32(metric, X + (int64_t)cand[i].id * d,
                                  X + (int64_t)out[j].id * d, d);
            if (sc < cand[i].dist)
                keep = 0;
        }
        if (keep)
            out[q++] = cand[i];
    }
    return q;
}

/*
 * Diversified graph of G (n rows of k entries over the rows of X, sorted by
 * (distance, id), id -1 = empty).  For each row a (Section 4):
 *   Q_f = Algorithm 3 on a's list;
 *   Q_r = Algorithm 3 on a's reverse list {b : a in G[b]}, each b at the
 *         distance G[b] stores for a, sorted by (distance, id);
 *   out[a] = the max_deg first entries, by (distance, id), of Q_f u Q_r
 *            (an id in both once), padded with (-1, +inf).
 * Reading: the paper merges the two diversified lists and keeps up to k/2
 * neighbours in its experiments; max_deg is that bound.
 */
int orc_diversify(const float *X, int64_t n, int d, int metric, const int32_t *ids,
                  const float *dist, int k, int max_deg, int32_t *out_ids, float *out_dist)
{
    if (n < 1 || d < 1 || k < 1 || max_deg < 1)
        return ORC_EINVAL;
    int64_t *deg = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int rc = ORC_OK;
    pair_t *rev = NULL, *cand = NULL, *qf = NULL, *qr = NULL;
    int64_t *fill = NULL;
    if (!deg) {
        rc = ORC_ENOMEM;
        goto out;
    }
    for (int64_t b = 0; b < n; b++)
        for (int j = 0; j < k; j++) {
            int32_t a = ids[b * k + j];
            if (a < -1 || a >= n || a == b) {
                rc = ORC_EINVAL;
                goto out;
            }
            if (a >= 0)
                deg[a + 1]++;
        }
    for (int64_t a = 0; a < n; a++)
        deg[a + 1] += deg[a];
    rev = (pair_t *)malloc(sizeof(pair_t) * (size_t)(deg[n] > 0 ? deg[n] : 1));
    fill = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    int64_t maxdeg_in = 0;
    for (int64_t a = 0; a < n; a++)
        if (deg[a + 1] - deg[a] > maxdeg_in)
            maxdeg_in = deg[a + 1] - deg[a];
    cand = (pair_t *)malloc(sizeof(pair_t) * (size_t)(maxdeg_in + k + 1));
    qf = (pair_t *)malloc(sizeof(pair_t) * (size_t)(k + 1));
    qr = (pair_t *)malloc(sizeof(pair_t) * (size_t)(maxdeg_in + 1));
    if (!rev || !fill || !cand || !qf || !qr) {
        rc = ORC_ENOMEM;
        goto out;
    }
    for (int64_t b = 0; b < n; b++)
        for (int j = 0; j < k; j++) {
            int32_t a = ids[b * k + j];
            if (a >= 0) {
                pair_t p = {dist[b * k + j], (int32_t)b};
                rev[deg[a] + fill[a]++] = p;
            }
        }
    for (int64_t a = 0; a < n; a++) {
        int m = 0;
        for (int j = 0; j < k; j++)
            if (ids[a * k + j] >= 0) {
                pair_t p = {dist[a * k + j], ids[a * k + j]};
                cand[m++] = p;
            }
        qsort(cand, (size_t)m, sizeof(pair_t), cmp_pair);
        int nf = gd_select(X, d, metric, cand, m, qf);
        int64_t r0 = deg[a], nr_in = deg[a + 1] - deg[a];
        qsort(rev + r0, (size_t)nr_in, sizeof(pair_t), cmp_pair);
        int nr = gd_select(X, d, metric, rev + r0, (int)nr_in, qr);
        /* union, (distance, id) order, each id once, first max_deg */
        int c = 0;
        for (int j = 0; j < nf; j++)
            cand[c++] = qf[j];
        for (int j = 0; j < nr; j++) {
            int dup = 0;
            for (int q = 0; q < nf; q++)
                dup |= qf[q].id == qr[j].id;
            if (!dup)
                cand[c++] = qr[j];
        }
        qsort(cand, (size_t)c, sizeof(pair_t), cmp_pair);
        for (int j = 0; j < max_deg; j++) {
            out_ids[a * max_deg + j] = j < c ? cand[j].id : -1;
            out_dist[a * max_deg + j] = j < c ? cand[j].dist : INFINITY;
        }
    }
out:
    free(deg);
    free(rev);
    free(fill);
    free(cand);
    free(qf);
    free(qr);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* NN search over the graph hierarchy (Section 4)                            */
/* ------------------------------------------------------------------------ */

#define TAG_SEARCH 0xD1u

/*
 * Top-down search of the query q over nl layer graphs.  Layer l holds
 * rows[l] vertices, the rows 0..rows[l]-1 of X (each layer a prefix of the
 * next, the last layer all n rows), and lists of deg[l] ids (-1 = empty).
 *   Stage 1 (layers 0 .. nl-2): start at a random vertex of the top layer,
 *     draw_below(H(seed, SEARCH, query, 0, 0), rows[0]); on each layer move
 *     to the closest, by (distance, id), of the current vertex's neighbours
 *     while it is closer than the current vertex; the vertex reached starts
 *     the next layer.
 *   Stage 2 (bottom layer): a ranked list of at most ef entries (distance,
 *     id), starting with the vertex reached; repeatedly the best entry not
 *     yet expanded is expanded: its neighbours not visited before are
 *     evaluated, marked visited, and the list becomes the ef best of itself
 *     and them; the search ends when every entry of the list is expanded.
 * The answer is the first topk entries (padded with (-1, +inf)).  Distances
 * are canonical FP32 m(q, x).  evals (may be NULL) receives the number of
 * distances evaluated.
 */
static int search_one(const float *X, int d, int metric, const int32_t *const *layer_ids,
                      const int64_t *rows, const int *deg, int nl, const float *q, int64_t qi,
                      int topk, int ef, uint64_t seed, uint8_t *visited, pair_t *pool,
                      uint8_t *expanded, int32_t *out_ids, float *out_dist, int64_t *evals)
{
    uint64_t h = orc_hash(seed, TAG_SEARCH, (uint64_t)qi, 0, 0);
    int32_t cur = (int32_t)draw_below(h, (uint32_t)rows[0]);
    float dcur = orc_dist32(metric, q, X + (int64_t)cur * d, d);
    int64_t ev = 1;
    for (int l = 0; l + 1 < nl; l++) {
        for (;;) {
            int32_t best = -1;
            float dbest = INFINITY;
            for (int j = 0; j < deg[l]; j++) {
                int32_t v = layer_ids[l][(int64_t)cur * deg[l] + j];
                if (v < 0)
                    continue;
                float dv = orc_dist32(metric, q, X + (int64_t)v * d, d);
                ev++;
                if (best < 0 || key_less(dv, v, dbest, best)) {
                    best = v;
                    dbest = dv;
                }
            }
            if (best >= 0 && key_less(dbest, best, dcur, cur)) {
                cur = best;
                dcur = dbest;
            } else {
                break;
            }
        }
    }
    const int b = nl - 1;
    memset(visited, 0, (size_t)rows[b]);
    int cnt = 1;
    pool[0].dist = dcur;
    pool[0].id = cur;
    expanded[0] = 0;
    visited[cur] = 1;
    for (;;) {
        int e = -1;
        for (int j = 0; j < cnt && e < 0; j++)
            if (!expanded[j])
                e = j;
        if (e < 0)
            break;
        expanded[e] = 1;
        int32_t u = pool[e].id;
        for (int j = 0; j < deg[b]; j++) {
            int32_t v = layer_ids[b][(int64_t)u * deg[b] + j];
            if (v < 0 || visited[v])
                continue;
            visited[v] = 1;
            float dv = orc_dist32(metric, q, X + (int64_t)v * d, d);
            ev++;
            /* the pool stays sorted by (distance, id): insert, drop the worst */
            if (cnt == ef && !key_less(dv, v, pool[ef - 1].dist, pool[ef - 1].id))
                continue;
            int pos = cnt < ef ? cnt : ef - 1;
            while (pos > 0 && key_less(dv, v, pool[pos - 1].dist, pool[pos - 1].id)) {
                pool[pos] = pool[pos - 1];
                expanded[pos] = expanded[pos - 1];
                pos--;
            }
            pool[pos].dist = dv;
            pool[pos].id = v;
            expanded[pos] = 0;
            if (cnt < ef)
                cnt++;
        }
    }
    for (int j = 0; j < topk; j++) {
        out_ids[j] = j < cnt ? pool[j].id : -1;
        out_dist[j] = j < cnt ? pool[j].dist : INFINITY;
    }
    if (evals)
        *evals += ev;
    return ORC_OK;
}

int orc_search(const float *X, int d, int metric, const int32_t *const *layer_ids,
               const int64_t *rows, const int *deg, int nl, const float *Q, int64_t nq, int topk,
               int ef, uint64_t seed, int32_t *out_ids, float *out_dist, int64_t *evals)
{
    if (nl < 1 || d < 1 || topk < 1 || ef < topk || nq < 0)
        return ORC_EINVAL;
    for (int l = 0; l < nl; l++)
        if (rows[l] < 1 || deg[l] < 1 || (l > 0 && rows[l] < rows[l - 1]))
            return ORC_EINVAL;
    uint8_t *visited = (uint8_t *)malloc((size_t)rows[nl - 1]);
    pair_t *pool = (pair_t *)malloc(sizeof(pair_t) * (size_t)ef);
    uint8_t *expanded = (uint8_t *)malloc((size_t)ef);
    if (!visited || !pool || !expanded) {
        free(visited);
        free(pool);
        free(expanded);
        return ORC_ENOMEM;
    }
    if (evals)
        *evals = 0;
    for (int64_t i = 0; i < nq; i++)
        search_one(X, d, metric, layer_ids, rows, deg, nl, Q + i * d, i, topk, ef, seed, visited,
                   pool, expanded, out_ids + i * topk, out_dist + i * topk, evals);
    free(visited);
    free(pool);
    free(expanded);
    return ORC_OK;
}
