// knng_search.hip -- graph diversification (Algorithm 3) and the top-down NN
// search over a graph hierarchy (Section 4 of Zhao et al., "On the Merge of
// k-NN Graph").
//
// Diversification of a k-NN graph G over the rows of X, per row a:
//   Q_f = Algorithm 3 on a's list: the first (nearest) entry is kept; each
//         later entry s, in (distance, id) order, is kept unless an already
//         kept c has m(s, c) < m(s, a) (c occludes s);
//   Q_r = Algorithm 3 on a's reverse list {b : a in G[b]}, each b at the
//         distance G[b] stores for a, in (distance, id) order;
//   out[a] = the max_degree first entries, by (distance, id), of Q_f u Q_r,
//         an id present in both taken once (the list's entry).
// m(s, a) is the distance the list stores, m(s, c) the canonical FP32
// distance.  The reverse lists come from two stable radix sorts of the
// edges: by (distance, source), then by target.  One wave per row evaluates
// the occlusion tests of 64 candidates at a time in parallel (every pair of
// the chunk, and every candidate against the entries kept before the chunk),
// then scans the chunk in order.  A reverse list is read only until
// max_degree + |Q_f| of its entries are kept: at least max_degree of those
// are not in Q_f, and every later one is farther than all of them, so it
// cannot enter the first max_degree of the union.
//
// Search over layers 0 (top) .. nl-1 (bottom), layer l a graph over the rows
// 0 .. rows_l - 1 (each layer a prefix of the next): greedy descent on the
// upper layers from a seeded random top vertex, then a best-first search on
// the bottom layer with a ranked list of ef entries; one wave per query.  A
// vertex is evaluated when it is not in the wave's visited filter (an LDS
// hash that stops admitting new vertices when full) and is offered to the
// list only when not already in it: a vertex evaluated before and no longer
// in the list was rejected or dropped by a full list whose worst entry has
// only improved since, so it is rejected again and the list evolves exactly
// as with a complete visited set.
#include <hipcub/hipcub.hpp>

#include "knng_host.h"

using namespace knng;
using namespace knng::host;

namespace knng {
namespace {

constexpr int SW = 4;  // waves per workgroup

__device__ __forceinline__ uint64_t pair_key(float d, int32_t id)
{
    return ((uint64_t)__float_as_uint(d) << 32) | (uint32_t)id;
}
__device__ __forceinline__ int32_t pk_id(uint64_t k) { return (int32_t)(uint32_t)k; }
__device__ __forceinline__ float pk_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }

// ------------------------------------------------------------ reverse lists

// one sort record per list entry: key (distance bits, source), value target;
// empty entries (id -1) get target n, which sorts after every row
__global__ __launch_bounds__(256) void k_rev_records(const int32_t *ids, const float *dist,
                                                     int64_t n, int k, uint64_t *key,
                                                     uint32_t *tgt, uint64_t *ctr)
{
    const int64_t E = n * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < E;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t b = e / k;
        const int32_t a = ids[e];
        const float d = dist[e];
        bool ok = a >= 0;
        if (a < -1 || a >= n) {
            raise_err(ctr + C_ERR, ERR_ID_RANGE);
            ok = false;
        } else if (a == b) {
            raise_err(ctr + C_ERR, ERR_SELF);
            ok = false;
        } else if (ok && !(d >= 0.0f && d < __uint_as_float(0x7F800000u))) {
            raise_err(ctr + C_ERR, ERR_BAD_DIST);
            ok = false;
        }
        key[e] = ok ? pair_key(d, (int32_t)b) : ~0ull;
        tgt[e] = ok ? (uint32_t)a : (uint32_t)n;
    }
}

// off[a] = first sorted record of target a (off[n] = the valid records)
__global__ __launch_bounds__(256) void k_rev_offsets(const uint32_t *tgt, int64_t E, int64_t n,
                                                     int64_t *off)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= E;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = i < E ? (int64_t)tgt[i] : n + 1;
        const int64_t p = i > 0 ? (int64_t)tgt[i - 1] : -1;
        for (int64_t a = p + 1; a <= t && a <= n; a++)
            off[a] = i;
    }
}

// ------------------------------------------------------------ diversification

template <int METRIC>
__device__ __forceinline__ float row_dist(const Rows &R, int32_t p, int32_t q)
{
    float na = 0.0f, nb = 0.0f;
    if (METRIC == M_COS) {
        na = R.norm[p];
        nb = R.norm[q];
    }
    return canon_dist<METRIC>(R.x + (int64_t)p * R.dp, R.x + (int64_t)q * R.dp, R.dp, na, nb);
}

// triangular index t -> (i, j), j < i
__device__ __forceinline__ void tri(int t, int &i, int &j)
{
    i = (int)((1.0f + __builtin_sqrtf(1.0f + 8.0f * (float)t)) * 0.5f);
    while (i * (i - 1) / 2 > t)
        i--;
    while ((i + 1) * i / 2 <= t)
        i++;
    j = t - i * (i - 1) / 2;
}

// Algorithm 3 over m <= 64 candidates in (distance, id) order, held one per
// lane in `cand` (lanes >= m: ~0), after `np` entries kept before them
// (prior[0..np), LDS).  Keeps at most `cap` - np more.  Appends the kept
// candidates, in order, to prior[np..) and returns how many were kept.
template <int METRIC>
__device__ inline int alg3_chunk(const Rows &R, uint64_t cand, int m, uint64_t *prior, int np,
                                 int cap, uint64_t *occ, uint64_t *ckeys)
{
    const int lane = lane_id();
    ckeys[lane] = cand;
    occ[lane] = 0ull;
    __builtin_amdgcn_wave_barrier();
    const int inner = m * (m - 1) / 2, outer = m * np;
    for (int t = lane; t < inner + outer; t += WAVE) {
        int i, j;
        int32_t other;
        if (t < inner) {
            tri(t, i, j);
            other = pk_id(ckeys[j]);
        } else {
            i = (t - inner) / np;
            j = 63;  // a prior entry: bit 63 marks "occluded before the chunk"
            other = pk_id(prior[(t - inner) - i * np]);
        }
        const uint64_t ci = ckeys[i];
        const float sc = row_dist<METRIC>(R, pk_id(ci), other);
        if (sc < pk_dist(ci))
            atomicOr((unsigned long long *)(occ + i), 1ull << j);
    }
    __builtin_amdgcn_wave_barrier();
    // in order: a candidate survives unless occluded by a prior entry or by a
    // candidate kept before it
    uint64_t kept = 0;
    int nk = 0;
    for (int i = 0; i < m && np + nk < cap; i++) {
        const uint64_t o = occ[i];
        if (!(o >> 63) && !(o & kept)) {
            kept |= 1ull << i;
            nk++;
        }
    }
    __builtin_amdgcn_wave_barrier();
    if (lane < m && ((kept >> lane) & 1))
        prior[np + __popcll(kept & ((1ull << lane) - 1ull))] = ckeys[lane];
    __builtin_amdgcn_wave_barrier();
    return nk;
}

template <int METRIC>
__global__ __launch_bounds__(SW *WAVE) void k_diversify(Rows R, const int32_t *ids,
                                                        const float *dist, int k,
                                                        const int64_t *off, const uint64_t *rkey,
                                                        int max_deg, int32_t *out_ids,
                                                        float *out_dist, uint64_t *ctr)
{
    __shared__ uint64_t s_occ[SW][WAVE];
    __shared__ uint64_t s_ck[SW][WAVE];
    __shared__ uint64_t s_qf[SW][MAX_K];
    __shared__ uint64_t s_qr[SW][2 * MAX_K];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    uint64_t *occ = s_occ[w], *ck = s_ck[w], *qf = s_qf[w], *qr = s_qr[w];
    const int64_t nw = (int64_t)gridDim.x * SW;
    for (int64_t a = blockIdx.x * (int64_t)SW + w; a < R.n; a += nw) {
        // forward list: valid entries in their (sorted) order
        int32_t id = -1;
        float dv = 0.0f;
        if (lane < k) {
            id = ids[a * k + lane];
            dv = dist[a * k + lane];
        }
        const bool valid = id >= 0 && id < R.n && id != a;
        const uint64_t vm = __ballot(valid);
        const int m = __popcll(vm);
        // the valid entries in (distance, id) order on the first m lanes
        const uint64_t key0 = valid ? pair_key(dv, id) : ~0ull;
        int rank = 0;
        for (int j = 0; j < WAVE; j++) {
            const uint64_t o = __shfl(key0, j, WAVE);
            rank += o < key0;
        }
        __builtin_amdgcn_wave_barrier();
        if (valid)
            ck[rank] = key0;
        __builtin_amdgcn_wave_barrier();
        const uint64_t key = lane < m ? ck[lane] : ~0ull;
        __builtin_amdgcn_wave_barrier();
        const int nf = alg3_chunk<METRIC>(R, key, m, qf, 0, MAX_K, occ, ck);
        // reverse list, in order, until max_deg of its kept entries are not
        // in Q_f (entries kept after those are farther than all of them and
        // cannot enter the first max_deg of the union)
        const int64_t lo = off[a], hi = off[a + 1];
        const int cap_r = max_deg + nf;
        int nr = 0;
        for (int64_t c0 = lo; c0 < hi && nr < cap_r; c0 += WAVE) {
            const int mm = hi - c0 < WAVE ? (int)(hi - c0) : WAVE;
            uint64_t rk = lane < mm ? rkey[c0 + lane] : ~0ull;
            if (lane < mm && pk_id(rk) >= R.n) {
                raise_err(ctr + C_ERR, ERR_ROW_GROUP);
                rk = ~0ull;
            }
            nr += alg3_chunk<METRIC>(R, rk, mm, qr, nr, cap_r, occ, ck);
        }
        // union: Q_f (lanes < nf), then Q_r minus ids already in Q_f (two
        // entries per lane), placed by their ranks among all of them
        uint64_t e0 = lane < nf ? qf[lane] : ~0ull;
        uint64_t e1[2];
        for (int h = 0; h < 2; h++) {
            const int j = lane + h * WAVE;
            e1[h] = j < nr ? qr[j] : ~0ull;
            if (e1[h] != ~0ull)
                for (int t = 0; t < nf; t++)
                    if (pk_id(qf[t]) == pk_id(e1[h]))
                        e1[h] = ~0ull;
        }
        int r0 = lane, r1[2] = {0, 0};
        for (int j = 0; j < WAVE; j++) {
            const uint64_t o0 = __shfl(e0, j, WAVE);
            const uint64_t oa = __shfl(e1[0], j, WAVE);
            const uint64_t ob = __shfl(e1[1], j, WAVE);
            r0 += (oa < e0) + (ob < e0);
            for (int h = 0; h < 2; h++)
                r1[h] += (o0 < e1[h]) + (oa < e1[h]) + (ob < e1[h]);
        }
        if (lane < max_deg) {
            out_ids[a * max_deg + lane] = -1;
            out_dist[a * max_deg + lane] = __uint_as_float(0x7F800000u);
        }
        __builtin_amdgcn_wave_barrier();
        if (e0 != ~0ull && r0 < max_deg) {
            out_ids[a * max_deg + r0] = pk_id(e0);
            out_dist[a * max_deg + r0] = pk_dist(e0);
        }
        for (int h = 0; h < 2; h++)
            if (e1[h] != ~0ull && r1[h] < max_deg) {
                out_ids[a * max_deg + r1[h]] = pk_id(e1[h]);
                out_dist[a * max_deg + r1[h]] = pk_dist(e1[h]);
            }
    }
}

// ------------------------------------------------------------ search

constexpr int MAX_LAYERS = 32;
constexpr int MAX_EF = 256;
constexpr int VH = 2048;  // visited filter slots per wave
constexpr uint32_t TAG_SEARCH = 0xD1u;

struct Layers {
    const int32_t *ids[MAX_LAYERS];
    int64_t rows[MAX_LAYERS];
    int deg[MAX_LAYERS];
    int nl;
};

// canonical distance of the query (LDS, padded) to row v of R
template <int METRIC>
__device__ __forceinline__ float query_dist(const Rows &R, const float *q, float qn, int32_t v)
{
    const float4 *b4 = reinterpret_cast<const float4 *>(R.x + (int64_t)v * R.dp);
    float acc = 0.0f;
    for (int t = 0; t < R.dp / 4; t++) {
        const float4 y = b4[t];
        acc = canon_step<METRIC>(acc, q[4 * t + 0], y.x);
        acc = canon_step<METRIC>(acc, q[4 * t + 1], y.y);
        acc = canon_step<METRIC>(acc, q[4 * t + 2], y.z);
        acc = canon_step<METRIC>(acc, q[4 * t + 3], y.w);
    }
    return canon_finish<METRIC>(acc, qn, METRIC == M_COS ? R.norm[v] : 0.0f);
}

__device__ __forceinline__ uint32_t vh_hash(uint32_t v) { return (v * 0x9E3779B1u) >> 21; }

template <int METRIC>
__global__ __launch_bounds__(SW *WAVE) void k_search(Rows R, Layers Ls, const float *Qx,
                                                     const float *Qn, int64_t nq, int dq, int topk,
                                                     int ef, uint64_t seed, int32_t *out_ids,
                                                     float *out_dist, uint64_t *ctr)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    const int w = threadIdx.x / WAVE, lane = lane_id();
    // per-wave carve: query (dq floats), pool keys x2, expanded flags x2,
    // candidate keys, visited filter
    const size_t per = (size_t)dq * 4 + 2 * MAX_EF * 8 + 2 * MAX_EF + WAVE * 8 + VH * 4;
    unsigned char *base = dyn + (size_t)w * ((per + 15) / 16 * 16);
    float *q = reinterpret_cast<float *>(base);
    uint64_t *pool[2] = {reinterpret_cast<uint64_t *>(base + (size_t)dq * 4),
                         reinterpret_cast<uint64_t *>(base + (size_t)dq * 4 + MAX_EF * 8)};
    uint8_t *expd[2] = {base + (size_t)dq * 4 + 2 * MAX_EF * 8,
                        base + (size_t)dq * 4 + 2 * MAX_EF * 8 + MAX_EF};
    uint64_t *cks = reinterpret_cast<uint64_t *>(base + (size_t)dq * 4 + 2 * MAX_EF * 8 +
                                                 2 * MAX_EF);
    uint32_t *vis = reinterpret_cast<uint32_t *>(cks + WAVE);
    const int64_t nw = (int64_t)gridDim.x * SW;
    uint64_t n_eval = 0;
    const int top = 0, bot = Ls.nl - 1;
    for (int64_t qi = blockIdx.x * (int64_t)SW + w; qi < nq; qi += nw) {
        for (int t = lane; t < dq; t += WAVE)
            q[t] = Qx[qi * dq + t];
        for (int t = lane; t < VH; t += WAVE)
            vis[t] = 0xFFFFFFFFu;
        const float qn = METRIC == M_COS ? Qn[qi] : 0.0f;
        __builtin_amdgcn_wave_barrier();
        // stage 1: greedy descent on the upper layers
        int32_t cur = (int32_t)draw_below(hash5(seed, TAG_SEARCH, (uint64_t)qi, 0, 0),
                                          (uint32_t)Ls.rows[top]);
        float dcur = query_dist<METRIC>(R, q, qn, cur);
        n_eval += lane == 0;
        for (int l = 0; l < bot; l++) {
            const int deg = Ls.deg[l];
            for (;;) {
                uint64_t best = ~0ull;
                for (int j0 = 0; j0 < deg; j0 += WAVE) {
                    const int32_t v = j0 + lane < deg ? Ls.ids[l][(int64_t)cur * deg + j0 + lane]
                                                      : -1;
                    const bool ok = v >= 0 && v < Ls.rows[l];
                    if (v >= 0 && !ok)
                        raise_err(ctr + C_ERR, ERR_ID_RANGE);
                    uint64_t kk = ~0ull;
                    if (ok) {
                        kk = pair_key(query_dist<METRIC>(R, q, qn, v), v);
                        n_eval++;
                    }
                    for (int o = WAVE / 2; o > 0; o >>= 1) {
                        const uint64_t x = __shfl_xor(kk, o, WAVE);
                        kk = x < kk ? x : kk;
                    }
                    best = kk < best ? kk : best;
                }
                if (best < pair_key(dcur, cur)) {
                    cur = pk_id(best);
                    dcur = pk_dist(best);
                } else {
                    break;
                }
            }
        }
        // stage 2: best-first search on the bottom layer with a ranked list
        const int deg = Ls.deg[bot];
        int cnt = 1, pb = 0;
        if (lane == 0) {
            pool[0][0] = pair_key(dcur, cur);
            expd[0][0] = 0;
            vis[vh_hash((uint32_t)cur) & (VH - 1)] = (uint32_t)cur;
        }
        bool lossy = false;  // the visited filter turned a vertex away
        __builtin_amdgcn_wave_barrier();
        for (;;) {
            // the best entry not yet expanded
            int e = -1;
            for (int j0 = 0; j0 < cnt && e < 0; j0 += WAVE) {
                const uint64_t bm = __ballot(j0 + lane < cnt && !expd[pb][j0 + lane]);
                if (bm)
                    e = j0 + __builtin_ctzll(bm);
            }
            if (e < 0)
                break;
            const int32_t u = pk_id(pool[pb][e]);
            __builtin_amdgcn_wave_barrier();
            if (lane == 0)
                expd[pb][e] = 1;
            for (int j0 = 0; j0 < deg; j0 += WAVE) {
                int32_t v = j0 + lane < deg ? Ls.ids[bot][(int64_t)u * deg + j0 + lane] : -1;
                if (v >= Ls.rows[bot]) {
                    raise_err(ctr + C_ERR, ERR_ID_RANGE);
                    v = -1;
                }
                // visited filter: claim a slot; a vertex found there is skipped
                bool fresh = false;
                if (v >= 0) {
                    uint32_t h = vh_hash((uint32_t)v);
                    fresh = true;
                    for (int p = 0; p < 16; p++) {
                        uint32_t *slot = vis + ((h + p) & (VH - 1));
                        const uint32_t old = atomicCAS(slot, 0xFFFFFFFFu, (uint32_t)v);
                        if (old == 0xFFFFFFFFu)
                            break;
                        if (old == (uint32_t)v) {
                            fresh = false;
                            break;
                        }
                        if (p == 15)
                            lossy = true;  // full neighbourhood of slots: not recorded
                    }
                }
                uint64_t kk = ~0ull;
                if (fresh) {
                    kk = pair_key(query_dist<METRIC>(R, q, qn, v), v);
                    n_eval++;
                }
                // a vertex the filter could not record may already be listed
                if (__ballot(lossy) && kk != ~0ull) {
                    for (int j = 0; j < cnt; j++)
                        if (pk_id(pool[pb][j]) == v)
                            kk = ~0ull;
                }
                // candidates better than the worst of a full list
                const uint64_t worst = cnt == ef ? pool[pb][ef - 1] : ~0ull;
                if (kk >= worst)
                    kk = ~0ull;
                const uint64_t cm = __ballot(kk != ~0ull);
                if (!cm)
                    continue;
                // ranks among the candidates, then merge with the list
                int rc = 0;
                for (int j = 0; j < WAVE; j++) {
                    const uint64_t o = __shfl(kk, j, WAVE);
                    rc += o < kk;
                }
                __builtin_amdgcn_wave_barrier();
                if (kk != ~0ull)
                    cks[rc] = kk;
                __builtin_amdgcn_wave_barrier();
                const int nc = __popcll(cm);
                const int nb = 1 - pb;
                // list entries move down by the candidates before them
                for (int j = lane; j < cnt; j += WAVE) {
                    const uint64_t x = pool[pb][j];
                    int lo = 0, hi = nc;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (cks[mid] < x)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    const int to = j + lo;
                    if (to < ef) {
                        pool[nb][to] = x;
                        expd[nb][to] = expd[pb][j];
                    }
                }
                // candidates move down by the list entries before them
                if (kk != ~0ull) {
                    int lo = 0, hi = cnt;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if (pool[pb][mid] < kk)
                            lo = mid + 1;
                        else
                            hi = mid;
                    }
                    const int to = rc + lo;
                    if (to < ef) {
                        pool[nb][to] = kk;
                        expd[nb][to] = 0;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                cnt = cnt + nc < ef ? cnt + nc : ef;
                pb = nb;
            }
            __builtin_amdgcn_wave_barrier();
        }
        for (int j = lane; j < topk; j += WAVE) {
            const bool has = j < cnt;
            out_ids[qi * topk + j] = has ? pk_id(pool[pb][j]) : -1;
            out_dist[qi * topk + j] = has ? pk_dist(pool[pb][j]) : __uint_as_float(0x7F800000u);
        }
        __builtin_amdgcn_wave_barrier();
    }
    for (int o = WAVE / 2; o > 0; o >>= 1)
        n_eval += __shfl_xor(n_eval, o, WAVE);
    if (lane == 0 && n_eval)
        atomicAdd((unsigned long long *)(ctr + C_EVALS), (unsigned long long)n_eval);
}

inline unsigned grid_of(int64_t items, int per_block, unsigned cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    return (unsigned)(g > cap ? cap : g);
}

size_t search_lds_per_wave(int dq)
{
    const size_t per = (size_t)dq * 4 + 2 * MAX_EF * 8 + 2 * MAX_EF + WAVE * 8 + VH * 4;
    return (per + 15) / 16 * 16;
}

// ------------------------------------------------------------ workspace

struct DivBufs {
    Layout w;
    uint64_t *key[2];
    uint32_t *tgt[2];
    int64_t *off;
    void *sort_tmp;
    size_t sort_bytes;
};

size_t radix_tmp_bytes(int64_t E)
{
    size_t a = 0, b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t *)nullptr,
                                             (uint64_t *)nullptr, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (int64_t)E);
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint32_t *)nullptr,
                                             (uint32_t *)nullptr, (const uint64_t *)nullptr,
                                             (uint64_t *)nullptr, (int64_t)E);
    return a > b ? a : b;
}

void carve_div(Carve &c, DivBufs &b, int64_t n, int d, int k, knng_metric m)
{
    b.w = Layout{};
    b.w.dp = pad4(d);
    b.w.ctr = c.take<uint64_t>(C_WORDS);
    b.w.x = c.take<float>((size_t)n * b.w.dp);
    b.w.norm = m == KNNG_COSINE ? c.take<float>(n) : nullptr;
    const int64_t E = n * k;
    for (int i = 0; i < 2; i++) {
        b.key[i] = c.take<uint64_t>((size_t)(E > 0 ? E : 1));
        b.tgt[i] = c.take<uint32_t>((size_t)(E > 0 ? E : 1));
    }
    b.off = c.take<int64_t>((size_t)n + 1);
    b.sort_bytes = radix_tmp_bytes(E) + 256;
    b.sort_tmp = c.take<uint8_t>(b.sort_bytes);
}

int bits_for(int64_t v)
{
    int b = 1;
    while (b < 63 && ((int64_t)1 << b) <= v)
        b++;
    return b;
}

} // namespace
} // namespace knng

extern "C" {

size_t knng_diversify_workspace_size(int64_t n, int32_t d, int32_t k, knng_metric metric)
{
    if (n < 1 || d < 1 || k < 1)
        return 0;
    try {
        Carve c(nullptr);
        DivBufs b;
        carve_div(c, b, n, d, k, metric);
        return c.off + 256;
    } catch (...) {
        return 0;
    }
}

static knng_status knng_diversify_impl(const knng_set *X, const knng_graph *G, int32_t max_degree,
                                       knng_metric metric, knng_graph *out, void *workspace,
                                       size_t workspace_bytes, void *stream)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(X, "X")))
        return s;
    const int64_t n = X->n;
    if (!G || G->n != n || G->k < 1 || G->k > MAX_K)
        return fail(KNNG_EINVAL, "G must hold n = %lld rows of 1..64 entries", (long long)n);
    if (!G->dist || !is_device_ptr(G->ids) || !is_device_ptr(G->dist))
        return fail(KNNG_EINVAL, "G->ids and G->dist must be device memory");
    if (max_degree < 1 || max_degree > MAX_K)
        return fail(KNNG_EINVAL, "max_degree = %d not in [1, 64]", max_degree);
    if ((s = check_out(out, n, max_degree)))
        return s;
    const size_t need = knng_diversify_workspace_size(n, X->d, G->k, metric);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    DivBufs b;
    carve_div(c, b, n, X->d, G->k, metric);
    knng_set none{0, X->d, nullptr};
    Rows R;
    s = prepare(&none, nullptr, X, nullptr, metric, false, b.w, 0, n, st, R);
    if (s != KNNG_OK)
        return s;
    const int64_t E = n * G->k;
    hipLaunchKernelGGL(k_rev_records, dim3(grid_of(E, 256, 1u << 16)), dim3(256), 0, st, G->ids,
                       G->dist, n, G->k, b.key[0], b.tgt[0], b.w.ctr);
    HIP_TRY(hipGetLastError());
    size_t tb = b.sort_bytes;
    HIP_TRY(hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tb, b.key[0], b.key[1], b.tgt[0],
                                               b.tgt[1], E, 0, 64, st));
    tb = b.sort_bytes;
    HIP_TRY(hipcub::DeviceRadixSort::SortPairs(b.sort_tmp, tb, b.tgt[1], b.tgt[0], b.key[1],
                                               b.key[0], E, 0, bits_for(n), st));
    hipLaunchKernelGGL(k_rev_offsets, dim3(grid_of(E + 1, 256, 1u << 16)), dim3(256), 0, st,
                       b.tgt[0], E, n, b.off);
    HIP_TRY(hipGetLastError());
    uint64_t h[C_WORDS];
    s = read_ctr(b.w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EINVAL, "%s", err_text(h[C_ERR]));
    const unsigned grid = grid_of(n, SW, 16384);
    if (metric == KNNG_L2)
        hipLaunchKernelGGL(k_diversify<M_L2>, dim3(grid), dim3(SW * WAVE), 0, st, R, G->ids,
                           G->dist, G->k, b.off, b.key[0], max_degree, out->ids, out->dist,
                           b.w.ctr);
    else if (metric == KNNG_COSINE)
        hipLaunchKernelGGL(k_diversify<M_COS>, dim3(grid), dim3(SW * WAVE), 0, st, R, G->ids,
                           G->dist, G->k, b.off, b.key[0], max_degree, out->ids, out->dist,
                           b.w.ctr);
    else
        hipLaunchKernelGGL(k_diversify<M_L1>, dim3(grid), dim3(SW * WAVE), 0, st, R, G->ids,
                           G->dist, G->k, b.off, b.key[0], max_degree, out->ids, out->dist,
                           b.w.ctr);
    HIP_TRY(hipGetLastError());
    s = read_ctr(b.w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EDEVICE, "%s", err_text(h[C_ERR]));
    return ok();
}

knng_status knng_diversify(const knng_set *X, const knng_graph *G, int32_t max_degree,
                           knng_metric metric, knng_graph *out, void *workspace,
                           size_t workspace_bytes, void *stream)
{
    try {
        return knng_diversify_impl(X, G, max_degree, metric, out, workspace, workspace_bytes,
                                   stream);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

size_t knng_search_workspace_size(int64_t n, int32_t d, int64_t nq, knng_metric metric)
{
    if (n < 1 || d < 1 || nq < 0)
        return 0;
    Carve c(nullptr);
    c.take<uint64_t>(C_WORDS);
    c.take<float>((size_t)n * pad4(d));
    if (metric == KNNG_COSINE)
        c.take<float>(n);
    c.take<float>((size_t)(nq > 0 ? nq : 1) * pad4(d));
    if (metric == KNNG_COSINE)
        c.take<float>((size_t)(nq > 0 ? nq : 1));
    return c.off + 256;
}

static knng_status knng_search_impl(const knng_set *X, const knng_graph *layers, int32_t nlayers,
                                    const knng_set *Q, int32_t topk, int32_t ef, uint64_t seed,
                                    knng_metric metric, int32_t *out_ids, float *out_dist,
                                    void *workspace, size_t workspace_bytes, void *stream,
                                    int64_t *evals)
{
    knng_status s;
    if ((s = check_metric(metric)) || (s = check_set(X, "X")) || (s = check_set(Q, "Q", true)))
        return s;
    if (Q->n > 0 && Q->d != X->d)
        return fail(KNNG_EINVAL, "Q->d = %d differs from X->d = %d", Q->d, X->d);
    if (!layers || nlayers < 1 || nlayers > MAX_LAYERS)
        return fail(KNNG_EINVAL, "nlayers = %d not in [1, %d]", nlayers, MAX_LAYERS);
    if (topk < 1 || ef < topk || ef > MAX_EF)
        return fail(KNNG_EINVAL, "need 1 <= topk <= ef <= %d (topk %d, ef %d)", MAX_EF, topk, ef);
    Layers Ls{};
    Ls.nl = nlayers;
    for (int l = 0; l < nlayers; l++) {
        const knng_graph &g = layers[l];
        if (g.n < 1 || g.k < 1 || g.k > 4 * MAX_K || g.n > X->n || (l && g.n < layers[l - 1].n))
            return fail(KNNG_EINVAL, "layer %d: %lld x %d (layers must be prefixes of X, growing)",
                        l, (long long)g.n, g.k);
        if (!is_device_ptr(g.ids))
            return fail(KNNG_EINVAL, "layer %d ids are not device memory", l);
        Ls.ids[l] = g.ids;
        Ls.rows[l] = g.n;
        Ls.deg[l] = g.k;
    }
    const int64_t nq = Q->n;
    if (nq > 0 && (!is_device_ptr(out_ids) || !is_device_ptr(out_dist)))
        return fail(KNNG_EINVAL, "out_ids / out_dist must be device memory");
    const size_t need = knng_search_workspace_size(X->n, X->d, nq, metric);
    if (!workspace || workspace_bytes < need)
        return fail(KNNG_ENOMEM, "workspace %zu bytes, need %zu", workspace_bytes, need);
    if (!is_device_ptr(workspace))
        return fail(KNNG_EINVAL, "workspace is not device memory");
    hipStream_t st = (hipStream_t)stream;
    Carve c(workspace);
    Layout w{};
    w.dp = pad4(X->d);
    w.ctr = c.take<uint64_t>(C_WORDS);
    w.x = c.take<float>((size_t)X->n * w.dp);
    w.norm = metric == KNNG_COSINE ? c.take<float>(X->n) : nullptr;
    float *qx = c.take<float>((size_t)(nq > 0 ? nq : 1) * w.dp);
    float *qn = metric == KNNG_COSINE ? c.take<float>((size_t)(nq > 0 ? nq : 1)) : nullptr;
    knng_set none{0, X->d, nullptr};
    Rows R;
    s = prepare(&none, nullptr, X, nullptr, metric, false, w, 0, X->n, st, R);
    if (s != KNNG_OK)
        return s;
    if (nq > 0) {
        HIP_TRY(launch_pack(nullptr, 0, Q->x, nq, Q->d, w.dp, qx, 0, nullptr, nullptr, 1, w.ctr,
                            st));
        if (qn)
            HIP_TRY(launch_norms(qx, nq, w.dp, qn, 1, w.ctr, st));
        const size_t lds = search_lds_per_wave(w.dp) * SW;
        const unsigned grid = grid_of(nq, SW, 8192);
        auto go = [&](auto kern) -> hipError_t {
            if (lds > 48 * 1024) {
                hipError_t e = hipFuncSetAttribute((const void *)kern,
                                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                                   (int)lds);
                if (e != hipSuccess)
                    return e;
            }
            hipLaunchKernelGGL(kern, dim3(grid), dim3(SW * WAVE), lds, st, R, Ls, qx, qn, nq,
                               w.dp, topk, ef, seed, out_ids, out_dist, w.ctr);
            return hipGetLastError();
        };
        if (lds > 160 * 1024)
            return fail(KNNG_EINVAL, "d = %d is too large for the search's LDS", X->d);
        if (metric == KNNG_L2)
            HIP_TRY(go(k_search<M_L2>));
        else if (metric == KNNG_COSINE)
            HIP_TRY(go(k_search<M_COS>));
        else
            HIP_TRY(go(k_search<M_L1>));
    }
    uint64_t h[C_WORDS];
    s = read_ctr(w.ctr, h, st);
    if (s != KNNG_OK)
        return s;
    if (h[C_ERR])
        return fail(KNNG_EINVAL, "%s", err_text(h[C_ERR]));
    if (evals)
        *evals = (int64_t)h[C_EVALS];
    return ok();
}

knng_status knng_search(const knng_set *X, const knng_graph *layers, int32_t nlayers,
                        const knng_set *Q, int32_t topk, int32_t ef, uint64_t seed,
                        knng_metric metric, int32_t *out_ids, float *out_dist, void *workspace,
                        size_t workspace_bytes, void *stream, int64_t *evals)
{
    try {
        return knng_search_impl(X, layers, nlayers, Q, topk, ef, seed, metric, out_ids, out_dist,
                                workspace, workspace_bytes, stream, evals);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

} // extern "C"
