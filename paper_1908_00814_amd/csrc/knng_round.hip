// knng_round.hip -- per-round sampling and Reverse(G) of the repeat loop of
// Algorithms 1 and 2 (Zhao et al., Sections 3.1-3.2).  The paper runs the
// NN-Descent iteration by citation; its sampling is realised as:
//   forward: each row takes up to s NEW entries with the smallest hash
//            priority as its NEW sample and marks them OLD; entries that were
//            OLD before form its OLD sample;
//   reverse: every sampled edge u -> v offers u to v's reverse NEW (or OLD)
//            list, which keeps the s offers of smallest hash priority.
// Both selections are order-independent, so the result does not depend on
// thread scheduling.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

// Rows are visited wave-strided (row u by wave u mod W), 64 candidate rows at
// a time: one tag load per lane and a ballot pick the rows to work on.
#define FOR_TAGGED_ROWS(u, n, tagarr, want)                                                   \
    const int64_t nwaves_ = (int64_t)gridDim.x * (blockDim.x / WAVE);                        \
    const int64_t wave0_ = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;          \
    for (int64_t b_ = wave0_; b_ < (n); b_ += nwaves_ * WAVE)                                 \
        for (uint64_t todo_ = __ballot(b_ + (int64_t)lane_id() * nwaves_ < (n) &&            \
                                       (tagarr)[b_ + (int64_t)lane_id() * nwaves_] == (want)); \
             todo_; todo_ &= todo_ - 1)                                                       \
            if (const int64_t u = b_ + (int64_t)__builtin_ctzll(todo_) * nwaves_; true)

// Forward sample of round t over the rows holding NEW entries (dtag == t), one
// wave per row (k <= 64 lanes).  Marks u and every sampled NEW entry as
// active in round t; a row left with more than s NEW entries is sampled
// again in round t+1.  The FRESH count of round t-1 is accumulated per wave.
__global__ __launch_bounds__(256) void k_sample(RoundArgs a)
{
    const int lane = lane_id();
    int fresh_total = 0;
    FOR_TAGGED_ROWS(u, a.n, a.dtag, a.round)
    {
        const bool act = lane < a.k;
        uint64_t v = act ? a.L[u * a.k + lane] : ~0ull;
        const bool empty = !act || key_empty(v);
        const bool fresh = !empty && (v & F_FRESH);
        const bool isnew = !empty && (v & F_NEW);
        const bool isold = !empty && !(v & F_NEW);
        const uint32_t id = key_id(v);
        uint64_t pk = ~0ull;
        if (isnew) {
            uint64_t h = hash5(a.seed, TAG_FWD, (uint64_t)a.round, (uint64_t)u, (uint64_t)id);
            pk = ((h >> 32) << 32) | id;
        }
        // rank among the NEW entries (ties, which a well-formed list never
        // has, go by slot so that the sample slots stay a permutation)
        int rank = 0, nnew = 0;
        for (int j = 0; j < a.k; j++) {
            uint64_t o = __shfl(pk, j, WAVE);
            rank += o < pk || (o == pk && j < lane);
            nnew += o != ~0ull;
        }
        const bool sampled = isnew && rank < a.s;
        if (sampled) {
            a.new_f[u * a.s + rank] = (int32_t)id;
            if (id < a.n)
                a.atag[id] = a.round;
            else
                raise_err(a.ctr + C_ERR, ERR_ROW_SAMPLE);
        }
        uint64_t nv = v & ~(uint64_t)F_FRESH;
        if (sampled)
            nv &= ~(uint64_t)F_NEW;
        if (act && !empty && nv != v)
            a.L[u * a.k + lane] = nv;
        const uint64_t below = (1ull << lane) - 1ull;
        const uint64_t om = __ballot(isold);
        if (isold)
            a.old_f[u * a.k + __popcll(om & below)] = (int32_t)id;
        uint64_t wv = act ? (empty ? v : key_strip(nv)) : 0ull;
        wv = wave_max_u64(wv);
        fresh_total += wave_sum((int)fresh);
        if (lane == 0) {
            a.worst[u] = wv;
            a.cnt_f[2 * u] = nnew < a.s ? nnew : a.s;
            a.cnt_f[2 * u + 1] = __popcll(om);
            if (nnew > 0)
                a.atag[u] = a.round;
            if (nnew > a.s)
                a.dtag[u] = a.round + 1;
        }
    }
    if (lane == 0 && fresh_total)
        atomicAdd((unsigned long long *)(a.ctr + C_FRESH), (unsigned long long)fresh_total);
}

// Rows active in round t: empty reverse reservoirs; a row that was not
// sampled (all its entries OLD) takes its whole list as its OLD sample.
__global__ __launch_bounds__(256) void k_prep_active(RoundArgs a)
{
    const int lane = lane_id();
    FOR_TAGGED_ROWS(u, a.n, a.atag, a.round)
    {
        if (lane < a.s) {
            a.rnew[u * a.s + lane] = empty_key(lane);
            a.rold[u * a.s + lane] = empty_key(lane);
        }
        if (lane < 2)
            a.rfill[2 * u + lane] = 0;
        if (a.dtag[u] < a.round) {
            const uint64_t v = lane < a.k ? a.L[u * a.k + lane] : ~0ull;
            const bool has = lane < a.k && !key_empty(v);
            const uint64_t m = __ballot(has);
            if (has)
                a.old_f[u * a.k + __popcll(m & ((1ull << lane) - 1ull))] = (int32_t)key_id(v);
            if (lane == 0) {
                a.cnt_f[2 * u] = 0;
                a.cnt_f[2 * u + 1] = __popcll(m);
            }
        }
    }
}

// Reverse(G) of round t, one thread per (row u, slot): a sampled edge u -> v
// offers u to v's reverse list of its kind.  NEW edges come from the rows
// sampled this round (their targets are active by construction); OLD edges
// from every row (a row not sampled this round has only OLD entries) and
// are kept only for active targets, the only rows whose neighbourhood is
// joined.
__global__ __launch_bounds__(256) void k_reverse(RoundArgs a)
{
    const int per = a.s + a.k;
    const int64_t total = a.n * per;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t u = e / per;
        int j = (int)(e - u * per);
        const bool sampled = a.dtag[u] >= a.round;
        int32_t v;
        uint32_t tag;
        uint64_t *res;
        int kind;
        if (j < a.s) {
            if (!sampled || j >= a.cnt_f[2 * u])
                continue;
            v = a.new_f[u * a.s + j];
            if (v < 0 || v >= a.n) {
                raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
                continue;
            }
            tag = TAG_RNEW;
            res = a.rnew;
            kind = 0;
        } else {
            j -= a.s;
            if (sampled) {
                if (j >= a.cnt_f[2 * u + 1])
                    continue;
                v = a.old_f[u * a.k + j];
            } else {
                const uint64_t w = a.L[u * a.k + j];
                if (key_empty(w))
                    continue;
                v = (int32_t)key_id(w);
            }
            if (v < 0 || v >= a.n) {
                raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
                continue;
            }
            if (a.atag[v] != a.round)
                continue;
            tag = TAG_ROLD;
            res = a.rold;
            kind = 1;
        }
        uint64_t h = hash5(a.seed, tag, (uint64_t)a.round, (uint64_t)v, (uint64_t)u);
        uint64_t key = ((h >> 32) << 32) | (uint64_t)u;
        uint64_t *slots = res + (int64_t)v * a.s;
        // the first s offers take a slot of their own (every slot change is a
        // compare-and-swap to a smaller word, as in bounded_insert, so a slot
        // that a competing insert has taken sends this offer the long way)
        const int pos = atomicAdd(a.rfill + 2 * (int64_t)v + kind, 1);
        if (pos < a.s && cas64(slots + pos, empty_key(pos), key))
            continue;
        bounded_insert<MAX_S>(slots, a.s, key, false, nullptr, a.ctr + C_ERR);
    }
}

// count the FRESH entries left by the last round (statistics only)
__global__ __launch_bounds__(256) void k_count_fresh(RoundArgs a)
{
    const int64_t total = a.n * a.k;
    int c = 0;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint64_t v = a.L[e];
        c += !key_empty(v) && (v & F_FRESH);
    }
    c = wave_sum(c);
    if (lane_id() == 0 && c)
        atomicAdd((unsigned long long *)(a.ctr + C_FRESH), (unsigned long long)c);
}

inline unsigned grid_for(int64_t items, int per_block, unsigned cap)
{
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1)
        g = 1;
    return (unsigned)(g > cap ? cap : g);
}

} // namespace

hipError_t launch_sample(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_sample, dim3(grid_for(a.n, 4, 8192)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_prep_active(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_prep_active, dim3(grid_for(a.n, 4, 8192)), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reverse(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_reverse, dim3(grid_for(a.n * (a.s + a.k), 256, 1u << 20)), dim3(256),
                       0, st, a);
    return hipGetLastError();
}

hipError_t launch_count_fresh(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_fresh, dim3(grid_for(a.n * a.k, 256, 16384)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

} // namespace knng
