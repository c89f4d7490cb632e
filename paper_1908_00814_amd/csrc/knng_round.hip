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

// Forward sample of round t over the rows holding NEW entries (dtag == t), one
// group of G lanes per row (k <= G), 64 / G rows per wave.  The sample is the s
// NEW entries of smallest hash priority (all of them when there are at most
// s; where they go in the sample slots does not matter).  Marks u and every
// sampled NEW entry as active in round t; a row left with more than s NEW
// entries is sampled again in round t+1.  The FRESH count of round t-1 is
// accumulated per wave.
template <int G>
__global__ __launch_bounds__(256) void k_sample(RoundArgs a)
{
    // graph mode: round max_rounds only counts the last round's entries
    // (k_count_fresh), as the host-driven loop does
    if (!take_round(a) || (a.dev && a.round >= a.dev->max_rounds))
        return;
    constexpr int RPW = WAVE / G;  // rows per wave step
    const int lane = lane_id();
    const int grp = lane / G, gl = lane % G, base = grp * G;
    const uint64_t gbits = G == WAVE ? ~0ull : ((1ull << G) - 1ull) << base;
    const uint64_t below = (1ull << lane) - 1ull;
    const int32_t tr = a.tag0 + a.round;
    int fresh_total = 0;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const int64_t wave0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    for (int64_t b = wave0; b < a.n; b += nwaves * WAVE) {
        const int64_t r0 = b + (int64_t)lane * nwaves;
        uint64_t todo = __ballot(r0 < a.n && a.dtag[r0] == tr);
        while (todo) {
            // the next RPW tagged rows, one per group
            int64_t u = -1;
#pragma unroll
            for (int q = 0; q < RPW; q++) {
                if (todo) {
                    if (grp == q)
                        u = b + (int64_t)__builtin_ctzll(todo) * nwaves;
                    todo &= todo - 1;
                }
            }
            const bool act = u >= 0 && gl < a.k;
            uint64_t v = act ? a.L[u * a.k + gl] : ~0ull;
            const bool empty = !act || key_empty(v);
            const bool fresh = !empty && (v & F_FRESH);
            const bool isnew = !empty && (v & F_NEW);
            const bool isold = !empty && !(v & F_NEW);
            const uint32_t id = key_id(v);
            // a row with at most s NEW entries samples them all, in slot order;
            // a row with more ranks them by hash priority (ties, which a
            // well-formed list never has, go by slot so that the sample slots
            // stay a permutation) and samples the s first
            const uint64_t nm = __ballot(isnew) & gbits;
            const int nnew = __popcll(nm);
            int rank = __popcll(nm & below);
            if (__ballot(nnew > a.s) != 0ull) {
                uint64_t pk = ~0ull;
                if (isnew && nnew > a.s) {
                    uint64_t h =
                        hash5(a.seed, TAG_FWD, (uint64_t)a.round, (uint64_t)u, (uint64_t)id);
                    pk = ((h >> 32) << 32) | id;
                }
                int rk = 0;
                for (int j = 0; j < a.k; j++) {
                    uint64_t o = __shfl(pk, base + j, WAVE);
                    rk += o < pk || (o == pk && j < gl);
                }
                if (nnew > a.s)
                    rank = rk;
            }
            const bool sampled = isnew && rank < a.s;
            bool mark = false;  // the sampled id becomes active
            if (sampled) {
                a.new_f[u * a.s + rank] = (int32_t)id;
                if (id < a.n)
                    mark = true;
                else
                    raise_err(a.ctr + C_ERR, ERR_ROW_SAMPLE);
            }
            uint64_t nv = v & ~(uint64_t)F_FRESH;
            if (sampled)
                nv &= ~(uint64_t)F_NEW;
            if (act && !empty && nv != v)
                a.L[u * a.k + gl] = nv;
            const uint64_t om = __ballot(isold) & gbits;
            if (isold)
                a.old_f[u * a.k + __popcll(om & below)] = (int32_t)id;
            uint64_t wv = act ? (empty ? v : key_strip(nv)) : 0ull;
            for (int o = G / 2; o > 0; o >>= 1) {
                const uint64_t w = __shfl_xor(wv, o, WAVE);
                wv = w > wv ? w : wv;
            }
            fresh_total += wave_sum((int)fresh);
            if (u >= 0 && gl == 0) {
                a.worst[u * a.ws] = wv;
                a.cnt_f[2 * u] = nnew < a.s ? nnew : a.s;
                a.cnt_f[2 * u + 1] = __popcll(om);
                if (nnew > a.s)
                    a.dtag[u] = tr + 1;
            }
            const bool mark_u = u >= 0 && gl == 0 && nnew > 0;  // u itself is active
            if (!a.alist) {
                if (mark)
                    a.atag[id] = tr;
                if (mark_u)
                    a.atag[u] = tr;
            } else {
                // the first mark of a row in this round appends it to the list
                const bool fm = mark && atomicExch(a.atag + id, tr) != tr;
                const bool fu = mark_u && atomicExch(a.atag + u, tr) != tr;
                const uint64_t m1 = __ballot(fm), m2 = __ballot(fu);
                const int cnt = __popcll(m1) + __popcll(m2);
                if (cnt) {
                    unsigned long long bs = 0;
                    if (lane == 0)
                        bs = atomicAdd((unsigned long long *)(a.ctr + C_ACTIVE),
                                       (unsigned long long)cnt);
                    bs = __shfl(bs, 0, WAVE);
                    if (fm)
                        a.alist[bs + __popcll(m1 & below)] = (int32_t)id;
                    if (fu)
                        a.alist[bs + __popcll(m1) + __popcll(m2 & below)] = (int32_t)u;
                }
            }
        }
    }
    if (lane == 0 && fresh_total)
        atomicAdd((unsigned long long *)(a.ctr + C_FRESH), (unsigned long long)fresh_total);
}

// Rows active in round t: empty reverse reservoirs; a row that was not
// sampled (all its entries OLD) takes its whole list as its OLD sample.
__global__ __launch_bounds__(256) void k_prep_active(RoundArgs a)
{
    if (!take_round(a))
        return;
    const int lane = lane_id();
    const int32_t tr = a.tag0 + a.round;
    FOR_ACTIVE_ROWS(u, a, tr)
    {
        if (lane < a.s) {
            a.rnew[u * a.s + lane] = empty_key(lane);
            a.rold[u * a.s + lane] = empty_key(lane);
        }
        if (lane < 2)
            a.rfill[2 * u + lane] = 0;
        if (a.dtag[u] < tr) {
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

// An offer past the s-th to a reservoir: every slot has been claimed by an
// earlier offer, whose store may still be on its way.  The offer reads the
// slots again until none is empty (a claimed slot is written once, by a wave
// already past its claim, so the wait ends), then replaces the largest word
// if it is smaller (compare-and-swap, as in bounded_insert: a failed swap
// reads the slots again).  A word read through the caches is the slot's
// current one or an older, larger one.
__device__ inline void reservoir_overflow(uint64_t *slots, int cap, uint64_t key, uint64_t *err)
{
    constexpr int B = MAX_S <= 16 ? MAX_S : (MAX_S == 32 ? 20 : 16);
    for (int spin = 0; spin < SPIN_BUDGET; spin++) {
        uint64_t mx = 0;
        int mj = 0;
        bool pend = false;
        for (int j0 = 0; j0 < cap; j0 += B) {
            uint64_t v[B];
#pragma unroll
            for (int j = 0; j < B; j++)
                v[j] = j0 + j < cap ? (spin == 0 ? slots[j0 + j] : ld_agent(slots + j0 + j))
                                    : 0ull;
#pragma unroll
            for (int j = 0; j < B; j++) {
                // an empty slot's id field is above every row id
                pend |= (uint32_t)v[j] >= 0x40000000u;
                if (v[j] > mx) {
                    mx = v[j];
                    mj = j0 + j;
                }
            }
        }
        if (pend)
            continue;
        if (key >= mx || cas64(slots + mj, mx, key))
            return;
    }
    atomicOr((unsigned long long *)err, (unsigned long long)ERR_SPIN);
}

// u offered to v's reverse reservoir of one kind (0: NEW, 1: OLD), which
// keeps the s offers of smallest hash priority.  The first s offers claim a
// slot each and store their word there (an agent-scope store, which the
// agent-scope reads of other waves see; nothing else writes an empty slot),
// the others go through reservoir_overflow.
__device__ inline void offer_reverse(const RoundArgs &a, int64_t v, int64_t u, int kind)
{
    const uint64_t h = hash5(a.seed, kind ? TAG_ROLD : TAG_RNEW, (uint64_t)a.round, (uint64_t)v,
                             (uint64_t)u);
    const uint64_t key = ((h >> 32) << 32) | (uint64_t)u;
    uint64_t *slots = (kind ? a.rold : a.rnew) + v * a.s;
    const int pos = atomicAdd(a.rfill + 2 * v + kind, 1);
    if (pos < a.s)
        __hip_atomic_store(slots + pos, key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // a claimed slot that an overflow offer waits for may be this wave's own:
    // the ballot (which every active lane reaches) keeps the claims' writes
    // ahead of the overflow loop in the wave's instruction stream
    if (__ballot(pos >= a.s) != 0ull && pos >= a.s)
        reservoir_overflow(slots, a.s, key, a.ctr + C_ERR);
}

// Reverse(G) of round t, one thread per (row u, slot): a sampled edge u -> v
// offers u to v's reverse list of its kind.  NEW edges come from the rows
// sampled this round (their targets are active by construction); OLD edges
// from every row (a row not sampled this round has only OLD entries) and
// are kept only for active targets, the only rows whose neighbourhood is
// joined.
__global__ __launch_bounds__(256) void k_reverse(RoundArgs a)
{
    if (!take_round(a))
        return;
    const int per = a.s + a.k;
    const int64_t total = a.n * per;
    const int32_t tr = a.tag0 + a.round;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        int64_t u = e / per;
        int j = (int)(e - u * per);
        const bool sampled = a.dtag[u] >= tr;
        int32_t v;
        int kind;
        if (j < a.s) {
            if (!sampled || j >= a.cnt_f[2 * u])
                continue;
            v = a.new_f[u * a.s + j];
            if (v < 0 || v >= a.n) {
                raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
                continue;
            }
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
            if (a.atag[v] != tr)
                continue;
            kind = 1;
        }
        offer_reverse(a, v, u, kind);
    }
}

// Reverse(G) with a reverse index of the initial lists, part 1: the rows that
// may differ from their initial list (dtag >= tag0: rows with appended or
// initialised entries, and every row an insert has reached), one wave per
// row, edges as in k_reverse.
__global__ __launch_bounds__(256) void k_reverse_rows(RoundArgs a)
{
    if (!take_round(a))
        return;
    const int lane = lane_id();
    const int32_t *dtag = a.dtag;
    const int32_t tag0 = a.tag0, tr = a.tag0 + a.round;
    FOR_ROWS_IF(u, a.n, [&](int64_t r) { return dtag[r] >= tag0; })
    {
        const bool sampled = dtag[u] >= tr;
        const int nn = sampled ? a.cnt_f[2 * u] : 0;
        const int no = sampled ? a.cnt_f[2 * u + 1] : a.k;
        for (int j = lane; j < nn; j += WAVE) {
            const int32_t v = a.new_f[u * a.s + j];
            if (v < 0 || v >= a.n)
                raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
            else
                offer_reverse(a, v, u, 0);
        }
        for (int j = lane; j < no; j += WAVE) {
            int32_t v;
            if (sampled) {
                v = a.old_f[u * a.k + j];
            } else {
                const uint64_t w = a.L[u * a.k + j];
                if (key_empty(w))
                    continue;
                v = (int32_t)key_id(w);
            }
            if (v < 0 || v >= a.n)
                raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
            else if (a.atag[v] == tr)
                offer_reverse(a, v, u, 1);
        }
    }
}

// Part 2, launched first: rows that still hold their initial list (dtag < tag0,
// never sampled, all entries OLD) offer themselves to the active targets their
// list holds, found through the index.  One wave per active target v < rev_m
// is the only writer of v's OLD reservoir while this kernel runs (k_prep_active
// has just emptied it), so the wave keeps the s offers of smallest priority
// itself and stores them, with no atomics; rfill counts every offer made, so
// that part 1's offers that follow take free slots or go through
// reservoir_overflow.
__global__ __launch_bounds__(256) void k_reverse_base(RoundArgs a)
{
    __shared__ uint64_t keep_all[256 / WAVE][MAX_S];
    if (!take_round(a))
        return;
    const int lane = lane_id();
    uint64_t *keep = keep_all[threadIdx.x / WAVE];
    const int32_t tr = a.tag0 + a.round;
    FOR_ACTIVE_ROWS(v, a, tr)
    {
        if (v >= a.rev_m)
            continue;  // rows past the base have no base sources
        const int64_t lo = a.rev_off[v], hi = a.rev_off[v + 1];
        uint64_t best = ~0ull;  // lane j < nkept: the offer of rank j so far
        int nkept = 0, offers = 0;
        for (int64_t b = lo; b < hi; b += WAVE) {
            const int64_t i = b + lane;
            uint64_t key = ~0ull;
            if (i < hi) {
                const int32_t u = a.rev_src[i];
                if (u < 0 || u >= a.rev_m) {
                    raise_err(a.ctr + C_ERR, ERR_ROW_REVERSE);
                } else if (a.dtag[u] < a.tag0) {
                    const uint64_t h = hash5(a.seed, TAG_ROLD, (uint64_t)a.round, (uint64_t)v,
                                             (uint64_t)u);
                    key = ((h >> 32) << 32) | (uint64_t)u;
                }
            }
            const uint64_t has = __ballot(key != ~0ull);
            offers += __popcll(has);
            const uint64_t thr = nkept == a.s ? __shfl(best, a.s - 1, WAVE) : ~0ull;
            if (!__ballot(key < thr))
                continue;
            // ranks in the union of the kept offers and this chunk's (all
            // distinct: the sources of one target are distinct rows)
            int rk = 0, rb = 0;
            for (int j = 0; j < WAVE; j++) {
                const uint64_t o = __shfl(key, j, WAVE);
                rk += o < key;
                rb += o < best;
            }
            for (int j = 0; j < nkept; j++) {
                const uint64_t o = __shfl(best, j, WAVE);
                rk += o < key;
                rb += o < best;
            }
            __builtin_amdgcn_wave_barrier();
            if (lane < nkept && rb < a.s)
                keep[rb] = best;
            if (key != ~0ull && rk < a.s)
                keep[rk] = key;
            __builtin_amdgcn_wave_barrier();
            nkept = nkept + __popcll(has) < a.s ? nkept + __popcll(has) : a.s;
            best = lane < nkept ? keep[lane] : ~0ull;
            __builtin_amdgcn_wave_barrier();
        }
        if (offers) {
            if (lane < nkept)
                a.rold[v * a.s + lane] = best;
            if (lane == 0)
                a.rfill[2 * v + 1] = offers;
        }
    }
}

// ------------------------------------------------ reverse index construction

constexpr int RI_PER_THREAD = 8, RI_CHUNK = 256 * RI_PER_THREAD;

__global__ __launch_bounds__(256) void k_ri_fill_zero(int32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// in-degree of every row over the first kk entries of the m lists
__global__ __launch_bounds__(256) void k_ri_count(const uint64_t *gin, int gs, int kk, int64_t m,
                                                  int32_t *deg, uint64_t *ctr)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * kk;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = e / kk;
        const uint64_t w = gin[u * gs + (e - u * kk)];
        if (key_empty(w))
            continue;
        const int64_t v = (int64_t)key_id(w);
        if (v >= m)
            raise_err(ctr + C_ERR, ERR_ROW_REVERSE);
        else
            atomicAdd(deg + v, 1);
    }
}

// exclusive prefix sum over a 256-thread block; *total gets the block's sum
__device__ inline int64_t block_exclusive_sum(int64_t x, int64_t *total)
{
    __shared__ int64_t wsum[256 / WAVE];
    const int lane = lane_id(), w = threadIdx.x / WAVE;
    int64_t inc = x;
    for (int o = 1; o < WAVE; o <<= 1) {
        const int64_t y = __shfl_up(inc, o, WAVE);
        if (lane >= o)
            inc += y;
    }
    if (lane == WAVE - 1)
        wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
    for (int q = 0; q < 256 / WAVE; q++) {
        before += q < w ? wsum[q] : 0;
        all += wsum[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - x;
}

// sum of each RI_CHUNK-row chunk of deg
__global__ __launch_bounds__(256) void k_ri_chunk_sums(const int32_t *deg, int64_t m, int64_t *part)
{
    const int64_t r0 = (int64_t)blockIdx.x * RI_CHUNK + (int64_t)threadIdx.x * RI_PER_THREAD;
    int64_t x = 0;
    for (int q = 0; q < RI_PER_THREAD; q++)
        x += r0 + q < m ? deg[r0 + q] : 0;
    int64_t tot;
    (void)block_exclusive_sum(x, &tot);
    if (threadIdx.x == 0)
        part[blockIdx.x] = tot;
}

// exclusive prefix sum of the chunk sums (one block)
__global__ __launch_bounds__(256) void k_ri_scan_parts(int64_t *part, int64_t nparts)
{
    int64_t carry = 0;
    for (int64_t b = 0; b < nparts; b += 256) {
        const int64_t i = b + threadIdx.x;
        const int64_t x = i < nparts ? part[i] : 0;
        int64_t tot;
        const int64_t ex = block_exclusive_sum(x, &tot);
        if (i < nparts)
            part[i] = carry + ex;
        carry += tot;
    }
}

// off[r] = sum of deg over rows before r (off[m] = all entries); deg is
// cleared for use as the fill cursor
__global__ __launch_bounds__(256) void k_ri_offsets(int32_t *deg, int64_t m, const int64_t *part,
                                                    int64_t *off)
{
    const int64_t r0 = (int64_t)blockIdx.x * RI_CHUNK + (int64_t)threadIdx.x * RI_PER_THREAD;
    int32_t dv[RI_PER_THREAD];
    int64_t x = 0;
    for (int q = 0; q < RI_PER_THREAD; q++) {
        dv[q] = r0 + q < m ? deg[r0 + q] : 0;
        x += dv[q];
    }
    int64_t tot;
    int64_t run = part[blockIdx.x] + block_exclusive_sum(x, &tot);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        off[0] = 0;
    for (int q = 0; q < RI_PER_THREAD; q++) {
        if (r0 + q < m) {
            run += dv[q];
            off[r0 + q + 1] = run;
            deg[r0 + q] = 0;
        }
    }
}

__global__ __launch_bounds__(256) void k_ri_fill(const uint64_t *gin, int gs, int kk, int64_t m,
                                                 const int64_t *off, int32_t *cur, int32_t *src)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < m * kk;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t u = e / kk;
        const uint64_t w = gin[u * gs + (e - u * kk)];
        if (key_empty(w))
            continue;
        const int64_t v = (int64_t)key_id(w);
        if (v < m) {
            const int pos = atomicAdd(cur + v, 1);
            src[off[v] + pos] = (int32_t)u;
        }
    }
}

// count the FRESH entries left by the last round (statistics only)
__global__ __launch_bounds__(256) void k_count_fresh(RoundArgs a)
{
    // graph mode: only in round max_rounds (otherwise k_sample counts)
    if (!take_round(a) || (a.dev && a.round < a.dev->max_rounds))
        return;
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

// graph mode: the round state at the start of a merge's loop
__global__ void k_set_round(DevRound *d, DevRound v)
{
    if (threadIdx.x == 0)
        *d = v;
}

// graph mode, after the round's sampling: stop test of the repeat loop (as
// in the host-driven loop: c of round t-1 against delta*n0*k for t > 0, the
// round cap, error bits), else the round's active rows and cleared per-round
// counters
__global__ void k_round_ctl(DevRound *d, uint64_t *ctr, int k)
{
    if (threadIdx.x != 0 || d->done)
        return;
    const int t = d->round;
    bool stop = ctr[C_ERR] != 0 || t >= d->max_rounds;
    if (t > 0 && (double)ctr[C_FRESH] <= d->delta * (double)ctr[C_N0] * (double)k)
        stop = true;
    if (stop) {
        d->rounds = t;
        d->done = 1;
        return;
    }
    d->n_active = (int64_t)ctr[C_ACTIVE];
    for (int w = 0; w < C_ROUND_WORDS; w++)
        ctr[w] = 0;
}

__global__ void k_round_next(DevRound *d)
{
    if (threadIdx.x == 0 && !d->done)
        d->round++;
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
    // 1,024 blocks of 4 waves: the waves walk many rows each, which measured
    // faster than one short walk per wave
    if (a.k <= 16)
        hipLaunchKernelGGL(k_sample<16>, dim3(grid_for(a.n, 16, 1024)), dim3(256), 0, st, a);
    else if (a.k <= 32)
        hipLaunchKernelGGL(k_sample<32>, dim3(grid_for(a.n, 8, 1024)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(k_sample<WAVE>, dim3(grid_for(a.n, 4, 1024)), dim3(256), 0, st, a);
    return hipGetLastError();
}

// rows an active-row kernel walks: the list, or all n
inline int64_t active_span(const RoundArgs &a) { return a.alist ? a.n_active : a.n; }

// graph mode: workgroups of the active-row kernels (their waves walk any
// number of listed rows)
constexpr unsigned GRAPH_ACTIVE_BLOCKS = 1024;

hipError_t launch_prep_active(const RoundArgs &a, hipStream_t st)
{
    const unsigned g = a.dev ? GRAPH_ACTIVE_BLOCKS : grid_for(active_span(a), 4, 8192);
    hipLaunchKernelGGL(k_prep_active, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_reverse(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_reverse, dim3(grid_for(a.n * (a.s + a.k), 256, 1u << 20)), dim3(256),
                       0, st, a);
    return hipGetLastError();
}

hipError_t launch_reverse_indexed(const RoundArgs &a, hipStream_t st)
{
    // base first: it writes the reservoirs of its targets without atomics
    if (a.rev_m > 0 || a.dev)
        hipLaunchKernelGGL(k_reverse_base,
                           dim3(a.dev ? GRAPH_ACTIVE_BLOCKS : grid_for(active_span(a), 4, 8192)),
                           dim3(256), 0, st, a);
    hipLaunchKernelGGL(k_reverse_rows, dim3(grid_for(a.n, 4, 8192)), dim3(256), 0, st, a);
    return hipGetLastError();
}

int64_t rindex_parts(int64_t m) { return (m + RI_CHUNK - 1) / RI_CHUNK; }

hipError_t launch_build_rindex(const uint64_t *gin, int gs, int kk, int64_t m, int64_t *off,
                               int32_t *src, int32_t *deg, int64_t *part, uint64_t *ctr,
                               hipStream_t st)
{
    if (m <= 0)
        return hipSuccess;
    const int64_t parts = rindex_parts(m);
    hipLaunchKernelGGL(k_ri_fill_zero, dim3(grid_for(m, 256, 16384)), dim3(256), 0, st, deg, m);
    hipLaunchKernelGGL(k_ri_count, dim3(grid_for(m * kk, 256, 1u << 16)), dim3(256), 0, st, gin,
                       gs, kk, m, deg, ctr);
    hipLaunchKernelGGL(k_ri_chunk_sums, dim3((unsigned)parts), dim3(256), 0, st, deg, m, part);
    hipLaunchKernelGGL(k_ri_scan_parts, dim3(1), dim3(256), 0, st, part, parts);
    hipLaunchKernelGGL(k_ri_offsets, dim3((unsigned)parts), dim3(256), 0, st, deg, m, part, off);
    hipLaunchKernelGGL(k_ri_fill, dim3(grid_for(m * kk, 256, 1u << 16)), dim3(256), 0, st, gin,
                       gs, kk, m, off, deg, src);
    return hipGetLastError();
}

hipError_t launch_set_round(DevRound *d, const DevRound &v, hipStream_t st)
{
    hipLaunchKernelGGL(k_set_round, dim3(1), dim3(64), 0, st, d, v);
    return hipGetLastError();
}

hipError_t launch_round_ctl(const RoundArgs &a, int k, hipStream_t st)
{
    hipLaunchKernelGGL(k_round_ctl, dim3(1), dim3(64), 0, st, const_cast<DevRound *>(a.dev),
                       a.ctr, k);
    return hipGetLastError();
}

hipError_t launch_round_next(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_round_next, dim3(1), dim3(64), 0, st, const_cast<DevRound *>(a.dev));
    return hipGetLastError();
}

hipError_t launch_count_fresh(const RoundArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_count_fresh, dim3(grid_for(a.n * a.k, 256, 16384)), dim3(256), 0, st,
                       a);
    return hipGetLastError();
}

} // namespace knng
