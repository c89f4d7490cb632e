// knng_join.hip -- the cross-set local join, the inner loop of Algorithms 1
// and 2 (Zhao et al., "On the Merge of k-NN Graph", Sections 3.1-3.2).
//
// For every point u the neighbourhood G[u] = reverse(u) u forward(u) is split
// into a NEW group (sampled NEW forward entries and reverse-NEW sources) and
// an OLD group (OLD forward entries and reverse-OLD sources, minus NEW ones).
// Every unordered pair {p, q} with p in NEW and q in NEW u OLD that the merge
// predicate admits is compared:
//   S-Merge: p and q from different sets (Algorithm 1);
//   J-Merge: not both from the built set S1 (Algorithm 2).
// l = m(p, q) is offered to both lists (UpdateNN in both directions) through
// the lock-free bounded insert; a pair is first screened against an upper
// bound of each list's worst entry (set at the round start, lowered after a
// list takes entries, read when u's neighbourhood is formed).  The worst entry
// only decreases during a round, so the screen never drops an edge that could
// stay.  The FP32 path queues its proposals and drains the queue with all
// lanes; the BF16 path gathers a tile's proposals in an insert grid and offers
// two grids at a time member by member (insert_local).
//
// Layout.  One wave owns one u at a time (4 independent waves per workgroup,
// no workgroup barriers).  The members are placed in LDS in four regions, each
// starting at a multiple of 4:  [ newA | oldA | newB | oldB ]  (A = first set,
// B = second set).  The admitted pairs are then dense rectangles:
//   R1 = newA x (newB u oldB)      R2 = newB x oldA
//   R3 = newB x (newB u oldB), upper triangle on newB x newB (J-Merge only)
// Coordinates are staged chunk by chunk, transposed ([coordinate][member]).
//
// FP32 path (k_join): each lane accumulates a 2 x 4 register tile of pairs in
// ascending coordinate order, so every distance is the canonical FP32 value.
//
// BF16 path (k_join_bf16, l2 and cosine): 16 x 16 tiles of dot products of the
// bf16-rounded members on MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation),
// operands gathered straight from a bf16 copy of the rows into registers;
// d~ = |p~|^2 + |q~|^2 - 2 p~.q~ screens a pair against the list's worst W with
// a margin M that bounds |d~ - d_canonical| whenever d_canonical <= W:
//   M = W g1 + 2 E sqrt(W (1 + g1)) + E^2 + g2 (|p~| + |q~|)^2
// with E = |p - p~| + |q - q~| (exact per-row bf16 rounding norms),
// g1 = (dp + 8) 2^-24 (canonical FP32 accumulation) and g2 = (2 dp + 16) 2^-24
// (FP32 accumulation of the MFMA chain and of the norms).  Pairs that pass
// are rescored in canonical FP32 before any insert, so the result is the FP32
// path's, bit for bit.  Each rescored pair also checks |d~ - d| <= M(d); a
// failure (never expected) is counted as a screen violation.  Rows certified
// exact at layout time (integer coordinates in [0, 256], squared norm below
// 2^23) need no rescore between each other: every product and partial sum of
// d~ and of the canonical sum is then an integer below 2^24, so d~ is the
// canonical value.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

constexpr int JOIN_WAVES = 4;
constexpr int CH = 8;                   // coordinates per staged chunk (FP32 path)
constexpr int QCAP = 256;               // BF16 path: rescore-queue words per wave
constexpr int QF = 192;                 // FP32 path: insert-queue entries per wave
constexpr int TMAX = 1;                 // MFMA tiles held per batch (4 waves per SIMD)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bool res_empty(uint64_t w) { return (uint32_t)w >= 0x40000000u; }
__host__ __device__ __forceinline__ int r4(int x) { return (x + 3) & ~3; }

struct Regions {
    int nA, oA, nB, oB;           // member counts
    int offOA, offNB, offOB, GP;  // region starts and padded total
};

// per-wave LDS carve
struct WaveLds {
    float *vecT;     // CH x GS staged coordinates, transposed (FP32 path)
    uint64_t *gw;    // GS worst bound of each member's list
    uint64_t *q64;   // QCAP queue words (FP32 path: the QF queued keys)
    int32_t *grp;    // GS member ids (-1 = padding)
    float *gnorm;    // GS canonical norms (cosine)
    float *gsq;      // GS squared norms of bf16 rows (BF16 path)
    float *gerr;     // GS bf16 rounding-error norms (BF16 path)
    int32_t *tnew;   // 2 s NEW members, first set then second
    int32_t *toldA;  // k + s accepted OLD members of the first set
    int32_t *toldB;  // k + s accepted OLD members of the second set
    int32_t *qdst;   // FP32 path: target rows of the QF queued keys
};

// The FP32 carve (bf = false) leaves out the BF16 arrays and holds QF queue
// words: 8.3 KB per wave for s = k = 20, so that four 4-wave blocks fit the
// CU's 160 KB of LDS (4 waves per SIMD).
// first region of a wave's carve: the staged coordinates (FP32 path), or the
// BF16 path's two insert grids, each a tile's 16 x 16 rescored distances
// (1 KB), 32 offer masks of its members (128 of 256 bytes) and the ids of its
// 16 row and 16 column members (128 bytes)
constexpr int GRID_BYTES = 16 * 16 * 4 + 16 * 16 + 32 * 4;
__host__ __device__ inline int stage_bytes(int GS, bool bf)
{
    return bf && CH * GS * 4 < 2 * GRID_BYTES ? 2 * GRID_BYTES : CH * GS * 4;
}

__host__ __device__ inline int wave_lds_bytes(int GS, int s, int k, bool bf)
{
    const int st = stage_bytes(GS, bf);
    int b = bf ? st + GS * 8 + QCAP * 8 + 4 * GS * 4 + (2 * s + 2 * (k + s) + QF) * 4
               : st + GS * 8 + QF * 8 + 2 * GS * 4 + (2 * s + 2 * (k + s) + QF) * 4;
    return (b + 15) / 16 * 16;
}

__device__ inline WaveLds carve_lds(unsigned char *base, int GS, int s, int k, bool bf)
{
    WaveLds L;
    L.vecT = reinterpret_cast<float *>(base);
    L.gw = reinterpret_cast<uint64_t *>(base + stage_bytes(GS, bf));
    L.q64 = L.gw + GS;
    L.grp = reinterpret_cast<int32_t *>(L.q64 + (bf ? QCAP : QF));
    L.gnorm = reinterpret_cast<float *>(L.grp + GS);
    L.gsq = bf ? L.gnorm + GS : nullptr;
    L.gerr = bf ? L.gsq + GS : nullptr;
    L.tnew = reinterpret_cast<int32_t *>(bf ? L.gerr + GS : L.gnorm + GS);
    L.toldA = L.tnew + 2 * s;
    L.toldB = L.toldA + (k + s);
    L.qdst = L.toldB + (k + s);
    return L;
}

// The id set of build_group: ID_SET slots (a power of two), linear probing.
constexpr int ID_SET = 256;
constexpr uint32_t ID_FREE = 0xFFFFFFFFu;

// claims id in the set; true when this lane's claim put it there (of lanes
// claiming one id together, exactly one succeeds)
__device__ __forceinline__ bool claim_id(uint32_t *tab, int32_t id)
{
    uint32_t h = ((uint32_t)id * 2654435761u) >> 24;
    for (int probe = 0; probe < ID_SET; probe++) {
        const uint32_t old = atomicCAS(tab + h, ID_FREE, (uint32_t)id);
        if (old == ID_FREE)
            return true;
        if (old == (uint32_t)id)
            return false;
        h = (h + 1) & (ID_SET - 1);
    }
    return false;
}

// Forms u's neighbourhood in LDS (regions, ids, worst bounds, norms).
// Returns false when u has no NEW member (no pair to join).  Two memory round
// trips: the counts, both samples and both reverse reservoirs together
// (entries past a count are read and ignored), then the members' bounds and
// norms.  Repeats are found through a small open-addressing set of ids in LDS
// (the BF16 path's queue words or the FP32 path's staging area, both free
// while a neighbourhood is formed): the NEW candidates claim their ids first,
// then the OLD ones; a candidate is kept when its claim succeeds.
template <int METRIC, bool BF>
__device__ inline bool build_group(int64_t u, const Rows &R, const RoundArgs &a, const WaveLds &L,
                                   Regions &g)
{
    static_assert(2 * MAX_S <= WAVE && MAX_K + MAX_S <= 2 * WAVE, "candidate lanes");
    const int lane = lane_id();
    const int s = a.s, k = a.k;
    const int nco = k + s;
    const uint64_t below = (1ull << lane) - 1ull;
    const int cnt_new = a.cnt_f[2 * u], cnt_old = a.cnt_f[2 * u + 1];
    uint32_t *tab = BF ? reinterpret_cast<uint32_t *>(L.q64) : reinterpret_cast<uint32_t *>(L.vecT);
    for (int i = lane; i < ID_SET; i += WAVE)
        tab[i] = ID_FREE;
    // NEW candidates: forward NEW sample (lanes < s), reverse NEW (s..2s);
    // OLD candidates: forward OLD (c < k), reverse OLD (k <= c < k+s), c =
    // lane + 64 * pass
    int32_t nf = -1;
    uint64_t nr = ~0ull;
    if (lane < s)
        nf = a.new_f[u * s + lane];
    else if (lane < 2 * s)
        nr = a.rnew[u * s + (lane - s)];
    int32_t of[2] = {-1, -1};
    uint64_t orv[2] = {~0ull, ~0ull};
#pragma unroll
    for (int p = 0; p < 2; p++) {
        const int c = p * WAVE + lane;
        if (c < k)
            of[p] = a.old_f[u * k + c];
        else if (c < nco)
            orv[p] = a.rold[u * s + (c - k)];
    }
    int32_t cid = -1;
    if (lane < s) {
        if (lane < cnt_new)
            cid = nf;
    } else if (lane < 2 * s) {
        if (!res_empty(nr))
            cid = (int32_t)(uint32_t)nr;
    }
    if (cid >= a.n) {
        raise_err(a.ctr + C_ERR, ERR_ROW_GROUP);
        cid = -1;
    }
    // a NEW member is kept once
    const bool keep = cid >= 0 && claim_id(tab, cid);
    const bool isA = cid < a.n1;
    const uint64_t mA = __ballot(keep && isA), mB = __ballot(keep && !isA);
    const int nA = __popcll(mA), nB = __popcll(mB);
    if (nA + nB == 0)
        return false;
    if (keep)
        L.tnew[isA ? __popcll(mA & below) : nA + __popcll(mB & below)] = cid;
    // an OLD candidate is kept unless it is a NEW member or repeats an earlier
    // candidate
    int32_t oc[2];
    bool ok[2];
#pragma unroll
    for (int p = 0; p < 2; p++) {
        const int c = p * WAVE + lane;
        oc[p] = -1;
        if (c < k) {
            if (c < cnt_old)
                oc[p] = of[p];
        } else if (c < nco) {
            if (!res_empty(orv[p]))
                oc[p] = (int32_t)(uint32_t)orv[p];
        }
        if (oc[p] >= a.n) {
            raise_err(a.ctr + C_ERR, ERR_ROW_GROUP);
            oc[p] = -1;
        }
        ok[p] = oc[p] >= 0;
    }
#pragma unroll
    for (int p = 0; p < 2; p++)
        ok[p] = ok[p] && claim_id(tab, oc[p]);
    int oA = 0, oB = 0;
#pragma unroll
    for (int p = 0; p < 2; p++) {
        const bool oa = oc[p] < a.n1;
        const uint64_t moA = __ballot(ok[p] && oa), moB = __ballot(ok[p] && !oa);
        if (ok[p]) {
            if (oa)
                L.toldA[oA + __popcll(moA & below)] = oc[p];
            else
                L.toldB[oB + __popcll(moB & below)] = oc[p];
        }
        oA += __popcll(moA);
        oB += __popcll(moB);
    }
    __builtin_amdgcn_wave_barrier();
    g.nA = nA;
    g.oA = oA;
    g.nB = nB;
    g.oB = oB;
    g.offOA = r4(nA);
    g.offNB = g.offOA + r4(oA);
    g.offOB = g.offNB + r4(nB);
    g.GP = g.offOB + r4(oB);
    if constexpr (!BF) {
        // FP32 path: slot by slot (fewer live registers in its larger kernels)
        for (int slot = lane; slot < g.GP; slot += WAVE) {
            int32_t id = -1;
            if (slot < nA)
                id = L.tnew[slot];
            else if (slot >= g.offOA && slot < g.offOA + oA)
                id = L.toldA[slot - g.offOA];
            else if (slot >= g.offNB && slot < g.offNB + nB)
                id = L.tnew[nA + (slot - g.offNB)];
            else if (slot >= g.offOB && slot < g.offOB + oB)
                id = L.toldB[slot - g.offOB];
            L.grp[slot] = id;
            L.gw[slot] = id >= 0 ? a.worst[id * a.ws] : 0ull;
            if (METRIC == M_COS)
                L.gnorm[slot] = id >= 0 ? R.norm[R.phys(id)] : 1.0f;
        }
    } else {
    // slots lane + 64 i: ids, then every bound and norm in one round trip
        constexpr int NSL = 3;
        int32_t id[NSL];
        uint64_t gw[NSL];
        float gn[NSL], gq[NSL], ge[NSL];
    #pragma unroll
        for (int i = 0; i < NSL; i++) {
            const int slot = lane + i * WAVE;
            int32_t v = -1;
            if (slot < nA)
                v = L.tnew[slot];
            else if (slot >= g.offOA && slot < g.offOA + oA)
                v = L.toldA[slot - g.offOA];
            else if (slot >= g.offNB && slot < g.offNB + nB)
                v = L.tnew[nA + (slot - g.offNB)];
            else if (slot >= g.offOB && slot < g.offOB + oB)
                v = L.toldB[slot - g.offOB];
            id[i] = slot < g.GP ? v : -1;
        }
    #pragma unroll
        for (int i = 0; i < NSL; i++) {
            const bool has = id[i] >= 0;
            gw[i] = has ? a.worst[id[i] * a.ws] : 0ull;
            gn[i] = METRIC == M_COS && has ? R.norm[R.phys(id[i])] : 1.0f;
            const float2 se =
                BF && has ? R.se[R.phys(id[i]) * R.se_stride] : make_float2(0.0f, 0.0f);
            gq[i] = se.x;
            ge[i] = se.y;
        }
    #pragma unroll
        for (int i = 0; i < NSL; i++) {
            const int slot = lane + i * WAVE;
            if (slot < g.GP) {
                L.grp[slot] = id[i];
                L.gw[slot] = gw[i];
                if (METRIC == M_COS)
                    L.gnorm[slot] = gn[i];
                if (BF) {
                    L.gsq[slot] = gq[i];
                    L.gerr[slot] = ge[i];
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    return true;
}

// Stage coordinates [c0, c0+CH) of every member slot into LDS, transposed.
template <int MU>
__device__ inline void stage_chunk(const Rows &R, const WaveLds &L, int GP, int GS, int c0)
{
    constexpr int q4 = CH / 4;
    const int lane = lane_id();
    const int units = GP * q4;
    __builtin_amdgcn_wave_barrier();
    float4 pre[MU];
#pragma unroll
    for (int j = 0; j < MU; j++) {
        const int e = lane + j * WAVE;
        pre[j] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (e < units) {
            const int m = e / q4, q = e - m * q4;
            const int32_t id = L.grp[m];
            if (id >= 0 && c0 + 4 * q < R.dp)
                pre[j] = *reinterpret_cast<const float4 *>(R.x + R.phys(id) * R.dp + c0 + 4 * q);
        }
    }
#pragma unroll
    for (int j = 0; j < MU; j++) {
        const int e = lane + j * WAVE;
        if (e < units) {
            const int m = e / q4, q = e - m * q4;
            L.vecT[(4 * q + 0) * GS + m] = pre[j].x;
            L.vecT[(4 * q + 1) * GS + m] = pre[j].y;
            L.vecT[(4 * q + 2) * GS + m] = pre[j].z;
            L.vecT[(4 * q + 3) * GS + m] = pre[j].w;
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// tile t -> (row start, column start, rectangle) for 2 x 4 tiles
__device__ __forceinline__ bool tile_of(int t, const Regions &g, int joint, int &r0, int &c0,
                                        int &reg)
{
    const int colsB = g.GP - g.offNB;  // newB u oldB, padded
    const int rt1 = (g.nA + 1) / 2, ct1 = colsB / 4;
    const int T1 = rt1 * ct1;
    if (t < T1) {
        r0 = 2 * (t / ct1);
        c0 = g.offNB + 4 * (t % ct1);
        reg = 1;
        return true;
    }
    t -= T1;
    const int rt2 = (g.nB + 1) / 2, ct2 = r4(g.oA) / 4;
    const int T2 = rt2 * ct2;
    if (t < T2) {
        r0 = g.offNB + 2 * (t / ct2);
        c0 = g.offOA + 4 * (t % ct2);
        reg = 2;
        return true;
    }
    t -= T2;
    if (joint && t < rt2 * ct1) {
        r0 = g.offNB + 2 * (t / ct1);
        c0 = g.offNB + 4 * (t % ct1);
        reg = 3;
        return true;
    }
    return false;
}

// UpdateNN of one proposal: the list of row dst takes key if it beats the
// worst entry and is not there yet; a row that took an entry is sampled in
// the next round
template <int KB>
__device__ __forceinline__ void insert_into(const RoundArgs &a, int64_t dst, uint64_t key)
{
    // dst and the key's id are neighbourhood members, range-checked when the
    // neighbourhood was formed
    if (bounded_insert<KB>(a.L + dst * a.k, a.k, key, DUP_ID, a.worst + dst * a.ws, a.ctr + C_ERR))
        a.dtag[dst] = a.tag0 + a.round + 1;
}

// UpdateNN of several proposals for one list by one lane: one read of the
// list into a local view, then one compare-and-swap per proposal on the
// maximum of the view; a failed swap returns the slot's current word, which
// replaces the view's, and the proposal is tried again.  Every word of the
// view is one its slot held at some time before the swap (the lane's own
// swaps included; a word read through the caches is an older, hence larger,
// value of its slot), which is all the argument of bounded_insert needs: each
// successful swap replaces the true maximum, and duplicates stay out.  The
// view's maximum is kept between proposals, so a proposal that does not beat
// it costs one comparison; the maximum of the final view bounds the list's.
// FULL: the list is exactly as long as the view, so no slot of the view is
// unused and no slot index needs a test (without it the compiler keeps one
// lane mask per slot, which spill and are reloaded in every pass of the loop).
template <int KB, bool FULL, class KeyFn>
__device__ __forceinline__ void insert_view(const RoundArgs &a, int64_t dst, uint32_t have,
                                            KeyFn key_of)
{
    constexpr int B = KB <= 16 ? KB : (KB == 32 ? 20 : 16);
    const int cap = FULL ? B : a.k;
    uint64_t *slots = a.L + dst * cap;
    bool any = false;
    uint64_t v[B];
#pragma unroll
    for (int j = 0; j < B; j++)
        v[j] = FULL || j < cap ? slots[j] : 0ull;
    uint64_t mx = 0;
    int mj = 0;
    auto rescan = [&]() {
        mx = 0;
        mj = 0;
#pragma unroll
        for (int j = 0; j < B; j++) {
            if ((FULL || j < cap) && v[j] > mx) {
                mx = v[j];
                mj = j;
            }
        }
    };
    rescan();
    for (int fails = 0; have && fails < SPIN_BUDGET;) {
        const uint64_t key = key_of(__builtin_ctz(have));
        if (key >= mx) {
            have &= have - 1;
            continue;
        }
        // equal ids mean equal entries (one pair, one canonical distance), so
        // the id field decides; empty slots' id fields are above every row id
        const uint32_t kid = key_id(key);
        bool dup = false;
#pragma unroll
        for (int j = 0; j < B; j++)
            dup |= (FULL || j < cap) && key_id(v[j]) == kid;
        if (dup) {
            have &= have - 1;
            continue;
        }
        uint64_t seen = mx;
        const bool ok = cas64_seen(slots + mj, seen, key);
#pragma unroll
        for (int j = 0; j < B; j++)
            v[j] = j == mj ? (ok ? key : seen) : v[j];
        rescan();
        if (!ok) {
            fails++;
            continue;
        }
        any = true;
        have &= have - 1;
    }
    if (have)
        atomicOr((unsigned long long *)(a.ctr + C_ERR), (unsigned long long)ERR_SPIN);
    if (any) {
        // every word of the view is at least its slot's current value
        atomic_min_u64(a.worst + dst * a.ws, key_strip(mx));
        a.dtag[dst] = a.tag0 + a.round + 1;
    }
}

// UpdateNN of the proposals in have (bits of key_of's index) for row dst: a
// list longer than the view takes them one by one, a shorter or equal one
// through the view
template <int KB, class KeyFn>
__device__ inline void insert_local(const RoundArgs &a, int64_t dst, uint32_t have, KeyFn key_of)
{
    constexpr int B = KB <= 16 ? KB : (KB == 32 ? 20 : 16);
    if (a.k > B) {
        for (; have; have &= have - 1)
            insert_into<KB>(a, dst, key_of(__builtin_ctz(have)));
    } else if (a.k == B) {
        insert_view<KB, true>(a, dst, have, key_of);
    } else {
        insert_view<KB, false>(a, dst, have, key_of);
    }
}

// Drain a queue of (target row, key) words: every entry is offered to its
// list (the insert's own read of the list rejects entries that no longer beat
// its worst).  Returns the number of inserts attempted (wave-uniform).
template <int KB>
__device__ inline int drain_keys(const uint64_t *qkey, const int32_t *qdst, int qn,
                                 const RoundArgs &a)
{
    for (int e0 = 0; e0 < qn; e0 += WAVE) {
        const int e = e0 + lane_id();
        if (e < qn) {
            const int32_t dst = qdst[e];
            insert_into<KB>(a, dst, qkey[e]);
        }
    }
    return qn;
}

__device__ inline void flush_counters(const RoundArgs &a, uint64_t pairs_lane, uint64_t gathered,
                                      uint64_t attempts, uint64_t rescored_lane,
                                      uint64_t viol_lane, int maxg)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        pairs_lane += __shfl_xor(pairs_lane, o, WAVE);
        rescored_lane += __shfl_xor(rescored_lane, o, WAVE);
        viol_lane += __shfl_xor(viol_lane, o, WAVE);
    }
    if (lane_id() == 0) {
        unsigned long long *c = (unsigned long long *)a.ctr;
        if (pairs_lane) {
            atomicAdd(c + C_PAIRS, (unsigned long long)pairs_lane);
            atomicAdd(c + C_EVALS, (unsigned long long)pairs_lane);
        }
        if (gathered)
            atomicAdd(c + C_GATHER, (unsigned long long)gathered);
        if (attempts)
            atomicAdd(c + C_ATTEMPT, (unsigned long long)attempts);
        if (rescored_lane)
            atomicAdd(c + C_RESCORE, (unsigned long long)rescored_lane);
        if (viol_lane)
            atomicAdd(c + C_VIOL, (unsigned long long)viol_lane);
        if (maxg)
            atomicMax(c + C_MAXG, (unsigned long long)maxg);
    }
}

// ============================================================ FP32 path
template <int METRIC, int KB, int MU>
__global__ __launch_bounds__(JOIN_WAVES * WAVE, MU == 4 ? 4 : 2) void k_join(Rows R, RoundArgs a, int GS,
                                                            int wave_bytes)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    if (!take_round(a, R))
        return;
    const int lane = lane_id();
    const WaveLds L = carve_lds(dyn + (size_t)(threadIdx.x / WAVE) * wave_bytes, GS, a.s, a.k, false);
    // the insert queue lives across tiles and rows: it is drained in whole
    // 64-entry steps when it runs full, and once more at the end
    uint64_t *qkey = L.q64;
    int32_t *qdst = L.qdst;
    int qn = 0;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t n_pairs = 0, n_gather = 0, n_attempt = 0;
    int maxg = 0;
    const int64_t nwaves = (int64_t)gridDim.x * JOIN_WAVES;
    const int64_t wave0 = (int64_t)blockIdx.x * JOIN_WAVES + threadIdx.x / WAVE;
    // rows (or active-list entries) wave0 + j*nwaves, 64 at a time; only rows
    // with a NEW member join
    const bool listed = a.alist != nullptr;
    const int64_t span = listed ? a.n_active : a.n;
    for (int64_t b = wave0; b < span; b += nwaves * WAVE) {
        const int64_t r = b + (int64_t)lane * nwaves;
        uint64_t todo = __ballot(r < span && (listed || a.atag[r] == a.tag0 + a.round));
        while (todo) {
        const int64_t j = b + (int64_t)__builtin_ctzll(todo) * nwaves;
        const int64_t u = listed ? (int64_t)a.alist[j] : j;
        todo &= todo - 1;
        __builtin_amdgcn_wave_barrier();
        Regions g;
        if (!build_group<METRIC, false>(u, R, a, L, g))
            continue;
        const int G = g.nA + g.oA + g.nB + g.oB;
        n_gather += (uint64_t)G;
        maxg = G > maxg ? G : maxg;
        const int colsB = g.GP - g.offNB;
        int T = ((g.nA + 1) / 2) * (colsB / 4) + ((g.nB + 1) / 2) * (r4(g.oA) / 4);
        if (a.joint)
            T += ((g.nB + 1) / 2) * (colsB / 4);
        for (int tb = 0; tb < T; tb += WAVE) {
            float acc[2][4];
            int tr0 = 0, tc0 = 0, treg = 0;
            const bool tv = tile_of(tb + lane, g, a.joint, tr0, tc0, treg);
#pragma unroll
            for (int x = 0; x < 2; x++)
#pragma unroll
                for (int y = 0; y < 4; y++)
                    acc[x][y] = 0.0f;
            for (int c0 = 0; c0 < R.dp; c0 += CH) {
                stage_chunk<MU>(R, L, g.GP, GS, c0);
                const int cw = R.dp - c0 < CH ? R.dp - c0 : CH;
                if (tv) {
#pragma unroll 2
                    for (int t = 0; t < cw; t++) {
                        const float2 xr =
                            *reinterpret_cast<const float2 *>(L.vecT + t * GS + tr0);
                        const float4 xc =
                            *reinterpret_cast<const float4 *>(L.vecT + t * GS + tc0);
                        const float xrs[2] = {xr.x, xr.y};
                        const float xcs[4] = {xc.x, xc.y, xc.z, xc.w};
#pragma unroll
                        for (int x = 0; x < 2; x++)
#pragma unroll
                            for (int y = 0; y < 4; y++)
                                acc[x][y] = canon_step<METRIC>(acc[x][y], xrs[x], xcs[y]);
                    }
                }
            }
            // screen; survivors go through the wave's insert queue, drained by
            // all lanes together (UpdateNN in both directions)
#pragma unroll
            for (int x = 0; x < 2; x++) {
                const int r = tr0 + x;
#pragma unroll
                for (int y = 0; y < 4; y++) {
                    const int c = tc0 + y;
                    const int32_t p = tv ? L.grp[r] : -1;
                    const int32_t q = tv ? L.grp[c] : -1;
                    const bool valid = p >= 0 && q >= 0 && !(treg == 3 && c <= r);
                    n_pairs += valid;
                    float na = 0.0f, nb = 0.0f;
                    if (METRIC == M_COS && valid) {
                        na = L.gnorm[r];
                        nb = L.gnorm[c];
                    }
                    const float l = canon_finish<METRIC>(acc[x][y], na, nb);
                    const uint64_t kp = make_key(l, (uint32_t)q, F_NEW | F_FRESH);
                    const uint64_t kq = make_key(l, (uint32_t)p, F_NEW | F_FRESH);
                    const bool vp = valid && kp < L.gw[r];
                    const bool vq = valid && kq < L.gw[c];
                    const uint64_t mp = __ballot(vp), mq = __ballot(vq);
                    if (vp) {
                        const int pos = qn + __popcll(mp & below);
                        qkey[pos] = kp;
                        qdst[pos] = p;
                    }
                    qn += __popcll(mp);
                    if (vq) {
                        const int pos = qn + __popcll(mq & below);
                        qkey[pos] = kq;
                        qdst[pos] = q;
                    }
                    qn += __popcll(mq);
                    if (qn > QF - 2 * WAVE) {
                        // drain the top whole steps, keep the rest (< 64)
                        const int keep = qn & (WAVE - 1);
                        __builtin_amdgcn_wave_barrier();
                        n_attempt += drain_keys<KB>(qkey + keep, qdst + keep, qn - keep, a);
                        qn = keep;
                        __builtin_amdgcn_wave_barrier();
                    }
                }
            }
        }
        }
    }
    __builtin_amdgcn_wave_barrier();
    n_attempt += drain_keys<KB>(qkey, qdst, qn, a);
    flush_counters(a, n_pairs, n_gather, n_attempt, 0, 0, maxg);
}

// ============================================================ BF16 path
// 16 x 16 tile t of the rectangles -> packed (row origin | col origin << 8 |
// rectangle << 16), rectangle 0 = none
__device__ __forceinline__ int tile16_of(int t, const Regions &g, int joint)
{
    const int colsB = g.GP - g.offNB;
    const int ct1 = (colsB + 15) / 16;
    const int T1 = ((g.nA + 15) / 16) * ct1;
    if (t < T1)
        return (16 * (t / ct1)) | ((g.offNB + 16 * (t % ct1)) << 8) | (1 << 16);
    t -= T1;
    const int rt2 = (g.nB + 15) / 16, ct2 = (g.oA + 15) / 16;
    const int T2 = rt2 * ct2;
    if (t < T2)
        return (g.offNB + 16 * (t / ct2)) | ((g.offOA + 16 * (t % ct2)) << 8) | (2 << 16);
    t -= T2;
    if (joint && t < rt2 * ct1)
        return (g.offNB + 16 * (t / ct1)) | ((g.offNB + 16 * (t % ct1)) << 8) | (3 << 16);
    return 0;
}

// is (r, c) inside rectangle `reg` (and above the diagonal for rectangle 3)?
__device__ __forceinline__ bool in_rect(int reg, int r, int c, const Regions &g)
{
    if (reg == 1)
        return r < g.nA && c >= g.offNB && c < g.GP;
    if (reg == 2)
        return r >= g.offNB && r < g.offNB + g.nB && c >= g.offOA && c < g.offOA + g.oA;
    if (reg == 3)
        return r >= g.offNB && r < g.offNB + g.nB && c > r && c < g.GP;
    return false;
}

__device__ __forceinline__ int tiles16(const Regions &g, int joint)
{
    const int ct1 = (g.GP - g.offNB + 15) / 16;
    int T = ((g.nA + 15) / 16) * ct1 + ((g.nB + 15) / 16) * ((g.oA + 15) / 16);
    if (joint)
        T += ((g.nB + 15) / 16) * ct1;
    return T;
}

// screening margin in l2 space (see the file header)
__device__ __forceinline__ float bf16_margin(float W, float E, float N2, int dp)
{
    const float g1 = (float)(dp + 8) * 0x1p-24f;
    const float g2 = (float)(2 * dp + 16) * 0x1p-24f;
    const float m = W * g1 + 2.0f * E * __builtin_sqrtf(W * (1.0f + g1)) + E * E + g2 * N2;
    return m * (1.0f + 0x1p-16f) + 1e-30f;
}

// the worst entry of a list as an l2-space threshold (+inf when not full)
template <int METRIC>
__device__ __forceinline__ float l2_threshold(uint64_t worst, float na, float nb)
{
    if (key_empty(worst))
        return __uint_as_float(0x7F800000u);
    const float W = key_dist(worst);
    if (METRIC == M_COS) {
        // canonical cosine r = (D - (na-nb)^2) / (2 na nb) is increasing in D;
        // r <= W implies D <= W 2 na nb + (na-nb)^2 up to a few roundings
        const float e = na - nb;
        return (W * (2.0f * na * nb) + e * e) * (1.0f + 0x1p-19f) + 1e-30f;
    }
    return W;
}

template <int METRIC, int KB>
__global__ __launch_bounds__(JOIN_WAVES * WAVE, 4) void k_join_bf16(Rows R, RoundArgs a, int GS,
                                                                 int wave_bytes)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    if (!take_round(a, R))
        return;
    const int lane = lane_id();
    const WaveLds L = carve_lds(dyn + (size_t)(threadIdx.x / WAVE) * wave_bytes, GS, a.s, a.k, true);
    // queue word: slot r | slot c << 8 | (p gets q) << 16 | (q gets p) << 17 in
    // the low half, the screening distance's bits in the high half
    uint64_t *qw = L.q64;
    const uint64_t below = (1ull << lane) - 1ull;
    const float inf = __uint_as_float(0x7F800000u);
    const int ksteps = R.db / 32;
    const int koff = 8 * (lane >> 4);  // this lane's 8 coordinates of a 32-step
    uint64_t n_pairs = 0, n_gather = 0, n_attempt = 0, n_rescore = 0, n_viol = 0;
    int maxg = 0;
    // Insert grids: a tile's proposals wait in grid 0 until the next tile (of
    // this row or a later one) fills grid 1; then lanes 0-31 offer grid 0's
    // and lanes 32-63 grid 1's, one lane per member (row members by lanes
    // 0-15 of a half, column members by 16-31), so the two lists' round trips
    // overlap.  A member of both grids is offered by two lanes, which the
    // insert's CAS keeps correct.
    auto grid_at = [&](int gi) { return reinterpret_cast<unsigned char *>(L.vecT) + gi * GRID_BYTES; };
    auto offer_grids = [&](int ng) {
        __builtin_amdgcn_wave_barrier();
        auto gids = [&](int gi) {
            return reinterpret_cast<const int32_t *>(grid_at(gi) + 16 * 16 * 4 + 16 * 16);
        };
        auto gmask = [&](int gi) {
            return reinterpret_cast<const uint32_t *>(grid_at(gi) + 16 * 16 * 4);
        };
        const int j = lane & 15;
        // two tiles of one row band share their row members: one lane then
        // offers a row member both grids' proposals (lanes 0-15), and the
        // column members of grid 0 and 1 take lanes 16-31 and 32-47
        const bool shared = ng == 2 && __ballot(gids(0)[j] != gids(1)[j]) == 0ull;
        int gi = lane >> 5;
        bool rowside = (lane & 31) < 16, both = false, act = gi < ng;
        if (shared) {
            gi = lane < 32 ? 0 : 1;
            rowside = lane < 16;
            both = rowside;
            act = lane < 48;
        }
        if (act) {
            const int32_t me = gids(gi)[rowside ? j : 16 + j];
            uint32_t have = 0;
            if (me >= 0) {
                const int mw = (rowside ? 0 : 16) + j;
                have = gmask(gi)[mw];
                if (both)
                    have |= gmask(gi + 1)[mw] << 16;
            }
            if (have)
                insert_local<KB>(a, me, have, [&](int t) {
                    const int g2 = gi + (t >> 4), tt = t & 15;
                    const float *gl = reinterpret_cast<const float *>(grid_at(g2));
                    const int cell = rowside ? j * 16 + tt : tt * 16 + j;
                    return make_key(gl[cell], (uint32_t)gids(g2)[rowside ? 16 + tt : tt],
                                    F_NEW | F_FRESH);
                });
        }
        __builtin_amdgcn_wave_barrier();
    };
    bool pending = false;  // grid 0 holds a tile not yet offered
    const int64_t nwaves = (int64_t)gridDim.x * JOIN_WAVES;
    const int64_t wave0 = (int64_t)blockIdx.x * JOIN_WAVES + threadIdx.x / WAVE;
    // rows (or active-list entries) wave0 + j*nwaves, 64 at a time; only rows
    // with a NEW member join
    const bool listed = a.alist != nullptr;
    const int64_t span = listed ? a.n_active : a.n;
    for (int64_t b = wave0; b < span; b += nwaves * WAVE) {
        const int64_t r = b + (int64_t)lane * nwaves;
        uint64_t todo = __ballot(r < span && (listed || a.atag[r] == a.tag0 + a.round));
        while (todo) {
        const int64_t j = b + (int64_t)__builtin_ctzll(todo) * nwaves;
        const int64_t u = listed ? (int64_t)a.alist[j] : j;
        todo &= todo - 1;
        __builtin_amdgcn_wave_barrier();
        Regions g;
        if (!build_group<METRIC, true>(u, R, a, L, g))
            continue;
        const int G = g.nA + g.oA + g.nB + g.oB;
        n_gather += (uint64_t)G;
        maxg = G > maxg ? G : maxg;
        const int T = tiles16(g, a.joint);
        const int kq = 4 * (lane >> 4);  // this lane's output rows of a tile
        for (int tb = 0; tb < T; tb += TMAX) {
            f32x4 acc[TMAX];
            int tl[TMAX];
#pragma unroll
            for (int i = 0; i < TMAX; i++) {
                acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
                tl[i] = tile16_of(tb + i, g, a.joint);
            }
            // operands straight from the bf16 rows: lane l holds row (l % 16)
            // of the tile's row band and of its column band, 8 coordinates
#pragma unroll
            for (int i = 0; i < TMAX; i++) {
                if (tl[i] == 0)
                    continue;
                const int rs = (tl[i] & 0xFF) + (lane & 15);
                const int cs = ((tl[i] >> 8) & 0xFF) + (lane & 15);
                const int32_t ir = rs < g.GP ? L.grp[rs] : -1;
                const int32_t ic = cs < g.GP ? L.grp[cs] : -1;
                const bf16x8 *pa =
                    reinterpret_cast<const bf16x8 *>(R.xb + R.phys(ir < 0 ? 0 : ir) * R.db + koff);
                const bf16x8 *pb =
                    reinterpret_cast<const bf16x8 *>(R.xb + R.phys(ic < 0 ? 0 : ic) * R.db + koff);
                const bf16x8 zero = {};
#pragma unroll 4
                for (int ks = 0; ks < ksteps; ks++) {
                    const bf16x8 A = ir >= 0 ? pa[4 * ks] : zero;
                    const bf16x8 B = ic >= 0 ? pb[4 * ks] : zero;
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[i], 0, 0, 0);
                }
            }
            // screen whole tiles into the queue while one more tile fits, then
            // drain it (one drain site); this lane holds rows rb + kq + rr of
            // column cb + lane % 16 of each tile
            int done = 0;
            while (done < TMAX) {
                int qn = 0;
#pragma unroll
                for (int i = 0; i < TMAX; i++) {
                    if (i < done || qn > QCAP - 4 * WAVE)
                        continue;
                    done = i + 1;
                    const int reg = tl[i] >> 16;
                    // the column member (lane % 16) is read once for the 4 rows
                    const int c = ((tl[i] >> 8) & 0xFF) + (lane & 15);
                    const int32_t qc = L.grp[c];
                    const float sqc = L.gsq[c], erc = L.gerr[c];
                    const float nbc = METRIC == M_COS ? L.gnorm[c] : 0.0f;
                    const uint64_t gwc = L.gw[c];
#pragma unroll
                    for (int rr = 0; rr < 4; rr++) {
                        const int r = (tl[i] & 0xFF) + kq + rr;
                        bool valid = in_rect(reg, r, c, g);
                        const int32_t p = valid ? L.grp[r] : -1, q = valid ? qc : -1;
                        valid = valid && p >= 0 && q >= 0;
                        n_pairs += valid;
                        bool vp = false, vq = false;
                        float dbf = 0.0f;
                        if (valid) {
                            const float sp = L.gsq[r], sq = sqc;
                            dbf = __builtin_fmaf(-2.0f, acc[i][rr], sp + sq);
                            const float na = METRIC == M_COS ? L.gnorm[r] : 0.0f;
                            const float nb = nbc;
                            if (signbit(L.gerr[r]) && signbit(erc)) {
                                // certified exact pair: d~ is the canonical value
                                const float l = METRIC == M_COS ? cos_finish(dbf, na, nb) : dbf;
                                vp = make_key(l, (uint32_t)q, F_NEW | F_FRESH) < L.gw[r];
                                vq = make_key(l, (uint32_t)p, F_NEW | F_FRESH) < gwc;
                            } else {
                                const float E =
                                    (fabsf(L.gerr[r]) + fabsf(erc)) * (1.0f + 0x1p-22f);
                                const float nn = __builtin_sqrtf(sp) + __builtin_sqrtf(sq);
                                const float N2 = nn * nn * (1.0f + 0x1p-20f);
                                const float Wp = l2_threshold<METRIC>(L.gw[r], na, nb);
                                const float Wq = l2_threshold<METRIC>(gwc, na, nb);
                                vp = Wp == inf || dbf <= (Wp + bf16_margin(Wp, E, N2, R.dp)) *
                                                             (1.0f + 0x1p-22f);
                                vq = Wq == inf || dbf <= (Wq + bf16_margin(Wq, E, N2, R.dp)) *
                                                             (1.0f + 0x1p-22f);
                            }
                        }
                        const bool any = vp || vq;
                        const uint64_t m = __ballot(any);
                        if (any) {
                            const uint32_t lo = (uint32_t)r | ((uint32_t)c << 8) |
                                                ((uint32_t)vp << 16) | ((uint32_t)vq << 17);
                            qw[qn + __popcll(m & below)] =
                                ((uint64_t)__float_as_uint(dbf) << 32) | lo;
                        }
                        qn += __popcll(m);
                    }
                }
                // rescore in canonical FP32 (unless certified) into a 16 x 16
                // grid of distances and offer flags with the tile's member
                // ids; the grids are then offered (UpdateNN both ways) member
                // by member, two tiles at a time
                static_assert(TMAX == 1, "an insert grid holds one tile");
                unsigned char *gb = grid_at(pending ? 1 : 0);
                float *gl = reinterpret_cast<float *>(gb);
                // bit t of word j: row member j is offered column member t;
                // of word 16 + j: column member j is offered row member t
                uint32_t *gm = reinterpret_cast<uint32_t *>(gb + 16 * 16 * 4);
                int32_t *gid = reinterpret_cast<int32_t *>(gb + 16 * 16 * 4 + 16 * 16);
                const int rb = tl[0] & 0xFF, cb = (tl[0] >> 8) & 0xFF;
                __builtin_amdgcn_wave_barrier();
                if (lane < 32) {
                    gm[lane] = 0u;
                    const int slot = (lane < 16 ? rb : cb) + (lane & 15);
                    gid[lane] = slot < g.GP ? L.grp[slot] : -1;
                }
                __builtin_amdgcn_wave_barrier();
                for (int e0 = 0; e0 < qn; e0 += WAVE) {
                    const int e = e0 + lane;
                    bool gp = false, gq = false;
                    if (e < qn) {
                        const uint64_t w = qw[e];
                        const int sr = (int)(w & 0xFF), sc = (int)((w >> 8) & 0xFF);
                        const int32_t pp = L.grp[sr], qq = L.grp[sc];
                        const float db = __uint_as_float((uint32_t)(w >> 32));
                        float D = db;
                        if (!(signbit(L.gerr[sr]) && signbit(L.gerr[sc]))) {
                            D = canon_dist<M_L2>(R.x + R.phys(pp) * R.dp,
                                                 R.x + R.phys(qq) * R.dp, R.dp, 0.0f, 0.0f);
                            n_rescore++;
                            // the margin also bounds |d~ - d| at d itself
                            const float sp = L.gsq[sr], sq2 = L.gsq[sc];
                            const float E =
                                (fabsf(L.gerr[sr]) + fabsf(L.gerr[sc])) * (1.0f + 0x1p-22f);
                            const float nn = __builtin_sqrtf(sp) + __builtin_sqrtf(sq2);
                            const float M =
                                bf16_margin(D, E, nn * nn * (1.0f + 0x1p-20f), R.dp);
                            n_viol += !(fabsf(db - D) <= M * (1.0f + 0x1p-20f));
                        }
                        float l = D;
                        if (METRIC == M_COS)
                            l = cos_finish(D, L.gnorm[sr], L.gnorm[sc]);
                        gp = ((w >> 16) & 1) != 0;
                        gq = ((w >> 17) & 1) != 0;
                        gl[(sr - rb) * 16 + (sc - cb)] = l;
                        if (gp)
                            atomicOr(gm + (sr - rb), 1u << (sc - cb));
                        if (gq)
                            atomicOr(gm + 16 + (sc - cb), 1u << (sr - rb));
                    }
                    n_attempt += __popcll(__ballot(gp)) + __popcll(__ballot(gq));
                }
                if (pending)
                    offer_grids(2);
                pending = !pending;
            }
        }
        }
    }
    if (pending)
        offer_grids(1);
    flush_counters(a, n_pairs, n_gather, n_attempt, n_rescore, n_viol, maxg);
}

} // namespace

hipError_t launch_join(const Rows &R, int metric, int bf16, const RoundArgs &a, hipStream_t st)
{
    // member slots: four regions, each rounded up to a multiple of 4 (+12);
    // the BF16 tiles read 16 slots past a region start (+16); +4 spreads banks
    const int g_max = 3 * a.s + a.k;
    const int GS = r4(g_max) + 12 + 16 + 4;
    const bool use_bf = bf16 && metric != M_L1;
    const int wave_bytes = wave_lds_bytes(GS, a.s, a.k, use_bf);
    const size_t shmem = (size_t)wave_bytes * JOIN_WAVES;
    const int units = GS * (CH / 4);
    if (units > 8 * WAVE)
        return hipErrorInvalidValue;  // neighbourhood larger than the staging bound
    const bool small = units <= 4 * WAVE;
    const int64_t rows = a.alist ? a.n_active : a.n;  // list mode: the listed rows
    // graph mode: a fixed grid whose waves walk however many rows are listed
    // BF16: 8,192 waves, twice what the chip holds at once at 4 waves per
    // SIMD (with more, the later batches of waves end in a tail of waves with
    // few rows); FP32: 32,768, which measured faster for its kernels
    const int64_t cap = use_bf ? 8192 : 32768;
    const int64_t waves = a.dev ? 8192 : (rows < cap ? rows : cap);
    int64_t grid = (waves + JOIN_WAVES - 1) / JOIN_WAVES;
    if (grid < 1)
        grid = 1;
    auto go = [&](auto kern) -> hipError_t {
        if (shmem > 48 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)shmem);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(JOIN_WAVES * WAVE), shmem, st, R, a,
                           GS, wave_bytes);
        return hipSuccess;
    };
    hipError_t e;
#define KNNG_FP32_SET(KBV, MUV)                                                                 \
    (metric == M_L2 ? go(k_join<M_L2, KBV, MUV>)                                                \
                    : (metric == M_COS ? go(k_join<M_COS, KBV, MUV>) : go(k_join<M_L1, KBV, MUV>)))
#define KNNG_BF16_SET(KBV, MUV)                                                                 \
    (metric == M_L2 ? go(k_join_bf16<M_L2, KBV>) : go(k_join_bf16<M_COS, KBV>))
    if (bf16 && metric != M_L1) {
        if (a.k <= 16)
            e = small ? KNNG_BF16_SET(16, 8) : KNNG_BF16_SET(16, 12);
        else if (a.k <= 32)
            e = small ? KNNG_BF16_SET(32, 8) : KNNG_BF16_SET(32, 12);
        else
            e = small ? KNNG_BF16_SET(64, 8) : KNNG_BF16_SET(64, 12);
    } else {
        if (a.k <= 16)
            e = small ? KNNG_FP32_SET(16, 4) : KNNG_FP32_SET(16, 8);
        else if (a.k <= 32)
            e = small ? KNNG_FP32_SET(32, 4) : KNNG_FP32_SET(32, 8);
        else
            e = small ? KNNG_FP32_SET(64, 4) : KNNG_FP32_SET(64, 8);
    }
#undef KNNG_FP32_SET
#undef KNNG_BF16_SET
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
}

} // namespace knng
