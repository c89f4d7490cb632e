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
// bound of each list's worst entry (set at the round start, lowered after
// every successful insert, read when u's neighbourhood is formed).  The worst
// entry only decreases during a round, so the screen never drops an edge that
// could stay.
//
// Layout.  One wave owns one u at a time (4 independent waves per workgroup,
// no workgroup barriers).  The members are placed in LDS in four regions, each
// starting at a multiple of 4:  [ newA | oldA | newB | oldB ]  (A = first set,
// B = second set).  The admitted pairs are then dense rectangles:
//   R1 = newA x (newB u oldB)      R2 = newB x oldA
//   R3 = newB x (newB u oldB), upper triangle on newB x newB (J-Merge only)
// Coordinates are staged chunk by chunk, transposed ([coordinate][member]),
// and each lane accumulates 2 x 4 register tiles of pairs in ascending
// coordinate order, so every distance is the canonical FP32 value.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

constexpr int JOIN_WAVES = 4;
constexpr int CH = 16;         // coordinates per staged chunk
constexpr int TPL = 1;         // 2x4 tiles per lane per batch
constexpr int OLD_CAP = MAX_K + MAX_S;  // OLD candidates per neighbourhood
constexpr int QCAP = 320;      // insert queue entries per wave

__device__ __forceinline__ bool res_empty(uint64_t w) { return (uint32_t)w >= 0x40000000u; }
__host__ __device__ __forceinline__ int r4(int x) { return (x + 3) & ~3; }

struct Regions {
    int nA, oA, nB, oB;           // member counts
    int offOA, offNB, offOB, GP;  // region starts and padded total
};

// tile t -> (row start, column start, rectangle); false past the last tile
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

// Drain a wave's insert queue: every entry is first re-checked against the
// live worst bound of its target list (one 8-byte load), the survivors are
// inserted.  Returns the number of inserts attempted (wave-uniform).
template <int KB>
__device__ inline int drain_queue(const uint64_t *qkey, const int32_t *qdst, int qn,
                                  const RoundArgs &a)
{
    int attempted = 0;
    for (int e0 = 0; e0 < qn; e0 += WAVE) {
        const int e = e0 + lane_id();
        bool go = false;
        uint64_t key = 0;
        int32_t dst = 0;
        if (e < qn) {
            key = qkey[e];
            dst = qdst[e];
            go = key < ld_agent(a.worst + dst);
        }
        attempted += __popcll(__ballot(go));
        if (go)
            bounded_insert<KB>(a.L + (int64_t)dst * a.k, a.k, key, true, a.worst + dst,
                               a.ctr + C_ERR);
    }
    return attempted;
}

template <int METRIC, int KB, int MAX_UNITS>
__global__ __launch_bounds__(JOIN_WAVES * WAVE) void k_join(Rows R, RoundArgs a, int GS,
                                                            int wave_bytes)
{
    extern __shared__ __align__(16) unsigned char dyn[];
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    unsigned char *base = dyn + (size_t)w * wave_bytes;
    float *vecT = reinterpret_cast<float *>(base);                    // CH x GS
    uint64_t *gw = reinterpret_cast<uint64_t *>(base + CH * GS * 4);  // GS
    int32_t *grp = reinterpret_cast<int32_t *>(gw + GS);              // GS
    float *gnorm = reinterpret_cast<float *>(grp + GS);               // GS (cosine)
    int32_t *tnew = reinterpret_cast<int32_t *>(gnorm + GS);          // 2 MAX_S
    int32_t *told = tnew + 2 * MAX_S;    // raw OLD candidates     (OLD_CAP)
    int32_t *toldA = told + OLD_CAP;     // accepted OLD, first set  (OLD_CAP)
    int32_t *toldB = toldA + OLD_CAP;    // accepted OLD, second set (OLD_CAP)
    uint64_t *qkey = reinterpret_cast<uint64_t *>(toldB + OLD_CAP);  // QCAP insert keys
    int32_t *qdst = reinterpret_cast<int32_t *>(qkey + QCAP);       // QCAP target rows

    const int s = a.s, k = a.k;
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t n_pairs = 0, n_gather = 0, n_attempt = 0;
    int maxg = 0;
    const int64_t nwaves = (int64_t)gridDim.x * JOIN_WAVES;
    for (int64_t u = (int64_t)blockIdx.x * JOIN_WAVES + w; u < a.n; u += nwaves) {
        __builtin_amdgcn_wave_barrier();
        // ---- NEW candidates: forward NEW sample (lanes < s), reverse NEW (s..2s)
        const int cnt_new = a.cnt_f[2 * u], cnt_old = a.cnt_f[2 * u + 1];
        int32_t cid = -1;
        if (lane < s) {
            if (lane < cnt_new)
                cid = a.new_f[u * s + lane];
        } else if (lane < 2 * s) {
            uint64_t wv = a.rnew[u * s + (lane - s)];
            if (!res_empty(wv))
                cid = (int32_t)(uint32_t)wv;
        }
        bool keep = cid >= 0;
        for (int j = 0; j < 2 * s; j++) {
            int32_t o = __shfl(cid, j, WAVE);
            keep = keep && !(j < lane && o == cid);
        }
        const bool isA = cid < a.n1;
        const uint64_t mA = __ballot(keep && isA), mB = __ballot(keep && !isA);
        const int nA = __popcll(mA), nB = __popcll(mB);
        if (nA + nB == 0)
            continue;  // no NEW member: no pair to join at u
        if (keep)
            tnew[isA ? __popcll(mA & below) : nA + __popcll(mB & below)] = cid;
        __builtin_amdgcn_wave_barrier();
        // ---- OLD candidates: forward OLD (c < k), reverse OLD (k <= c < k+s),
        //      minus NEW members and repeats
        const int nco = k + s;
        int oA = 0, oB = 0;
        for (int pass = 0; pass * WAVE < nco; pass++) {
            const int c = pass * WAVE + lane;
            int32_t oc = -1;
            if (c < k) {
                if (c < cnt_old)
                    oc = a.old_f[u * k + c];
            } else if (c < nco) {
                uint64_t wv = a.rold[u * s + (c - k)];
                if (!res_empty(wv))
                    oc = (int32_t)(uint32_t)wv;
            }
            if (c < nco)
                told[c] = oc;
            __builtin_amdgcn_wave_barrier();
            bool ok = oc >= 0;
            for (int j = 0; j < nA + nB && ok; j++)
                ok = tnew[j] != oc;
            for (int j = 0; j < c && ok; j++)
                ok = told[j] != oc;
            const bool oa = oc < a.n1;
            const uint64_t moA = __ballot(ok && oa), moB = __ballot(ok && !oa);
            if (ok) {
                if (oa)
                    toldA[oA + __popcll(moA & below)] = oc;
                else
                    toldB[oB + __popcll(moB & below)] = oc;
            }
            oA += __popcll(moA);
            oB += __popcll(moB);
            __builtin_amdgcn_wave_barrier();
        }
        // ---- regions [newA | oldA | newB | oldB], each start a multiple of 4
        Regions g;
        g.nA = nA;
        g.oA = oA;
        g.nB = nB;
        g.oB = oB;
        g.offOA = r4(nA);
        g.offNB = g.offOA + r4(oA);
        g.offOB = g.offNB + r4(nB);
        g.GP = g.offOB + r4(oB);
        const int G = nA + oA + nB + oB;
        for (int slot = lane; slot < g.GP; slot += WAVE) {
            int32_t id = -1;
            if (slot < nA)
                id = tnew[slot];
            else if (slot >= g.offOA && slot < g.offOA + oA)
                id = toldA[slot - g.offOA];
            else if (slot >= g.offNB && slot < g.offNB + nB)
                id = tnew[nA + (slot - g.offNB)];
            else if (slot >= g.offOB && slot < g.offOB + oB)
                id = toldB[slot - g.offOB];
            grp[slot] = id;
            gw[slot] = id >= 0 ? a.worst[id] : 0ull;
            if (METRIC == M_COS)
                gnorm[slot] = id >= 0 ? R.norm[id] : 1.0f;
        }
        __builtin_amdgcn_wave_barrier();
        n_gather += (uint64_t)G;
        maxg = G > maxg ? G : maxg;

        // ---- 2x4 tiles of the admitted rectangles
        const int colsB = g.GP - g.offNB;
        int T = ((nA + 1) / 2) * (colsB / 4) + ((nB + 1) / 2) * (r4(oA) / 4);
        if (a.joint)
            T += ((nB + 1) / 2) * (colsB / 4);
        constexpr int q4 = CH / 4;
        const int units = g.GP * q4;  // float4 units per staged chunk
        for (int tb = 0; tb < T; tb += WAVE * TPL) {
            float acc[TPL][2][4];
            int tr0[TPL], tc0[TPL], treg[TPL];
            bool tv[TPL];
#pragma unroll
            for (int i = 0; i < TPL; i++) {
                tv[i] = tile_of(tb + i * WAVE + lane, g, a.joint, tr0[i], tc0[i], treg[i]);
#pragma unroll
                for (int x = 0; x < 2; x++)
#pragma unroll
                    for (int y = 0; y < 4; y++)
                        acc[i][x][y] = 0.0f;
            }
            for (int c0 = 0; c0 < R.dp; c0 += CH) {
                // chunk -> LDS, transposed ([coordinate][member])
                __builtin_amdgcn_wave_barrier();
                float4 pre[MAX_UNITS];
#pragma unroll
                for (int j = 0; j < MAX_UNITS; j++) {
                    const int e = lane + j * WAVE;
                    pre[j] = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (e < units) {
                        const int m = e / q4, q = e - m * q4;
                        const int32_t id = grp[m];
                        if (id >= 0 && c0 + 4 * q < R.dp)
                            pre[j] = *reinterpret_cast<const float4 *>(R.x + (int64_t)id * R.dp +
                                                                       c0 + 4 * q);
                    }
                }
#pragma unroll
                for (int j = 0; j < MAX_UNITS; j++) {
                    const int e = lane + j * WAVE;
                    if (e < units) {
                        const int m = e / q4, q = e - m * q4;
                        vecT[(4 * q + 0) * GS + m] = pre[j].x;
                        vecT[(4 * q + 1) * GS + m] = pre[j].y;
                        vecT[(4 * q + 2) * GS + m] = pre[j].z;
                        vecT[(4 * q + 3) * GS + m] = pre[j].w;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                const int cw = R.dp - c0 < CH ? R.dp - c0 : CH;
#pragma unroll
                for (int i = 0; i < TPL; i++) {
                    if (!tv[i])
                        continue;
#pragma unroll 2
                    for (int t = 0; t < cw; t++) {
                        const float2 xr =
                            *reinterpret_cast<const float2 *>(vecT + t * GS + tr0[i]);
                        const float4 xc =
                            *reinterpret_cast<const float4 *>(vecT + t * GS + tc0[i]);
                        const float xrs[2] = {xr.x, xr.y};
                        const float xcs[4] = {xc.x, xc.y, xc.z, xc.w};
#pragma unroll
                        for (int x = 0; x < 2; x++)
#pragma unroll
                            for (int y = 0; y < 4; y++)
                                acc[i][x][y] = canon_step<METRIC>(acc[i][x][y], xrs[x], xcs[y]);
                    }
                }
            }
            // ---- screen; survivors go through the wave's insert queue, drained
            //      by all lanes together (UpdateNN in both directions)
            int qn = 0;
#pragma unroll
            for (int i = 0; i < TPL; i++) {
#pragma unroll
                for (int x = 0; x < 2; x++) {
                    const int r = tr0[i] + x;
#pragma unroll
                    for (int y = 0; y < 4; y++) {
                        const int c = tc0[i] + y;
                        const int32_t p = tv[i] ? grp[r] : -1;
                        const int32_t q = tv[i] ? grp[c] : -1;
                        const bool valid = p >= 0 && q >= 0 && !(treg[i] == 3 && c <= r);
                        n_pairs += valid;
                        float na = 0.0f, nb = 0.0f;
                        if (METRIC == M_COS && valid) {
                            na = gnorm[r];
                            nb = gnorm[c];
                        }
                        const float l = canon_finish<METRIC>(acc[i][x][y], na, nb);
                        const uint64_t kp = make_key(l, (uint32_t)q, F_NEW | F_FRESH);
                        const uint64_t kq = make_key(l, (uint32_t)p, F_NEW | F_FRESH);
                        const bool vp = valid && kp < gw[r];
                        const bool vq = valid && kq < gw[c];
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
                        if (qn > QCAP - 2 * WAVE) {
                            __builtin_amdgcn_wave_barrier();
                            n_attempt += drain_queue<KB>(qkey, qdst, qn, a);
                            qn = 0;
                            __builtin_amdgcn_wave_barrier();
                        }
                    }
                }
            }
            __builtin_amdgcn_wave_barrier();
            n_attempt += drain_queue<KB>(qkey, qdst, qn, a);
            __builtin_amdgcn_wave_barrier();
        }
    }
    // ---- counters: one atomic per wave
    uint64_t tp = n_pairs, ta = n_attempt;  // pairs: per lane; attempts: per wave
    for (int o = WAVE / 2; o > 0; o >>= 1)
        tp += __shfl_xor(tp, o, WAVE);
    if (lane == 0) {
        if (tp) {
            atomicAdd((unsigned long long *)(a.ctr + C_PAIRS), (unsigned long long)tp);
            atomicAdd((unsigned long long *)(a.ctr + C_EVALS), (unsigned long long)tp);
        }
        if (n_gather)
            atomicAdd((unsigned long long *)(a.ctr + C_GATHER), (unsigned long long)n_gather);
        if (ta)
            atomicAdd((unsigned long long *)(a.ctr + C_ATTEMPT), (unsigned long long)ta);
        if (maxg)
            atomicMax((unsigned long long *)(a.ctr + C_MAXG), (unsigned long long)maxg);
    }
}

} // namespace

hipError_t launch_join(const Rows &R, int metric, int bf16, const RoundArgs &a, hipStream_t st)
{
    (void)bf16;
    // member slots: four regions, each rounded up to a multiple of 4 (+12),
    // plus 4 to spread the LDS banks of consecutive coordinate rows
    const int g_max = 3 * a.s + a.k;
    const int GS = r4(g_max) + 16;
    int wave_bytes = CH * GS * 4 + GS * 8 + GS * 4 + GS * 4 + (2 * MAX_S + 3 * OLD_CAP) * 4 +
                     QCAP * 12;
    wave_bytes = (wave_bytes + 15) / 16 * 16;
    const size_t shmem = (size_t)wave_bytes * JOIN_WAVES;
    const int units = GS * (CH / 4);
    if (units > 12 * WAVE)
        return hipErrorInvalidValue;  // neighbourhood larger than the staging bound
    const bool small = units <= 8 * WAVE;
    const int64_t waves = a.n < 32768 ? a.n : 32768;
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
    auto by_metric = [&](auto l2, auto cs, auto l1) -> hipError_t {
        return metric == M_L2 ? go(l2) : (metric == M_COS ? go(cs) : go(l1));
    };
#define KNNG_JOIN_SET(KBV, MU) by_metric(k_join<M_L2, KBV, MU>, k_join<M_COS, KBV, MU>, k_join<M_L1, KBV, MU>)
    hipError_t e;
    if (a.k <= 16)
        e = small ? KNNG_JOIN_SET(16, 8) : KNNG_JOIN_SET(16, 12);
    else if (a.k <= 32)
        e = small ? KNNG_JOIN_SET(32, 8) : KNNG_JOIN_SET(32, 12);
    else
        e = small ? KNNG_JOIN_SET(64, 8) : KNNG_JOIN_SET(64, 12);
#undef KNNG_JOIN_SET
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
}

} // namespace knng
