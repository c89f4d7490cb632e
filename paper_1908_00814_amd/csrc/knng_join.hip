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
// the lock-free bounded insert; a pair is first screened against the worst
// entry each list had at the start of the round (the worst only decreases
// during a round, so the screen never drops an edge that could stay).
//
// One workgroup of 256 threads owns one u at a time (grid-stride over u).
// The member vectors are staged in LDS in chunks of CH coordinates; each
// thread accumulates up to PPT pairs in registers across chunks, so every
// pair is evaluated in the canonical ascending-coordinate order.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

constexpr int JOIN_THREADS = 256;
constexpr int PPT = 4;  // pairs per thread per pass

__device__ __forceinline__ bool res_empty(uint64_t w) { return (uint32_t)w >= 0x40000000u; }

struct JoinSmem {
    int32_t grp[MAX_G];
    uint64_t gworst[MAX_G];
    int32_t cand[MAX_G];
    int nn, ng, np, nc;
    unsigned long long pairs, gathered;
    int maxg;
};

template <int METRIC>
__global__ __launch_bounds__(JOIN_THREADS) void k_join_f32(Rows R, RoundArgs a, int CH,
                                                           int g_max, int p_max)
{
    extern __shared__ float dyn[];
    __shared__ JoinSmem sm;
    float *vec = dyn;                                                   // g_max x (CH+1)
    uint16_t *plist = reinterpret_cast<uint16_t *>(dyn + g_max * (CH + 1));  // p_max
    const int tid = threadIdx.x;
    const int s = a.s, k = a.k;
    if (tid == 0) {
        sm.pairs = 0;
        sm.gathered = 0;
        sm.maxg = 0;
    }
    for (int64_t u = blockIdx.x; u < a.n; u += gridDim.x) {
        __syncthreads();
        if (tid == 0) {
            sm.nn = 0;
            sm.ng = 0;
            sm.np = 0;
            sm.nc = 0;
        }
        __syncthreads();
        // ---- NEW group: forward NEW sample and reverse NEW sources
        const int cnt_new = a.cnt_f[2 * u], cnt_old = a.cnt_f[2 * u + 1];
        int32_t cid = -1;
        if (tid < s) {
            if (tid < cnt_new)
                cid = a.new_f[u * s + tid];
        } else if (tid < 2 * s) {
            uint64_t w = a.rnew[u * s + (tid - s)];
            if (!res_empty(w))
                cid = (int32_t)(uint32_t)w;
        }
        if (tid < 2 * s)
            sm.cand[tid] = cid;
        __syncthreads();
        if (tid < 2 * s && cid >= 0) {
            bool dup = false;
            for (int j = 0; j < tid; j++)
                dup |= sm.cand[j] == cid;
            if (!dup)
                sm.grp[atomicAdd(&sm.nn, 1)] = cid;
        }
        __syncthreads();
        const int nn = sm.nn;
        if (nn == 0)
            continue;  // no NEW member: no pair to join at u
        // ---- OLD group: forward OLD sample and reverse OLD sources, minus NEW
        const int nco = k + s;
        cid = -1;
        if (tid < k) {
            if (tid < cnt_old)
                cid = a.old_f[u * k + tid];
        } else if (tid < nco) {
            uint64_t w = a.rold[u * s + (tid - k)];
            if (!res_empty(w))
                cid = (int32_t)(uint32_t)w;
        }
        if (tid < nco)
            sm.cand[tid] = cid;
        __syncthreads();
        if (tid < nco && cid >= 0) {
            bool drop = false;
            for (int j = 0; j < nn; j++)
                drop |= sm.grp[j] == cid;
            for (int j = 0; j < tid; j++)
                drop |= sm.cand[j] == cid;
            if (!drop)
                sm.grp[nn + atomicAdd(&sm.ng, 1)] = cid;
        }
        __syncthreads();
        const int G = nn + sm.ng;
        if (tid < G)
            sm.gworst[tid] = a.worst[sm.grp[tid]];
        // ---- admitted pairs (a in NEW, a < b): compacted list in LDS
        const int64_t p_all = (int64_t)nn * (G - 1) - (int64_t)nn * (nn - 1) / 2;
        for (int64_t idx = tid; idx < p_all; idx += JOIN_THREADS) {
            int ai = 0;
            int64_t off = 0;
            while (off + (G - 1 - ai) <= idx) {
                off += G - 1 - ai;
                ai++;
            }
            int bi = ai + 1 + (int)(idx - off);
            int32_t p = sm.grp[ai], q = sm.grp[bi];
            bool p1 = p < a.n1, q1 = q < a.n1;
            bool ok = a.joint ? !(p1 && q1) : (p1 != q1);
            if (ok) {
                int pos = atomicAdd(&sm.np, 1);
                plist[pos] = (uint16_t)((ai << 8) | bi);
            }
        }
        __syncthreads();
        const int np = sm.np;
        if (tid == 0) {
            sm.pairs += np;
            sm.gathered += G;
            sm.maxg = G > sm.maxg ? G : sm.maxg;
        }
        // ---- distances, PPT pairs per thread per pass
        for (int base = 0; base < np; base += JOIN_THREADS * PPT) {
            float acc[PPT];
            int pa[PPT], pb[PPT];
#pragma unroll
            for (int j = 0; j < PPT; j++) {
                acc[j] = 0.0f;
                int pi = base + tid + j * JOIN_THREADS;
                uint16_t e = pi < np ? plist[pi] : (uint16_t)0xFFFF;
                pa[j] = pi < np ? (e >> 8) : -1;
                pb[j] = pi < np ? (e & 0xFF) : -1;
            }
            for (int c0 = 0; c0 < R.dp; c0 += CH) {
                const int cw = R.dp - c0 < CH ? R.dp - c0 : CH;
                const int q4 = cw / 4;
                __syncthreads();
                for (int e = tid; e < G * q4; e += JOIN_THREADS) {
                    int m = e / q4, qq = e - m * q4;
                    float4 v = *reinterpret_cast<const float4 *>(R.x + (int64_t)sm.grp[m] * R.dp +
                                                                  c0 + 4 * qq);
                    float *dst = vec + m * (CH + 1) + 4 * qq;
                    dst[0] = v.x;
                    dst[1] = v.y;
                    dst[2] = v.z;
                    dst[3] = v.w;
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < PPT; j++) {
                    if (pa[j] < 0)
                        continue;
                    const float *x = vec + pa[j] * (CH + 1);
                    const float *y = vec + pb[j] * (CH + 1);
                    float t_acc = acc[j];
                    for (int t = 0; t < cw; t++)
                        t_acc = canon_step<METRIC>(t_acc, x[t], y[t]);
                    acc[j] = t_acc;
                }
            }
            // ---- screen and insert in both directions (UpdateNN)
#pragma unroll
            for (int j = 0; j < PPT; j++) {
                if (pa[j] < 0)
                    continue;
                int32_t p = sm.grp[pa[j]], q = sm.grp[pb[j]];
                float na = 0.0f, nb = 0.0f;
                if constexpr (METRIC == M_COS) {
                    na = R.norm[p];
                    nb = R.norm[q];
                }
                float l = canon_finish<METRIC>(acc[j], na, nb);
                uint64_t kp = make_key(l, (uint32_t)q, F_NEW | F_FRESH);
                uint64_t kq = make_key(l, (uint32_t)p, F_NEW | F_FRESH);
                if (kp < sm.gworst[pa[j]])
                    bounded_insert(a.L + (int64_t)p * k, k, kp, true, a.ctr + C_ERR);
                if (kq < sm.gworst[pb[j]])
                    bounded_insert(a.L + (int64_t)q * k, k, kq, true, a.ctr + C_ERR);
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        atomicAdd((unsigned long long *)(a.ctr + C_PAIRS), sm.pairs);
        atomicAdd((unsigned long long *)(a.ctr + C_EVALS), sm.pairs);
        atomicAdd((unsigned long long *)(a.ctr + C_GATHER), sm.gathered);
        atomicMax((unsigned long long *)(a.ctr + C_MAXG), (unsigned long long)sm.maxg);
    }
}

} // namespace

hipError_t launch_join(const Rows &R, int metric, int bf16, const RoundArgs &a, hipStream_t st)
{
    (void)bf16;
    const int g_max = 3 * a.s + a.k;
    const int nn_max = 2 * a.s;
    const int p_max = nn_max * (g_max - 1) - nn_max * (nn_max - 1) / 2;
    // chunk of coordinates staged per pass: at most ~40 KB of member vectors
    int ch = (40 * 1024 / 4) / g_max - 1;
    ch = ch / 4 * 4;
    if (ch > R.dp)
        ch = R.dp;
    if (ch < 4)
        ch = 4;
    size_t shmem = (size_t)g_max * (ch + 1) * 4 + (size_t)p_max * 2;
    shmem = (shmem + 15) / 16 * 16;
    int64_t grid = a.n < 8192 ? a.n : 8192;
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
        hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(JOIN_THREADS), shmem, st, R, a, ch,
                           g_max, p_max);
        return hipSuccess;
    };
    hipError_t e = metric == M_L2 ? go(k_join_f32<M_L2>)
                                  : (metric == M_COS ? go(k_join_f32<M_COS>) : go(k_join_f32<M_L1>));
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
}

} // namespace knng
