// knng_brute.hip -- exhaustive comparison of row blocks: the brute-force cross
// merge that Zhao et al. describe in Section 1 (every pair of S1 x S2 is
// compared and offered to both lists), and the exact k-NN graph (Section 1's
// definition of G[i]).
//
// A workgroup owns TM = 64 rows of A and streams B in tiles of TN = 64 rows.
// Coordinates are staged through LDS in chunks of KC; each thread holds a
// 4 x 4 block of accumulators, updated in ascending coordinate order, so
// every distance is the canonical FP32 value.  Keys that beat the row's
// current k-th entry go to a per-row candidate buffer, merged into the row's
// sorted top-k list (in LDS) after each tile by one wave per row.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

constexpr int TM = 64, TN = 64, KC = 32;

template <int METRIC>
__global__ __launch_bounds__(256) void k_brute(Rows R, int64_t a_lo, int64_t a_hi, int64_t b_lo,
                                               int64_t b_hi, const uint64_t *__restrict__ init,
                                               int kin, int k, int exclude_self,
                                               int64_t out_base, int64_t id_base,
                                               int32_t *__restrict__ out_ids,
                                               float *__restrict__ out_dist)
{
    __shared__ float As[KC][TM];
    __shared__ float Bs[KC][TN];
    __shared__ uint64_t thr[TM];
    __shared__ int tcount[TM], ccount[TM];
    extern __shared__ uint64_t dyn64[];
    uint64_t *top = dyn64;            // TM x k
    uint64_t *cbuf = dyn64 + TM * k;  // TM x TN
    const int tid = threadIdx.x, lane = lane_id(), wv = tid / WAVE;
    const int tx = tid % 16, ty = tid / 16;
    const int64_t a0 = a_lo + (int64_t)blockIdx.x * TM;
    const int kk = kin < k ? kin : k;
    // initial lists (already sorted)
    for (int e = tid; e < TM * k; e += 256) {
        int r = e / k, j = e - r * k;
        uint64_t v = ~0ull;
        if (init && j < kk && a0 + r < a_hi) {
            v = init[(a0 + r - a_lo) * kin + j];
            v = key_empty(v) ? ~0ull : key_strip(v);
        }
        top[e] = v;
    }
    __syncthreads();
    if (tid < TM) {
        int c = 0;
        for (int j = 0; j < k; j++)
            c += top[tid * k + j] != ~0ull;  // valid entries are a sorted prefix
        tcount[tid] = c;
        ccount[tid] = 0;
    }
    __syncthreads();
    if (tid < TM)
        thr[tid] = tcount[tid] == k ? top[tid * k + k - 1] : ~0ull;
    float na[4], nb[4];
#pragma unroll
    for (int i = 0; i < 4; i++) {
        int64_t a = a0 + 4 * ty + i;
        na[i] = (METRIC == M_COS && a < a_hi) ? R.norm[R.phys(a)] : 0.0f;
    }
    for (int64_t b0 = b_lo; b0 < b_hi; b0 += TN) {
        float acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++)
                acc[i][j] = 0.0f;
        for (int t0 = 0; t0 < R.dp; t0 += KC) {
            const int kc = R.dp - t0 < KC ? R.dp - t0 : KC;
            const int q4 = kc / 4;
            __syncthreads();
            for (int e = tid; e < TM * q4; e += 256) {
                int r = e / q4, q = e - r * q4;
                int64_t a = a0 + r, b = b0 + r;
                float4 va = make_float4(0.f, 0.f, 0.f, 0.f), vb = va;
                if (a < a_hi)
                    va = *reinterpret_cast<const float4 *>(R.x + R.phys(a) * R.dp + t0 + 4 * q);
                if (b < b_hi)
                    vb = *reinterpret_cast<const float4 *>(R.x + R.phys(b) * R.dp + t0 + 4 * q);
                As[4 * q + 0][r] = va.x;
                As[4 * q + 1][r] = va.y;
                As[4 * q + 2][r] = va.z;
                As[4 * q + 3][r] = va.w;
                Bs[4 * q + 0][r] = vb.x;
                Bs[4 * q + 1][r] = vb.y;
                Bs[4 * q + 2][r] = vb.z;
                Bs[4 * q + 3][r] = vb.w;
            }
            __syncthreads();
            for (int t = 0; t < kc; t++) {
                float4 x = *reinterpret_cast<const float4 *>(&As[t][4 * ty]);
                float4 y = *reinterpret_cast<const float4 *>(&Bs[t][4 * tx]);
                float xa[4] = {x.x, x.y, x.z, x.w}, ya[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[i][j] = canon_step<METRIC>(acc[i][j], xa[i], ya[j]);
            }
        }
        // candidates that beat the current k-th entry of their row
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const int r = 4 * ty + i;
            const int64_t a = a0 + r;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int64_t b = b0 + 4 * tx + j;
                if (a >= a_hi || b >= b_hi || (exclude_self && a == b))
                    continue;
                float nbv = METRIC == M_COS ? R.norm[R.phys(b)] : 0.0f;
                float dv = canon_finish<METRIC>(acc[i][j], na[i], nbv);
                uint64_t key = make_key(dv, (uint32_t)(b - id_base), 0);
                if (key < thr[r]) {
                    int pos = atomicAdd(&ccount[r], 1);
                    cbuf[r * TN + pos] = key;
                }
            }
        }
        __syncthreads();
        // merge each row's candidates into its sorted top-k (one wave per row)
        for (int r = wv; r < TM; r += 4) {
            const int cc = ccount[r];
            if (cc == 0)
                continue;
            const int tc = tcount[r];
            const int tot = tc + cc;
            uint64_t e0 = lane < tot ? (lane < tc ? top[r * k + lane] : cbuf[r * TN + lane - tc])
                                     : ~0ull;
            int l1 = lane + WAVE;
            uint64_t e1 = l1 < tot ? (l1 < tc ? top[r * k + l1] : cbuf[r * TN + l1 - tc]) : ~0ull;
            int r0 = 0, r1 = 0;
            for (int j = 0; j < tot; j++) {
                uint64_t o = j < tc ? top[r * k + j] : cbuf[r * TN + j - tc];
                r0 += o < e0;
                r1 += o < e1;
            }
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_wave_barrier();
            if (lane < tot && r0 < k)
                top[r * k + r0] = e0;
            if (l1 < tot && r1 < k)
                top[r * k + r1] = e1;
            __builtin_amdgcn_wave_barrier();
            if (lane == 0) {
                int nt = tot < k ? tot : k;
                tcount[r] = nt;
                ccount[r] = 0;
            }
        }
        __syncthreads();
        if (tid < TM)
            thr[tid] = tcount[tid] == k ? top[tid * k + k - 1] : ~0ull;
    }
    __syncthreads();
    for (int e = tid; e < TM * k; e += 256) {
        int r = e / k, j = e - r * k;
        int64_t a = a0 + r;
        if (a >= a_hi)
            continue;
        int64_t o = (a - out_base) * k + j;
        if (j < tcount[r]) {
            uint64_t v = top[e];
            out_ids[o] = (int32_t)key_id(v);
            out_dist[o] = key_dist(v);
        } else {
            out_ids[o] = -1;
            out_dist[o] = __uint_as_float(0x7F800000u);
        }
    }
}

} // namespace

hipError_t launch_brute(const Rows &R, int metric, int64_t a_lo, int64_t a_hi, int64_t b_lo,
                        int64_t b_hi, const uint64_t *init, int kin, int k, int exclude_self,
                        int64_t out_base, int64_t id_base, int32_t *out_ids, float *out_dist,
                        hipStream_t st)
{
    if (a_hi <= a_lo)
        return hipSuccess;
    unsigned grid = (unsigned)((a_hi - a_lo + TM - 1) / TM);
    size_t shmem = (size_t)TM * k * 8 + (size_t)TM * TN * 8;
    auto go = [&](auto kern) -> hipError_t {
        if (shmem > 48 * 1024) {
            hipError_t e = hipFuncSetAttribute((const void *)kern,
                                               hipFuncAttributeMaxDynamicSharedMemorySize,
                                               (int)shmem);
            if (e != hipSuccess)
                return e;
        }
        hipLaunchKernelGGL(kern, dim3(grid), dim3(256), shmem, st, R, a_lo, a_hi, b_lo, b_hi,
                           init, kin, k, exclude_self, out_base, id_base, out_ids, out_dist);
        return hipSuccess;
    };
    hipError_t e = metric == M_L2 ? go(k_brute<M_L2>)
                                  : (metric == M_COS ? go(k_brute<M_COS>) : go(k_brute<M_L1>));
    if (e != hipSuccess)
        return e;
    return hipGetLastError();
}

} // namespace knng
