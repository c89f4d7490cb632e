// knng_prep.hip -- input layout, Divide/Append/Initialize and Merge-and-Sort.
//
// Steps of Algorithms 1 and 2 (Zhao et al., "On the Merge of k-NN Graph",
// Sections 3.1-3.2) that run once per call: building the device layout,
// reading the input graphs, the Divide/Append (or Initialize) steps before the
// repeat loop, and the final Merge and Sort with the set-aside rear lists.
#include "knng_common.h"
#include "knng_internal.h"

namespace knng {

namespace {

// Concatenate the two sets into one zero-padded fp32 array and, for the BF16
// path, a zero-padded bf16 copy with rows of db elements plus, per row
// (se[r * se_stride]), the squared norm of the bf16-rounded row and an upper
// bound of |x - bf16(x)|.  One wave per row at a time (rows wave-strided),
// lane l taking coordinates l, l + 64, ...; the two per-row values are wave
// sums.  A row whose coordinates are integers in [0, 256] and whose squared
// norm is below 2^23 gets the exactness certificate (the bound -0.0): its
// partial sums are integers below 2^24, so its squared norm is exact in any
// order of summation.  For two certified rows p, q every partial dot product
// is at most |p||q| < 2^23 and every canonical partial sum of (p_t - q_t)^2 at
// most |p|^2 + |q|^2 < 2^24; all are integers, so the bf16 evaluation and the
// canonical FP32 one are exact and equal bit for bit.  Other rows use the
// norm only under the screen's margin, which bounds the rounding of any
// order of summation (a sum of dp terms).
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ x1, int64_t n1,
                                              const float *__restrict__ x2, int64_t n2, int d,
                                              int dp, float *__restrict__ x, int db,
                                              uint16_t *__restrict__ xb, float2 *__restrict__ se,
                                              int se_stride, uint64_t *ctr)
{
    const int lane = lane_id();
    const int64_t n = n1 + n2;
    const int w = xb && db > dp ? db : dp;
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    uint32_t bad = 0;
    for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE; r < n;
         r += nwaves) {
        const float *src = r < n1 ? x1 + r * d : x2 + (r - n1) * d;
        float acc = 0.0f;
        double e2 = 0.0;
        bool integral = true;  // every coordinate an integer in [0, 256]
        for (int c = lane; c < w; c += WAVE) {
            float v = 0.0f;
            if (c < d) {
                v = src[c];
                if (!isfinite(v)) {
                    bad = 1;
                    v = 0.0f;
                }
            }
            if (c < dp)
                x[r * dp + c] = v;
            if (xb && c < db) {
                const uint16_t h = f32_to_bf16(v);
                xb[r * db + c] = h;
                const float b = bf16_to_f32(h);
                acc = __builtin_fmaf(b, b, acc);
                const double dd = (double)v - (double)b;
                e2 += dd * dd;
                integral = integral && v == rintf(v) && v >= 0.0f && v <= 256.0f;
            }
        }
        if (se) {
            for (int o = WAVE / 2; o > 0; o >>= 1) {
                acc += __shfl_xor(acc, o, WAVE);
                e2 += __shfl_xor(e2, o, WAVE);
            }
            const bool cert = __ballot(!integral) == 0ull && acc < 0x1p23f;
            if (lane == 0) {
                // the FP64 sum of exact squares is within (dp * 2^-53)
                // relative; inflate it and the sqrt so the fp32 value is an
                // upper bound
                float e = __double2float_ru(__builtin_sqrt(e2 * (1.0 + 0x1p-36)) * (1.0 + 0x1p-50));
                se[r * se_stride] = make_float2(acc, cert ? -0.0f : e);
            }
        }
    }
    if (bad)
        atomicOr((unsigned long long *)(ctr + C_ERR), (unsigned long long)ERR_NONFINITE);
}

// canonical norms (ascending fused accumulation, correctly rounded sqrt)
__global__ void k_norms(const float *__restrict__ x, int64_t n, int dp, float *__restrict__ norm,
                        int check_zero, uint64_t *ctr)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n)
        return;
    const float4 *p = reinterpret_cast<const float4 *>(x + r * dp);
    float acc = 0.0f;
    for (int t = 0; t < dp / 4; t++) {
        float4 v = p[t];
        acc = __builtin_fmaf(v.x, v.x, acc);
        acc = __builtin_fmaf(v.y, v.y, acc);
        acc = __builtin_fmaf(v.z, v.z, acc);
        acc = __builtin_fmaf(v.w, v.w, acc);
    }
    float nr = __builtin_sqrtf(acc);  // correctly rounded (see build flags)
    norm[r] = nr;
    if (check_zero && !(nr > 0.0f))
        atomicOr((unsigned long long *)(ctr + C_ERR), (unsigned long long)ERR_ZERO_NORM);
}

// one wave per input row: local ids -> global keys, validated, sorted
template <int METRIC>
__global__ __launch_bounds__(256) void k_prep_input(Rows R, int64_t row0, int64_t nrows,
                                                    int64_t id_offset, int64_t n_local,
                                                    const int32_t *__restrict__ ids,
                                                    const float *__restrict__ dist, int kin,
                                                    int gstride, uint64_t *__restrict__ gin,
                                                    uint64_t *ctr)
{
    const int lane = lane_id();
    const int64_t wid = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    if (wid >= nrows)
        return;
    const int64_t r = row0 + wid;
    uint32_t err = 0;
    bool act = lane < kin;
    int64_t g = -1;
    uint64_t key = ~0ull;
    if (act) {
        int32_t loc = ids[wid * kin + lane];
        if (loc < 0 || loc >= n_local) {
            err |= ERR_ID_RANGE;
        } else {
            g = loc + id_offset;
            if (g == r)
                err |= ERR_SELF;
        }
    }
    // l2 between rows certified exact (integer coordinates in [0, 256],
    // squared norm below 2^23): every partial sum of squared differences is an
    // integer below 2^24, so any order gives the canonical value; two lanes
    // then share a distance, each summing half of the bf16 row
    float dsplit = 0.0f;
    bool split = false;
    if (METRIC == M_L2 && !dist && R.se && kin <= WAVE / 2 &&
        signbit(R.se[R.phys(r) * R.se_stride].y)) {
        const int q = lane >> 1, part = lane & 1;
        const int64_t gq = __shfl(g, q, WAVE);
        const bool mine = q < kin && gq >= 0;
        if (__ballot(mine && !signbit(R.se[R.phys(gq) * R.se_stride].y)) == 0ull) {
            split = true;
            const int half = R.db / 2;  // a multiple of 16
            const uint16_t *xr = R.xb + R.phys(r) * R.db + part * half;
            const uint16_t *xg = R.xb + R.phys(mine ? gq : r) * R.db + part * half;
            float acc = 0.0f;
            for (int c = 0; c < half; c += 8) {
                const uint4 pr = *reinterpret_cast<const uint4 *>(xr + c);
                const uint4 pg = *reinterpret_cast<const uint4 *>(xg + c);
                const uint32_t wr[4] = {pr.x, pr.y, pr.z, pr.w}, wg[4] = {pg.x, pg.y, pg.z, pg.w};
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const float d0 = __uint_as_float(wr[t] << 16) - __uint_as_float(wg[t] << 16);
                    const float d1 = __uint_as_float(wr[t] & 0xFFFF0000u) -
                                     __uint_as_float(wg[t] & 0xFFFF0000u);
                    acc += d0 * d0;
                    acc += d1 * d1;
                }
            }
            acc += __shfl_xor(acc, 1, WAVE);
            dsplit = __shfl(acc, 2 * lane, WAVE);
        }
    }
    if (act) {
        float dv = 0.0f;
        if (g >= 0) {
            if (dist) {
                dv = dist[wid * kin + lane];
                if (!(dv >= 0.0f) || isinf(dv))
                    err |= ERR_BAD_DIST;
            } else if (split) {
                dv = dsplit;
            } else {
                const float *a = R.x + R.phys(r) * R.dp, *b = R.x + R.phys(g) * R.dp;
                float na = R.norm ? R.norm[R.phys(r)] : 0.0f;
                float nb = R.norm ? R.norm[R.phys(g)] : 0.0f;
                dv = canon_dist<METRIC>(a, b, R.dp, na, nb);
            }
        }
        key = make_key(dv > 0.0f ? dv : 0.0f, (uint32_t)(g < 0 ? 0 : g), 0);
    }
    // duplicates, and the order of recomputed distances (ids are below 2^31)
    int rank = 0;
    const int32_t g32 = (int32_t)g;
    for (int j = 0; j < kin; j++) {
        const int32_t og = __builtin_amdgcn_readlane(g32, j);
        if (act && j != lane && og == g32 && g >= 0)
            err |= ERR_DUP;
    }
    if (!dist) {
        for (int j = 0; j < kin; j++) {
            const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, j);
            const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), j);
            if (act && (((uint64_t)hi << 32) | lo) < key)
                rank++;
        }
    }
    if (dist) {
        uint64_t prev = __shfl_up(key, 1, WAVE);
        if (act && lane > 0 && !(prev < key))
            err |= ERR_UNSORTED;
        rank = lane;
    }
    if (act && err == 0)
        gin[r * gstride + rank] = key;
    if (lane >= kin && lane < gstride)
        gin[r * gstride + lane] = ~0ull;  // padding of a shorter row
    if (err)
        atomicOr((unsigned long long *)(ctr + C_ERR), (unsigned long long)err);
}

// one wave per row: Divide + Append (rows with a list) or Initialize (raw)
template <int METRIC>
__global__ __launch_bounds__(256) void k_init(Rows R, InitArgs a)
{
    __shared__ int32_t picked_all[4][MAX_K];
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    int32_t *picked = picked_all[w];
    uint64_t evals = 0;
    int n0 = 0;
    auto init_row = [&](const int64_t i) {
    __builtin_amdgcn_wave_barrier();
    const bool has_list = !a.joint || i < a.n1;
    int first, m;
    uint32_t N;
    int64_t skip, cand_off;
    if (has_list) {
        // Append: k - k1 samples of the other set (S-Merge) / of the raw set
        int64_t n_other = a.joint ? a.n - a.n1 : (i < a.n1 ? a.n - a.n1 : a.n1);
        N = (uint32_t)n_other;
        cand_off = a.joint ? a.n1 : (i < a.n1 ? a.n1 : 0);
        skip = -1;
        first = a.k1;
        m = (int64_t)(a.k - a.k1) < n_other ? a.k - a.k1 : (int)n_other;
        if (a.joint && !selected_base_row(a.seed, a.balanced, i, a.n1, a.n - a.n1)) {
            // balanced append, row not selected: the whole list stays (OLD)
            first = a.kin < a.k ? a.kin : a.k;
            m = 0;
        }
    } else {
        // Initialize: k samples of S u raw, self excluded
        N = (uint32_t)a.n;
        cand_off = 0;
        skip = i;
        first = 0;
        m = (int64_t)a.k < a.n - 1 ? a.k : (int)(a.n - 1);
    }
    const uint32_t tag = has_list ? TAG_APPEND : TAG_INIT;
    const uint32_t avail = N - (skip >= 0 ? 1u : 0u);
    // m distinct draws in draw order (the first m distinct values of the stream)
    int got = 0;
    if (m == 0) {
    } else if ((uint32_t)m >= avail) {
        if (lane < m)
            picked[lane] = (int32_t)((skip >= 0 && lane >= skip) ? lane + 1 : lane);
        got = m;
    } else {
        // the first m draws, when they are distinct, are the answer
        {
            const uint64_t h = hash5(a.seed, tag, (uint64_t)i, (uint64_t)lane, 0);
            uint32_t v;
            if (skip >= 0) {
                v = draw_below(h, N - 1);
                if ((int64_t)v >= skip)
                    v++;
            } else {
                v = draw_below(h, N);
            }
            bool dup = false;
            for (int j = 0; j < m; j++)
                dup |= j < lane && (uint32_t)__builtin_amdgcn_readlane((int)v, j) == v;
            if (__ballot(lane < m && dup) == 0ull) {
                if (lane < m)
                    picked[lane] = (int32_t)v;
                got = m;
            }
        }
        const int64_t budget = 64 * (int64_t)m + 4096;
        const uint64_t below = (1ull << lane) - 1ull;
        for (int64_t base = 0; got < m && base < budget; base += WAVE) {
            int64_t t = base + lane;
            bool valid = t < budget;
            uint64_t h = hash5(a.seed, tag, (uint64_t)i, (uint64_t)t, 0);
            uint32_t v;
            if (skip >= 0) {
                v = draw_below(h, N - 1);
                if ((int64_t)v >= skip)
                    v++;
            } else {
                v = draw_below(h, N);
            }
            bool dup = false;
            for (int j = 0; j < WAVE; j++) {
                uint32_t o = __shfl(v, j, WAVE);
                if (j < lane && o == v)
                    dup = true;
            }
            for (int q = 0; q < got; q++)
                if ((uint32_t)picked[q] == v)
                    dup = true;
            bool acc = valid && !dup;
            uint64_t mask = __ballot(acc);
            int pos = got + __popcll(mask & below);
            if (acc && pos < m)
                picked[pos] = (int32_t)v;
            int add = __popcll(mask);
            got = got + add < m ? got + add : m;
            __builtin_amdgcn_wave_barrier();
        }
        if (got < m && lane == 0) {
            // draw budget exhausted: smallest values not yet taken
            for (uint32_t v = 0; v < N && got < m; v++) {
                if ((int64_t)v == skip)
                    continue;
                bool dup = false;
                for (int q = 0; q < got; q++)
                    if ((uint32_t)picked[q] == v)
                        dup = true;
                if (!dup)
                    picked[got++] = (int32_t)v;
            }
        }
        got = __shfl(got, 0, WAVE);
    }
    __builtin_amdgcn_wave_barrier();
    // l2 between rows certified exact (integer coordinates in [0, 256],
    // squared norm below 2^23): every partial sum of squared differences is an
    // integer below 2^24, so any order of summation gives the canonical value;
    // four lanes then share a distance, each summing a quarter of the bf16 row
    float dsplit = 0.0f;
    bool split = false;
    if (METRIC == M_L2 && R.se && m > 0 && m <= WAVE / 4 &&
        signbit(R.se[R.phys(i) * R.se_stride].y)) {
        const int q = lane >> 2, part = lane & 3;
        const bool mine = q < m;
        const int64_t g = mine ? picked[q] + cand_off : i;
        const bool cert = signbit(R.se[R.phys(g) * R.se_stride].y);
        if (__ballot(mine && !cert) == 0ull) {
            split = true;
            const int per = R.db / 4;  // a multiple of 8
            const uint16_t *xi = R.xb + R.phys(i) * R.db + part * per;
            const uint16_t *xg = R.xb + R.phys(g) * R.db + part * per;
            float acc = 0.0f;
            for (int c = 0; c < per; c += 8) {
                const uint4 pi = *reinterpret_cast<const uint4 *>(xi + c);
                const uint4 pg = *reinterpret_cast<const uint4 *>(xg + c);
                const uint32_t wi[4] = {pi.x, pi.y, pi.z, pi.w}, wg[4] = {pg.x, pg.y, pg.z, pg.w};
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const float d0 = __uint_as_float(wi[t] << 16) - __uint_as_float(wg[t] << 16);
                    const float d1 = __uint_as_float(wi[t] & 0xFFFF0000u) -
                                     __uint_as_float(wg[t] & 0xFFFF0000u);
                    acc += d0 * d0;
                    acc += d1 * d1;
                }
            }
            acc += __shfl_xor(acc, 1, WAVE);
            acc += __shfl_xor(acc, 2, WAVE);
            // list lane first + q takes group q's sum
            dsplit = __shfl(acc, 4 * (lane - first), WAVE);
        }
    }
    uint64_t key = 0;
    if (lane < a.k) {
        if (lane < first) {
            key = a.gin[i * a.kin + lane];  // kept entries start OLD
            key = key_empty(key) ? empty_key(lane) : key_strip(key);
        } else if (lane < first + m) {
            int64_t g = picked[lane - first] + cand_off;
            float dv;
            if (split) {
                dv = dsplit;
            } else {
                float na = R.norm ? R.norm[R.phys(i)] : 0.0f,
                      nb = R.norm ? R.norm[R.phys(g)] : 0.0f;
                dv = canon_dist<METRIC>(R.x + R.phys(i) * R.dp, R.x + R.phys(g) * R.dp, R.dp, na,
                                        nb);
            }
            key = make_key(dv, (uint32_t)g, F_NEW);
        } else {
            key = empty_key(lane);
        }
        a.L[i * a.k + lane] = key;
    }
    // the list's maximum word (an empty slot when the list is not full); the
    // row is sampled in round 0 iff it holds a NEW entry
    const uint64_t wv = wave_max_u64(key_empty(key) ? key : key_strip(key));
    if (lane == 0) {
        a.worst[i * a.ws] = wv;
        a.dtag[i] = m > 0 ? a.tag0 : a.tag0 - 1;
        a.atag[i] = a.tag0 - 1;
    }
    evals += (uint64_t)m;
    n0 += m > 0;
    __builtin_amdgcn_wave_barrier();
    };
    if (!a.incremental) {
        const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
        for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE; i < a.n;
             i += nwaves)
            init_row(i);
    } else {
        // unselected base rows already hold their initial state
        FOR_ROWS_IF(i, a.n, [&](int64_t r) {
            return r >= a.n1 || selected_base_row(a.seed, a.balanced, r, a.n1, a.n - a.n1);
        })
        init_row(i);
    }
    // one atomic per wave for the distance evaluations of all its rows
    if (lane == 0 && evals)
        atomicAdd((unsigned long long *)(a.ctr + C_EVALS), (unsigned long long)evals);
    if (lane == 0 && n0)
        atomicAdd((unsigned long long *)(a.ctr + C_N0), (unsigned long long)n0);
}

// top k of row i's list and its rear part, deduplicated, by a group of G
// lanes (G = 64: one row per wave, G = 32: two); cand and kept are the
// group's 2 x G words of LDS; live: the row exists (a group past the last row
// takes part in the group sum only)
template <int G>
__device__ inline void final_row(const FinalArgs &a, const int64_t i, const bool live,
                                 uint64_t *cand, uint64_t *kept)
{
    const uint64_t *__restrict__ L = a.L;
    const uint64_t *gin = a.gin;
    const int k = a.k, kin = a.kin;
    int32_t *out_ids = a.out_ids;
    float *out_dist = a.out_dist;
    uint64_t *out_keys = a.out_keys;  // may alias gin: row i is read before it is written
    const int lane = lane_id() % G;
    __builtin_amdgcn_wave_barrier();  // the previous row's reads of cand / kept are done
    int rear0 = a.k1;
    if (!selected_base_row(a.seed, a.balanced, i, a.rows_with_rear, a.n_raw))
        rear0 = kin < k ? kin : k;
    const int nrear = live && i < a.rows_with_rear ? kin - rear0 : 0;
    uint64_t c0 = live && lane < k ? key_strip(L[i * k + lane]) : ~0ull;
    uint64_t c1 = lane < nrear ? key_strip(gin[i * kin + rear0 + lane]) : ~0ull;
    if (key_empty(c0))
        c0 = ~0ull;
    if (key_empty(c1))
        c1 = ~0ull;  // padding of rows shorter than the row stride
    cand[lane] = c0;
    cand[G + lane] = c1;
    __builtin_amdgcn_wave_barrier();
    // keep the first occurrence of each entry (only slots [0, k) and
    // [G, G + nrear) hold candidates; the rest hold ~0, which matches and
    // outranks nothing)
    bool v0 = c0 != ~0ull, v1 = c1 != ~0ull;
    for (int j = 0; j < k; j++) {
        const uint64_t o = cand[j];
        if (o == c0 && j < lane)
            v0 = false;
        if (o == c1)
            v1 = false;
    }
    for (int j = G; j < G + nrear; j++) {
        const uint64_t o = cand[j];
        if (o == c1 && j < G + lane)
            v1 = false;
    }
    kept[lane] = v0 ? c0 : ~0ull;
    kept[G + lane] = v1 ? c1 : ~0ull;
    __builtin_amdgcn_wave_barrier();
    int r0 = 0, r1 = 0;
    for (int j = 0; j < k; j++) {
        const uint64_t o = kept[j];
        r0 += o < c0;
        r1 += o < c1;
    }
    for (int j = G; j < G + nrear; j++) {
        const uint64_t o = kept[j];
        r0 += o < c0;
        r1 += o < c1;
    }
    int nvalid = (int)v0 + (int)v1;
    for (int o = G / 2; o > 0; o >>= 1)
        nvalid += __shfl_xor(nvalid, o, WAVE);
    if (!live)
        return;
    if (out_ids) {
        if (v0 && r0 < k) {
            out_ids[i * k + r0] = (int32_t)key_id(c0);
            out_dist[i * k + r0] = key_dist(c0);
        }
        if (v1 && r1 < k) {
            out_ids[i * k + r1] = (int32_t)key_id(c1);
            out_dist[i * k + r1] = key_dist(c1);
        }
        if (lane >= nvalid && lane < k) {
            out_ids[i * k + lane] = -1;
            out_dist[i * k + lane] = __uint_as_float(0x7F800000u);
        }
    }
    if (out_keys) {
        __builtin_amdgcn_wave_barrier();  // every read of row i precedes its writes
        if (v0 && r0 < k)
            out_keys[i * kin + r0] = c0;
        if (v1 && r1 < k)
            out_keys[i * kin + r1] = c1;
        if (lane >= (nvalid < k ? nvalid : k) && lane < kin)
            out_keys[i * kin + lane] = ~0ull;
    }
}

// G = 64: one wave per row, or with a.touched a wave-strided walk over the
// rows that held a NEW entry and the rows without a rear part; G = 32: two
// rows per wave, for lists and kept input entries of at most 32 each
template <int G>
__global__ __launch_bounds__(256) void k_final(FinalArgs a)
{
    __shared__ uint64_t cand_all[4][2 * WAVE];
    __shared__ uint64_t kept_all[4][2 * WAVE];
    const int w = threadIdx.x / WAVE;
    const int g = (threadIdx.x % WAVE) / G;
    uint64_t *cand = cand_all[w] + g * 2 * G;
    uint64_t *kept = kept_all[w] + g * 2 * G;
    if constexpr (G == WAVE) {
        if (a.touched) {
            const int32_t *touched = a.touched;
            FOR_ROWS_IF(i, a.n, [&](int64_t r) {
                return r >= a.rows_with_rear || touched[r] >= a.tag0;
            })
            final_row<WAVE>(a, i, true, cand, kept);
            return;
        }
    }
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE * (WAVE / G) + g;
    final_row<G>(a, i, i < a.n, cand, kept);
}

// commit of row i of one request into the resident lists (one wave)
template <int KB>
__device__ inline void commit_row(const CommitArgs &a, const int64_t i)
{
    const int lane = lane_id();
    const uint64_t e = lane < a.k ? a.out[i * a.gs + lane] : ~0ull;
    const bool real = lane < a.k && !key_empty(e);
    const uint32_t id = key_id(e);
    const uint32_t gid = id < a.m_base ? id : (uint32_t)(a.first + (id - a.m_base));
    const uint64_t ge = make_key(key_dist(e), gid, 0);
    if (real && id >= a.m_base + a.n_req) {
        raise_err(a.ctr + C_ERR, ERR_ROW_COMMIT);
        return;
    }
    if (i < a.m_base) {
        if (!real || id < a.m_base)
            return;
        bounded_insert<KB>(a.res + i * a.k, a.k, ge, DUP_ID, nullptr, a.ctr + C_ERR);
    } else if (lane < a.k) {
        a.res[(a.first + (i - a.m_base)) * a.k + lane] = real ? ge : empty_key(lane);
    }
}

// Rows of the base that never held a NEW entry were not written by the
// merge's Merge and Sort and are skipped before their entries are read: a
// wave-strided walk over the touched base rows and the request's rows.
template <int KB>
__global__ __launch_bounds__(256) void k_commit(CommitArgs a)
{
    const int32_t *touched = a.touched;
    FOR_ROWS_IF(i, a.m_base + a.n_req, [&](int64_t r) {
        return r >= a.m_base || touched[r] >= a.tag0;
    })
    commit_row<KB>(a, i);
}

// Restore of the rows an earlier merge changed (see launch_restore)
__global__ __launch_bounds__(256) void k_restore(uint64_t *L, uint64_t *worst, const int32_t *dtag,
                                                 const uint64_t *gin, int kin, int k, int64_t m,
                                                 int32_t since)
{
    const int lane = lane_id();
    const int first = kin < k ? kin : k;
    FOR_ROWS_IF(u, m, [&](int64_t r) { return dtag[r] >= since; })
    {
        uint64_t key = 0;
        if (lane < k) {
            if (lane < first) {
                key = gin[u * kin + lane];
                key = key_empty(key) ? empty_key(lane) : key_strip(key);
            } else {
                key = empty_key(lane);
            }
            L[u * k + lane] = key;
        }
        const uint64_t wv = wave_max_u64(key_empty(key) ? key : key_strip(key));
        if (lane == 0)
            worst[u] = wv;
    }
}

// one wave per row: sort k keys by value (empties last)
__global__ __launch_bounds__(256) void k_sort_rows(const uint64_t *__restrict__ src, int sst,
                                                   int64_t n, int k, uint64_t *dst, int dstst,
                                                   int32_t *ids, float *dist)
{
    const int lane = lane_id();
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    if (i >= n)
        return;
    uint64_t v = lane < k ? src[i * sst + lane] : ~0ull;
    if (lane < k && key_empty(v))
        v = ~0ull;
    v = v == ~0ull ? v : key_strip(v);
    int rank = 0;
    for (int j = 0; j < k; j++) {
        const uint64_t o = __shfl(v, j, WAVE);
        rank += o < v || (o == v && j < lane);
    }
    if (lane < k) {
        const bool empty = v == ~0ull;
        if (dst)
            dst[i * dstst + rank] = empty ? empty_key(rank) : v;
        if (ids) {
            ids[i * k + rank] = empty ? -1 : (int32_t)key_id(v);
            dist[i * k + rank] = empty ? __uint_as_float(0x7F800000u) : key_dist(v);
        }
    }
    if (dst && lane >= k && lane < dstst)
        dst[i * dstst + lane] = empty_key(lane);
}

// position i -> row: Feistel network with cycle walking (a bijection of
// [0, n) for any n; Black and Rogaway's construction for arbitrary domains).
// Round r maps (L, R) to (R, L ^ F_r(R)) with F_r(R) the low `half` bits of
// H(seed, PERM, r, R).
__device__ inline uint32_t perm_position(uint64_t seed, uint32_t i, uint32_t n, int half)
{
    const uint32_t mask = (1u << half) - 1u;
    uint32_t x = i;
    do {
        uint32_t L = x >> half, R = x & mask;
        for (int r = 0; r < 4; r++) {
            const uint32_t f =
                (uint32_t)hash5(seed, TAG_PERM, (uint64_t)r, (uint64_t)R, 0) & mask;
            const uint32_t t = L ^ f;
            L = R;
            R = t;
        }
        x = (L << half) | R;
    } while (x >= n);  // i < n lies on the cycle, so the walk ends
    return x;
}

__global__ __launch_bounds__(256) void k_perm(uint64_t seed, int64_t n, int half, int32_t *perm)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n)
        perm[i] = (int32_t)perm_position(seed, (uint32_t)i, (uint32_t)n, half);
}

__global__ __launch_bounds__(256) void k_gather_rows(const float *__restrict__ x, int64_t n, int d,
                                                     const int32_t *__restrict__ perm,
                                                     float *__restrict__ xp)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * d;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / d;
        xp[e] = x[(int64_t)perm[i] * d + (e - i * d)];
    }
}

// one wave per position
__global__ __launch_bounds__(256) void k_unpermute(const int32_t *__restrict__ ids,
                                                   const float *__restrict__ dist, int64_t n,
                                                   int k, const int32_t *__restrict__ perm,
                                                   int32_t *out_ids, float *out_dist)
{
    const int lane = lane_id();
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;
    if (i >= n)
        return;
    uint64_t key = ~0ull;
    if (lane < k) {
        const int32_t id = ids[i * k + lane];
        if (id >= 0 && id < n)
            key = make_key(dist[i * k + lane], (uint32_t)perm[id], 0);
    }
    int rank = 0;
    for (int j = 0; j < k; j++) {
        const uint64_t o = __shfl(key, j, WAVE);
        rank += o < key || (o == key && j < lane);
    }
    if (lane < k) {
        const int64_t row = perm[i];
        const bool real = key != ~0ull;
        out_ids[row * k + rank] = real ? (int32_t)key_id(key) : -1;
        out_dist[row * k + rank] = real ? key_dist(key) : __uint_as_float(0x7F800000u);
    }
}

__global__ void k_zero(uint64_t *p, int words)
{
    int t = threadIdx.x;
    if (t < words)
        p[t] = 0;
}

inline unsigned grid_for(int64_t items, int per_block)
{
    int64_t g = (items + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

} // namespace

hipError_t launch_pack(const float *x1, int64_t n1, const float *x2, int64_t n2, int d, int dp,
                       float *x, int db, uint16_t *xb, float2 *se, int se_stride, uint64_t *ctr,
                       hipStream_t st)
{
    // at most 2,048 blocks of 4 waves, each wave walking rows
    unsigned g = grid_for(n1 + n2, 4);
    if (g > 2048u)
        g = 2048u;
    hipLaunchKernelGGL(k_pack, dim3(g), dim3(256), 0, st, x1, n1, x2, n2, d, dp, x, db, xb, se,
                       se_stride, ctr);
    return hipGetLastError();
}

hipError_t launch_norms(const float *x, int64_t n, int dp, float *norm, int check_zero,
                        uint64_t *ctr, hipStream_t st)
{
    hipLaunchKernelGGL(k_norms, dim3(grid_for(n, 256)), dim3(256), 0, st, x, n, dp, norm,
                       check_zero, ctr);
    return hipGetLastError();
}

hipError_t launch_prep_input(const Rows &R, int metric, int64_t row0, int64_t nrows,
                             int64_t id_offset, int64_t n_local, const int32_t *ids,
                             const float *dist, int kin, int gstride, uint64_t *gin,
                             uint64_t *ctr, hipStream_t st)
{
    if (nrows <= 0 || gstride <= 0)
        return hipSuccess;
    dim3 grid(grid_for(nrows, 4)), block(256);
    if (metric == M_L2)
        hipLaunchKernelGGL(k_prep_input<M_L2>, grid, block, 0, st, R, row0, nrows, id_offset,
                           n_local, ids, dist, kin, gstride, gin, ctr);
    else if (metric == M_COS)
        hipLaunchKernelGGL(k_prep_input<M_COS>, grid, block, 0, st, R, row0, nrows, id_offset,
                           n_local, ids, dist, kin, gstride, gin, ctr);
    else
        hipLaunchKernelGGL(k_prep_input<M_L1>, grid, block, 0, st, R, row0, nrows, id_offset,
                           n_local, ids, dist, kin, gstride, gin, ctr);
    return hipGetLastError();
}

hipError_t launch_init(const Rows &R, int metric, const InitArgs &a, hipStream_t st)
{
    unsigned g = grid_for(a.n, 4);
    dim3 grid(g > 8192u ? 8192u : g), block(256);
    if (metric == M_L2)
        hipLaunchKernelGGL(k_init<M_L2>, grid, block, 0, st, R, a);
    else if (metric == M_COS)
        hipLaunchKernelGGL(k_init<M_COS>, grid, block, 0, st, R, a);
    else
        hipLaunchKernelGGL(k_init<M_L1>, grid, block, 0, st, R, a);
    return hipGetLastError();
}

hipError_t launch_final(const FinalArgs &a, hipStream_t st)
{
    if (!a.touched && a.k <= 32 && a.kin <= 32) {
        hipLaunchKernelGGL(k_final<32>, dim3(grid_for(a.n, 8)), dim3(256), 0, st, a);
        return hipGetLastError();
    }
    unsigned g = grid_for(a.n, 4);
    if (a.touched && g > 8192u)
        g = 8192u;
    hipLaunchKernelGGL(k_final<WAVE>, dim3(g), dim3(256), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_restore(uint64_t *L, uint64_t *worst, const int32_t *dtag, const uint64_t *gin,
                          int kin, int k, int64_t m, int32_t since, hipStream_t st)
{
    if (m <= 0)
        return hipSuccess;
    unsigned g = grid_for(m, 4);
    hipLaunchKernelGGL(k_restore, dim3(g > 8192u ? 8192u : g), dim3(256), 0, st, L, worst, dtag,
                       gin, kin, k, m, since);
    return hipGetLastError();
}

hipError_t launch_commit(const CommitArgs &a, hipStream_t st)
{
    const int64_t rows = a.m_base + a.n_req;
    if (rows <= 0)
        return hipSuccess;
    unsigned g = grid_for(rows, 4);
    dim3 grid(g > 8192u ? 8192u : g), block(256);
    if (a.k <= 16)
        hipLaunchKernelGGL(k_commit<16>, grid, block, 0, st, a);
    else if (a.k <= 32)
        hipLaunchKernelGGL(k_commit<32>, grid, block, 0, st, a);
    else
        hipLaunchKernelGGL(k_commit<64>, grid, block, 0, st, a);
    return hipGetLastError();
}

hipError_t launch_sort_rows(const uint64_t *src, int src_stride, int64_t n, int k, uint64_t *dst,
                            int dst_stride, int32_t *ids, float *dist, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_sort_rows, dim3(grid_for(n, 4)), dim3(256), 0, st, src, src_stride, n, k,
                       dst, dst_stride, ids, dist);
    return hipGetLastError();
}

hipError_t launch_permute_rows(const float *x, int64_t n, int d, uint64_t seed, int half,
                               int32_t *perm, float *xp, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_perm, dim3(grid_for(n, 256)), dim3(256), 0, st, seed, n, half, perm);
    unsigned g = grid_for(n * d, 256);
    hipLaunchKernelGGL(k_gather_rows, dim3(g > 65536u ? 65536u : g), dim3(256), 0, st, x, n, d,
                       perm, xp);
    return hipGetLastError();
}

hipError_t launch_unpermute_graph(const int32_t *ids, const float *dist, int64_t n, int k,
                                  const int32_t *perm, int32_t *out_ids, float *out_dist,
                                  hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3(grid_for(n, 4)), dim3(256), 0, st, ids, dist, n, k, perm,
                       out_ids, out_dist);
    return hipGetLastError();
}

// rows x k list words set to empty slots (~0 - slot)
__global__ __launch_bounds__(256) void k_fill_empty(uint64_t *p, int64_t rows, int k)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * k;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = empty_key((int)(e % k));
}

hipError_t launch_fill_empty(uint64_t *p, int64_t rows, int k, hipStream_t st)
{
    int64_t g = (rows * k + 255) / 256;
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    hipLaunchKernelGGL(k_fill_empty, dim3((unsigned)g), dim3(256), 0, st, p, rows, k);
    return hipGetLastError();
}

hipError_t launch_zero_counters(uint64_t *ctr, int words, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, ctr, words);
    return hipGetLastError();
}

} // namespace knng
