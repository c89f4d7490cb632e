// knng_common.h -- device helpers shared by the HIP kernels of libknngmerge.
//
// Packed list entries, the counter-based random stream, canonical FP32
// distances and the lock-free bounded-set insert.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace knng {

enum { M_L2 = 0, M_COS = 1, M_L1 = 2 };

constexpr int WAVE = 64;
constexpr int MAX_K = 64;      // list capacity
constexpr int MAX_S = 32;      // sample size
constexpr int MAX_G = 160;     // neighbourhood size bound: 2s + k + s

// error bits collected in the device error word
enum : uint32_t {
    ERR_NONFINITE = 1u << 0,
    ERR_ZERO_NORM = 1u << 1,
    ERR_ID_RANGE = 1u << 2,
    ERR_SELF = 1u << 3,
    ERR_DUP = 1u << 4,
    ERR_UNSORTED = 1u << 5,
    ERR_BAD_DIST = 1u << 6,
    ERR_SPIN = 1u << 7,  // an insert exceeded its retry budget
    ERR_GROUP = 1u << 8, // neighbourhood larger than the kernel bound
    // internal consistency: a row id read from a list, sample or queue fell
    // outside [0, n); the access is skipped and the call fails
    ERR_ROW_REVERSE = 1u << 10,
    ERR_ROW_GROUP = 1u << 11,
    ERR_ROW_SAMPLE = 1u << 12,
    ERR_ROW_COMMIT = 1u << 13,
};

__device__ __forceinline__ void raise_err(uint64_t *err_word, uint32_t bit)
{
    atomicOr((unsigned long long *)err_word, (unsigned long long)bit);
}

// counters block (uint64 words)
enum : int {
    // per-round words (cleared before each round's reverse/join)
    C_FRESH = 0,    // entries inserted during the last round and still present
    C_PAIRS = 1,    // joined pairs this round
    C_GATHER = 2,   // neighbourhood members staged this round
    C_ACTIVE = 3,   // rows appended to the round's active list (list mode)
    C_ROUND_WORDS = 4,
    // whole-call words
    C_EVALS = 4,    // distance evaluations (scanning-rate numerator)
    C_RESCORE = 5,  // pairs rescored in FP32 (BF16 path)
    C_MAXG = 6,     // largest neighbourhood (max)
    C_ERR = 7,      // error bits
    C_ATTEMPT = 8,  // list inserts attempted after the screen
    C_VIOL = 9,     // BF16 path: rescored pairs outside the screening margin
    C_N0 = 10,       // rows holding a NEW entry when the loop starts
    C_WORDS = 11,
};

// ---------------------------------------------------------------- keys
// A list entry is one 64-bit word ordered as an unsigned integer:
//   bits 63..32  IEEE bits of the distance (always >= +0, so the unsigned
//                order of the bits is the numeric order)
//   bits 31..2   id (< 2^30)
//   bit 1        FRESH: inserted during the current round
//   bit 0        NEW:   not yet taken as a NEW sample
// Unsigned order of the word = (distance, id) order; the flags never decide
// between different entries.  Empty slots hold ~0 - slot: above every real
// entry and distinct from each other.
constexpr uint32_t F_NEW = 1u;
constexpr uint32_t F_FRESH = 2u;

__device__ __forceinline__ uint64_t make_key(float d, uint32_t id, uint32_t flags)
{
    return ((uint64_t)__float_as_uint(d) << 32) | ((uint64_t)id << 2) | flags;
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return ((uint32_t)k) >> 2; }
__device__ __forceinline__ float key_dist(uint64_t k) { return __uint_as_float((uint32_t)(k >> 32)); }
__device__ __forceinline__ uint64_t key_strip(uint64_t k) { return k & ~3ull; }
__device__ __forceinline__ uint64_t empty_key(int slot) { return ~0ull - (uint64_t)slot; }
__device__ __forceinline__ bool key_empty(uint64_t k) { return (uint32_t)(k >> 32) == 0xFFFFFFFFu; }

// ---------------------------------------------------------------- random stream
// SplitMix64 (Steele, Lea, Flood 2014): state x -> mix(x + golden gamma).
__device__ __forceinline__ uint64_t sm64(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// hash of a tuple: the generator chained over (seed ^ tag, a, b, c)
__device__ __forceinline__ uint64_t hash5(uint64_t seed, uint64_t tag, uint64_t a, uint64_t b,
                                          uint64_t c)
{
    uint64_t h = sm64(seed ^ tag);
    h = sm64(h ^ a);
    h = sm64(h ^ b);
    return sm64(h ^ c);
}

constexpr uint32_t TAG_APPEND = 0xA1u, TAG_INIT = 0xA2u, TAG_SELECT = 0xA3u, TAG_FWD = 0xB1u,
                   TAG_RNEW = 0xB2u, TAG_ROLD = 0xB3u, TAG_PERM = 0xC1u;

// uniform draw below N from the high 32 bits (multiply-shift)
__device__ __forceinline__ uint32_t draw_below(uint64_t h, uint32_t N)
{
    return (uint32_t)(((h >> 32) * (uint64_t)N) >> 32);
}

// Balanced append (J-Merge of a raw set smaller than the base): base row i
// takes part in Divide and Append when draw_below(H(seed, SELECT, i), nb) <
// nr, i.e. with probability nr/nb; all rows when nr >= nb or when off.
__device__ __forceinline__ bool selected_base_row(uint64_t seed, int balanced, int64_t i,
                                                  int64_t nb, int64_t nr)
{
    if (!balanced || nr >= nb)
        return true;
    return (int64_t)draw_below(hash5(seed, TAG_SELECT, (uint64_t)i, 0, 0), (uint32_t)nb) < nr;
}

// ---------------------------------------------------------------- canonical FP32
// Rows are padded with zeros to a multiple of 4 floats; a zero pair adds
// exactly nothing to any accumulator below, so padded lengths give the same
// bits as the true length.
template <int METRIC>
__device__ __forceinline__ float canon_step(float acc, float a, float b)
{
    if constexpr (METRIC == M_L1) {
        return acc + fabsf(a - b);
    } else {
        float diff = a - b;
        return __builtin_fmaf(diff, diff, acc);
    }
}

// cosine distance from the l2 accumulator and the two canonical norms
__device__ __forceinline__ float cos_finish(float D, float na, float nb)
{
    float e = na - nb;
    float num = __builtin_fmaf(-e, e, D);
    float den = (2.0f * na) * nb;
    float r = num / den;  // correctly rounded (see build flags)
    return r > 0.0f ? r : 0.0f;
}

template <int METRIC>
__device__ __forceinline__ float canon_finish(float acc, float na, float nb)
{
    if constexpr (METRIC == M_COS)
        return cos_finish(acc, na, nb);
    else
        return acc;
}

// full canonical distance of two padded rows read from global memory
template <int METRIC>
__device__ __forceinline__ float canon_dist(const float *__restrict__ a, const float *__restrict__ b,
                                            int dp, float na, float nb)
{
    float acc = 0.0f;
    const float4 *a4 = reinterpret_cast<const float4 *>(a);
    const float4 *b4 = reinterpret_cast<const float4 *>(b);
#pragma unroll 4
    for (int t = 0; t < dp / 4; t++) {
        float4 x = a4[t], y = b4[t];
        acc = canon_step<METRIC>(acc, x.x, y.x);
        acc = canon_step<METRIC>(acc, x.y, y.y);
        acc = canon_step<METRIC>(acc, x.z, y.z);
        acc = canon_step<METRIC>(acc, x.w, y.w);
    }
    return canon_finish<METRIC>(acc, na, nb);
}

// round-to-nearest-even fp32 -> bf16 (bits in the high half), finite inputs
__device__ __forceinline__ uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- atomics
__device__ __forceinline__ uint64_t ld_agent(const uint64_t *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool cas64(uint64_t *p, uint64_t expect, uint64_t desired)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// As cas64; on failure `expect` receives the word the slot held instead.
__device__ __forceinline__ bool cas64_seen(uint64_t *p, uint64_t &expect, uint64_t desired)
{
    return __hip_atomic_compare_exchange_strong(p, &expect, desired, __ATOMIC_RELAXED,
                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr int SPIN_BUDGET = 1 << 16;

__device__ __forceinline__ void atomic_min_u64(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A slot is a duplicate of a key when the two agree under the mask: the
// (distance, id) of a list word, or the whole word of a reverse-reservoir key
// (whose low bits are the source id).
constexpr uint64_t DUP_NONE = 0, DUP_ID = ~3ull, DUP_EXACT = ~0ull;

// Insert `key` into the unordered bounded set slots[0..cap) (cap <= KB): when
// the key is below the current maximum and no slot is a duplicate of it under
// `dup_mask` (DUP_NONE: no test), the maximum slot is replaced by a CAS.
//
// Correctness: slot values only ever decrease and are pairwise distinct, so if
// the CAS on the slot that held the maximum M of the values read succeeds,
// that slot held M throughout and every other slot is <= what was read <= M:
// M was still the maximum (this holds even when some reads were older than
// others).  A duplicate present at CAS time would have replaced a value > M in
// some slot before that slot was read, so the read would have seen it.  Hence
// every interleaving of inserts leaves the `cap` smallest distinct keys offered.
//
// Slots are loaded in batches (all 20 of a k = 20 list at once) before any
// decision on them, one memory round trip per batch.  The first pass reads
// through the caches: a stale value is an older, hence larger, value of its
// slot, which the argument above allows (a stale duplicate was evicted for
// good, since the list's maximum has been below it ever since), and it can
// only make the CAS fail; later passes read at device scope.  On success,
// `live_worst` (when given) is lowered to an upper bound of the new maximum:
// max(key, largest value read besides M).
template <int KB>
__device__ inline bool bounded_insert(uint64_t *slots, int cap, uint64_t key, uint64_t dup_mask,
                                      uint64_t *live_worst, uint64_t *err_word)
{
    constexpr int B = KB <= 16 ? KB : (KB == 32 ? 20 : 16);
    const uint64_t kid = key & dup_mask;
    for (int spin = 0; spin < SPIN_BUDGET; spin++) {
        uint64_t mx = 0, second = 0;
        int mj = 0;
        bool dup = false;
        for (int j0 = 0; j0 < cap; j0 += B) {
            uint64_t v[B];
#pragma unroll
            for (int j = 0; j < B; j++)
                v[j] = j0 + j < cap ? (spin == 0 ? slots[j0 + j] : ld_agent(slots + j0 + j))
                                    : 0ull;
#pragma unroll
            for (int j = 0; j < B; j++) {
                if (j0 + j < cap) {
                    dup |= dup_mask != DUP_NONE && (v[j] & dup_mask) == kid;
                    if (v[j] > mx) {
                        second = mx;
                        mx = v[j];
                        mj = j0 + j;
                    } else if (v[j] > second) {
                        second = v[j];
                    }
                }
            }
        }
        if (dup || key >= mx)
            return false;
        if (cas64(slots + mj, mx, key)) {
            if (live_worst)
                atomic_min_u64(live_worst, key > second ? key_strip(key) : key_strip(second));
            return true;
        }
    }
    atomicOr((unsigned long long *)err_word, (unsigned long long)ERR_SPIN);
    return false;
}

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }

// wave-wide sums / max through shuffles
__device__ __forceinline__ int wave_sum(int v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1)
        v += __shfl_xor(v, o, WAVE);
    return v;
}
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        uint64_t w = __shfl_xor(v, o, WAVE);
        v = w > v ? w : v;
    }
    return v;
}

// ---------------------------------------------------------------- row walks
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

// The same walk over the rows r < n for which pred(r) holds.
template <class P>
__device__ inline uint64_t ballot_rows(int64_t b, int64_t stride, int64_t n, P pred)
{
    const int64_t r = b + (int64_t)lane_id() * stride;
    return __ballot(r < n && pred(r));
}

#define FOR_ROWS_IF(u, n, pred)                                                               \
    const int64_t nwaves_ = (int64_t)gridDim.x * (blockDim.x / WAVE);                        \
    const int64_t wave0_ = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / WAVE;          \
    for (int64_t b_ = wave0_; b_ < (n); b_ += nwaves_ * WAVE)                                 \
        for (uint64_t todo_ = ballot_rows(b_, nwaves_, (n), pred); todo_; todo_ &= todo_ - 1) \
            if (const int64_t u = b_ + (int64_t)__builtin_ctzll(todo_) * nwaves_; true)

// Rows active in round tag tr: from the round's active list when there is one
// (a.alist, a.n_active entries), else by a walk over a.atag.
#define FOR_ACTIVE_ROWS(u, a, tr)                                                              \
    const bool listed_ = (a).alist != nullptr;                                                 \
    const int64_t span_ = listed_ ? (a).n_active : (a).n;                                      \
    FOR_ROWS_IF(j_, span_, [&](int64_t r) { return listed_ || (a).atag[r] == (tr); })          \
    if (const int64_t u = listed_ ? (int64_t)(a).alist[j_] : j_; true)

} // namespace knng
