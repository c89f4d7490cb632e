// knng_noalloc.hip -- knng_merge for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc): the merge's scratch lives in a file-scope device array
// of fixed size instead of a caller workspace.
//
// Each GPU the library runs on holds its own copy of `scratch` (allocated
// when the code object is loaded there) until the process ends.  In host code
// the array's name is only a host-side stand-in, so its device address is
// taken once per device with hipGetSymbolAddress and kept; only that address
// is ever passed to kernels or copies.  Every call on a device shares that
// device's array: calls that overlap on one GPU race.  The merge writes every
// scratch word it reads before reading it (counters are cleared by a kernel,
// lists, tags and samples are initialised by Divide/Append), so nothing left
// by an earlier call changes a result.
#include <mutex>

#include "knng_host.h"

using namespace knng;
using namespace knng::host;

namespace knng {
namespace host {
knng_status merge_on_scratch(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                             const knng_graph *G2, int32_t k, knng_metric metric,
                             const knng_opts *opts, knng_graph *out, void *scratch,
                             size_t scratch_bytes, void *stream, knng_stats *stats);
} // namespace host
} // namespace knng

static constexpr size_t SCRATCH_BYTES = (size_t)KNNG_NOALLOC_SCRATCH_BYTES;

static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

std::mutex g_mu;
void *g_ptr[MAX_DEVICES];  // device address of `scratch`, per device

// the current device's address of `scratch`, taken on first use
knng_status scratch_address(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(KNNG_EDEVICE, "device %d beyond the %d the library tracks", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(KNNG_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return KNNG_OK;
}

} // namespace

extern "C" {

knng_status knng_merge_noalloc(const knng_set *S1, const knng_graph *G1, const knng_set *S2,
                               const knng_graph *G2, int32_t k, knng_metric metric,
                               const knng_opts *opts, knng_graph *out, void *stream,
                               knng_stats *stats)
{
    try {
        if (!S1 || !S2 || !G1 || !G2 || !opts)
            return fail(KNNG_EINVAL, "S1, S2, G1, G2 and opts must not be NULL");
        if (opts->flags & KNNG_FLAG_PROFILE)
            return fail(KNNG_EINVAL,
                        "KNNG_FLAG_PROFILE creates HIP events; the no-allocation merge refuses it");
        const size_t need = knng_merge_workspace_size(S1->n, S2->n, S1->d, k, G1->k, G2->k,
                                                      metric, opts);
        if (need == 0)
            return fail(KNNG_EINVAL, "invalid sizes or options");
        if (need > SCRATCH_BYTES)
            return fail(KNNG_ENOMEM,
                        "this merge needs %zu bytes of scratch; the no-allocation entry point "
                        "holds %zu (use knng_merge with a workspace)",
                        need, SCRATCH_BYTES);
        void *p = nullptr;
        const knng_status s = scratch_address(&p);
        if (s != KNNG_OK)
            return s;
        return merge_on_scratch(S1, G1, S2, G2, k, metric, opts, out, p, SCRATCH_BYTES, stream,
                                stats);
    } catch (const std::bad_alloc &) {
        return fail(KNNG_ENOMEM, "host memory exhausted");
    } catch (...) {
        return fail(KNNG_EDEVICE, "unexpected host exception");
    }
}

size_t knng_merge_noalloc_scratch_bytes(void) { return SCRATCH_BYTES; }

} // extern "C"
