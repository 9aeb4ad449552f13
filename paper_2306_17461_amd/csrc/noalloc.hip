// ed_distance_noalloc: the single-pair distance with its frontier rows in a
// file-scope device array instead of memory from the context's pool, for
// callers that cannot allocate device memory.
//
// The rows of the frontier (two int32 arrays of 2K + 5 entries, Algorithm 1's
// f_{t-1} and f_t) are the only device memory ed_distance allocates per call;
// here they live in `scratch`, one copy per device, whose device address is
// taken once per context at ed_init (with the device current) and used for
// every launch.  Every call on a device shares that device's array: calls that
// overlap on one device (two threads, or two contexts, with work in flight on
// different streams) race on it, and the contents of the last call remain.
#include <climits>

#include "../../include/ed.h"
#include "host.h"
#include "internal.h"

using namespace ed;

namespace {

constexpr int64_t kScratchRowLen = 2 * static_cast<int64_t>(ED_NOALLOC_MAX_K) + 5;
constexpr int64_t kScratchInts = 2 * kScratchRowLen;

}  // namespace

// Two frontier rows for rounds up to ED_NOALLOC_MAX_K (8,000,040 bytes).
static __device__ __align__(256) int32_t scratch[kScratchInts];

int ed::scratch_setup(ed_ctx* c) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
        set_error("ed_init: hipGetSymbolAddress(scratch) failed on device %d: %s", c->device,
                  hipGetErrorString(e));
        return ED_EDEVICE;
    }
    c->d_scratch = static_cast<int32_t*>(ptr);
    return ED_OK;
}

int ed_distance_noalloc(ed_ctx* c, ed_pair* p, int64_t k_max, uint64_t* k_out, void* hip_stream) {
    if (!c || !p || !k_out || p->ctx != c) return ED_EINVAL;
    if (k_max < 0 || k_max > static_cast<int64_t>(ED_NOALLOC_MAX_K)) {
        set_error("ed_distance_noalloc: k_max = %lld, must be in [0, %llu] (the rows of the scratch array)",
                  static_cast<long long>(k_max), static_cast<unsigned long long>(ED_NOALLOC_MAX_K));
        return ED_EINVAL;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->d_scratch) {
        set_error("ed_distance_noalloc: no scratch address on this context");
        return ED_EINTERNAL;
    }
    if (p->engine == ED_ENGINE_HASH && p->r != c->r) {
        // switching the context's power tables builds them on the host
        set_error("ed_distance_noalloc: the pair's hash base is not the context's current one");
        return ED_EINVAL;
    }
    if (hipSetDevice(c->device) != hipSuccess) {
        set_error("ed_distance_noalloc: hipSetDevice(%d) failed", c->device);
        return ED_EDEVICE;
    }
    return distance_locked(c, p, k_max, k_out, nullptr, 0, static_cast<hipStream_t>(hip_stream), c->d_scratch,
                           static_cast<int64_t>(ED_NOALLOC_MAX_K));
}
