// Dependent-access latency probe (measurement only, not on the distance
// path): the time of one global memory access whose address is the value
// the previous access returned.  A frontier round (Algorithm 1) takes at
// least one such access, its LCP loads, whose addresses come from the
// previous round's row; the probe gives that floor on this device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/ed.h"
#include "host.h"

namespace {

constexpr int kLineWords = 32;  // one link per 128-byte line

// link j holds (a j + 1) mod L at the start of line j: with L a power of two,
// a = 1 (mod 4) and an odd increment the map is one cycle through all L
// links (Hull-Dobell), and consecutive links lie far apart in memory
__global__ void chain_kernel(uint32_t* buf, uint32_t lines, uint32_t a) {
    for (uint64_t j = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; j < lines;
         j += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        buf[j * kLineWords] = static_cast<uint32_t>((static_cast<uint64_t>(a) * j + 1) & (lines - 1));
}

// one wavefront; lane l follows the cycle from link l L / 64 for `steps`
// links and leaves where it ended in sink[l]
__global__ void chase_kernel(const uint32_t* buf, uint32_t lines, uint32_t steps, uint32_t* sink) {
    uint32_t j = threadIdx.x * (lines / 64);
    for (uint32_t s = 0; s < steps; ++s) j = buf[static_cast<uint64_t>(j) * kLineWords];
    sink[threadIdx.x] = j;
}

}  // namespace

extern "C" int ed_debug_mem_latency(ed_ctx* c, uint64_t region_bytes, uint32_t steps, int warm,
                                    double* ns_per_access) {
    if (!c || !ns_per_access || steps == 0 || steps > (1u << 24) || region_bytes < 64 * 128 ||
        (region_bytes & (region_bytes - 1)) != 0 || region_bytes / 128 > (1ull << 31)) {
        ed::set_error("ed_debug_mem_latency: region must be a power of two of at least 8 KiB and at most "
                      "256 GiB, steps in [1, 2^24]");
        return ED_EINVAL;
    }
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) {
        ed::set_error("ed_debug_mem_latency: hipSetDevice failed");
        return ED_EDEVICE;
    }
    const uint32_t lines = static_cast<uint32_t>(region_bytes / 128);
    uint32_t* buf = nullptr;
    uint32_t* sink = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    int rc = ED_OK;
    float ms = 0;
    auto fail = [&](const char* what, hipError_t e) {
        ed::set_error("ed_debug_mem_latency: %s: %s", what, hipGetErrorString(e));
        rc = ED_EDEVICE;
    };
    hipError_t e = hipMalloc(&buf, region_bytes);
    if (e != hipSuccess) {
        ed::set_error("ed_debug_mem_latency: %llu bytes of device memory: %s",
                      static_cast<unsigned long long>(region_bytes), hipGetErrorString(e));
        return ED_ENOMEM;
    }
    if ((e = hipMalloc(&sink, 64 * sizeof(uint32_t))) != hipSuccess) fail("hipMalloc", e);
    if (rc == ED_OK && ((e = hipEventCreate(&ev[0])) != hipSuccess || (e = hipEventCreate(&ev[1])) != hipSuccess))
        fail("hipEventCreate", e);
    if (rc == ED_OK) {
        const uint32_t blocks = std::min<uint32_t>(4096, (lines + 255) / 256);
        hipLaunchKernelGGL(chain_kernel, dim3(blocks), dim3(256), 0, nullptr, buf, lines, 0x9E3779B1u);
        if (warm) hipLaunchKernelGGL(chase_kernel, dim3(1), dim3(64), 0, nullptr, buf, lines, steps, sink);
        hipEventRecord(ev[0], nullptr);
        hipLaunchKernelGGL(chase_kernel, dim3(1), dim3(64), 0, nullptr, buf, lines, steps, sink);
        hipEventRecord(ev[1], nullptr);
        if ((e = hipEventSynchronize(ev[1])) != hipSuccess || (e = hipGetLastError()) != hipSuccess)
            fail("chase", e);
        else if ((e = hipEventElapsedTime(&ms, ev[0], ev[1])) != hipSuccess)
            fail("hipEventElapsedTime", e);
    }
    for (hipEvent_t x : ev)
        if (x) hipEventDestroy(x);
    hipFree(sink);
    hipFree(buf);
    if (rc == ED_OK) *ns_per_access = static_cast<double>(ms) * 1e6 / steps;
    return rc;
}
