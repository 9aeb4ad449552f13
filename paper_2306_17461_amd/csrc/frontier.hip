// The Landau-Vishkin frontier (section 3.1, Algorithm 1; appendix A).
//
// Round t computes, for every diagonal i in [max(-t,-m), min(t,n)],
//   c = max(f[i] + 1, f[i-1] + 1, f[i+1])       (substitution, deletion, insertion)
//   c = min(c, n, m + i)                         (the last cell of the diagonal)
//   f'[i] = c + LCP(c, c - i)
// which is Algorithm 1 with its three slides merged into one: sliding along a
// diagonal is monotone and a slide from a lower start that passes a higher
// start ends where that one ends, so the largest of three slides equals the
// slide of the largest start.  Rows hold every index in [-(t+2), t+2] (kNone
// outside the grid), so the next round reads neighbours without bound tests.
// The search stops at the first t with f_t[n-m] = n; that t is the distance.
//
// Kernels:
//   frontier_kernel  one pair, all rounds in one persistent launch: workgroup
//                    0 runs the first rounds alone with both rows in LDS
//                    (barriers are s_barrier only); when the rows outgrow LDS
//                    the frontier moves to global memory and every workgroup
//                    takes a slice of the diagonals, with a device-wide
//                    barrier between rounds.
//   batch_kernel     many pairs in one persistent launch: workgroups take
//                    pairs from a device queue (largest first) and run all
//                    rounds of a pair with workgroup barriers only.
//   lcp_query_kernel one LCP query per wavefront (tests of the engines).
#include "device.h"

namespace ed {

namespace {

__device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

// One round over entries [e_begin, e_end) of the 2t+5 row entries (entry e
// is diagonal e - (t+2)).  `prev` and `cur` point at diagonal 0 of their
// rows.  The loop trip count is uniform over the calling threads, so every
// wavefront reaches the wave-level LCP code with all 64 lanes.  Returns true
// in the thread that found f_t[target] = n.
template <typename PrevPtr, typename CurPtr>
__device__ __forceinline__ bool do_round(const Engine& en, int32_t t, PrevPtr prev, CurPtr cur,
                                         int32_t e_begin, int32_t e_end, int tid, int nthr,
                                         int32_t* dump_row, CountersDev& cnt) {
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t lo = imax(-t, -m), hi = imin(t, n);
    const int32_t target = n - m;
    bool found = false;
    for (int32_t base = e_begin; base < e_end; base += nthr) {
        const int32_t e = base + tid;
        const bool active = e < e_end;
        const int32_t i = e - (t + 2);
        const bool inr = active && i >= lo && i <= hi;
        int32_t c = -1;
        if (inr) {
            if (t == 0) {
                c = 0;
            } else {
                const int32_t a = prev[i], b = prev[i - 1], d = prev[i + 1];
                c = imax(imax(a + 1, b + 1), d);  // kNone + 1 stays negative
                if (c >= 0) c = imin(imin(c, n), m + i);
            }
        }
        const bool valid = inr && c >= 0;
        const int32_t l = slide(en, valid, c, c - i, cnt);
        const int32_t f = valid ? c + l : kNone;
        if (active) {
            cur[i] = f;
            if (dump_row && i >= -t && i <= t) dump_row[i + t] = f;
        }
        if (valid) {
            cnt.updates++;
            if (i == target && f == n) found = true;
        }
    }
    return found;
}

__device__ __forceinline__ void grid_barrier(FrontierCtl* ctl) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int g = __hip_atomic_load(&ctl->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int arrived =
            __hip_atomic_fetch_add(&ctl->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == gridDim.x - 1) {
            __hip_atomic_store(&ctl->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ctl->bar_gen, g + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            while (__hip_atomic_load(&ctl->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g)
                __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
}

__device__ __forceinline__ Engine make_engine(const PairDev& p, const HashDev& h, int engine,
                                              int lane_words, const uint64_t* lut4) {
    Engine en;
    const uint32_t alpha = *p.alpha;
    pair_views(p, alpha, en.A, en.B);
    en.TA = p.a.tab;
    en.TB = p.b.tab;
    en.q.h = h;
    en.q.r4 = engine == 1 ? mp_mul(mp_mul(h.r, h.r), mp_mul(h.r, h.r)) : 0;
    en.q.lut4 = lut4;
    en.q.log2b = p.log2b;
    en.kind = engine;
    en.lane_words = lane_words;
    return en;
}

struct LdsState {
    int32_t row[2][kLdsRowLen];
    uint64_t lut4[256];
    int32_t flag;
    int32_t pair;
};

// Rounds of one pair inside one workgroup, starting from round 0, first in
// LDS (up to lds_rounds rounds), then in the global rows g0/g1 (capacity K).
// Returns k, kmax + 1, or -3 when the rows are too small.
__device__ int32_t pair_in_workgroup(const Engine& en, LdsState& L, int32_t lds_rounds, int32_t kmax,
                                     int32_t* g0, int32_t* g1, int32_t K, CountersDev& cnt) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t maxnm = imax(n, m);
    const int32_t off = kLdsRoundsMax + 2;
    int32_t* la = L.row[0] + off;
    int32_t* lb = L.row[1] + off;
    if (tid == 0) L.flag = 0;
    __syncthreads();
    int32_t t = 0;
    if (do_round(en, 0, la, la, 0, 5, tid, nthr, nullptr, cnt)) L.flag = 1;
    __syncthreads();
    const int32_t lr = imin(lds_rounds, kLdsRoundsMax);
    // LDS phase
    for (;;) {
        if (L.flag) return t;
        if (kmax >= 0 && t >= kmax) return kmax + 1;
        if (t > maxnm) return -3;
        if (t >= lr) break;
        ++t;
        if (do_round(en, t, la, lb, 0, 2 * t + 5, tid, nthr, nullptr, cnt)) L.flag = 1;
        int32_t* tmp = la;
        la = lb;
        lb = tmp;
        __syncthreads();
    }
    // global phase: copy the last LDS row out
    if (t + 2 > K + 2 || g0 == nullptr) return -3;
    int32_t* ga = g0 + K + 2;
    int32_t* gb = g1 + K + 2;
    for (int32_t e = tid; e < 2 * t + 5; e += nthr) ga[e - (t + 2)] = la[e - (t + 2)];
    __syncthreads();
    for (;;) {
        if (L.flag) return t;
        if (kmax >= 0 && t >= kmax) return kmax + 1;
        if (t > maxnm || t >= K) return -3;
        ++t;
        if (do_round(en, t, ga, gb, 0, 2 * t + 5, tid, nthr, nullptr, cnt)) L.flag = 1;
        int32_t* tmp = ga;
        ga = gb;
        gb = tmp;
        __syncthreads();
    }
}

}  // namespace

__global__ void ctl_init_kernel(FrontierCtl* ctl, CountersDev* cnt) {
    if (threadIdx.x == 0) {
        ctl->bar_count = 0;
        ctl->bar_gen = 0;
        ctl->phase = 0;
        ctl->phase_t = 0;
        ctl->found_t = -1;
        ctl->status = 0;
        ctl->result_t = 0;
        ctl->wbuf = 0;
    }
    if (cnt && threadIdx.x < sizeof(CountersDev) / 8)
        reinterpret_cast<unsigned long long*>(cnt)[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kFrontierThreads) void frontier_kernel(FrontierParams P) {
    __shared__ LdsState L;
    const int tid = threadIdx.x, nthr = blockDim.x;
    CountersDev cnt = {};
    if (P.engine == 1) build_lut4(L.lut4, P.h.r, tid, nthr);
    __syncthreads();
    const Engine en = make_engine(P.p, P.h, P.engine, P.lane_words, L.lut4);
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t maxnm = imax(n, m);
    FrontierCtl* ctl = P.ctl;
    const int32_t K = P.K;
    int32_t t = P.t0;
    int32_t* gp = P.f0 + K + 2;  // holds f_t
    int32_t* gc = P.f1 + K + 2;
    bool finished = false;

    if (P.t0 == 0) {
        if (P.lds_rounds > 0) {
            // ---------------- phase A: workgroup 0, rows in LDS ----------------
            if (blockIdx.x == 0) {
                const int32_t off = kLdsRoundsMax + 2;
                int32_t* la = L.row[0] + off;
                int32_t* lb = L.row[1] + off;
                if (tid == 0) L.flag = 0;
                __syncthreads();
                if (do_round(en, 0, la, la, 0, 5, tid, nthr, P.dump, cnt)) L.flag = 1;
                __syncthreads();
                const int32_t lr = imin(imin(P.lds_rounds, kLdsRoundsMax), K);
                int32_t status = 0, result = 0;
                for (;;) {
                    if (L.flag) { status = 1; result = t; break; }
                    if (P.kmax >= 0 && t >= P.kmax) { status = 2; result = P.kmax + 1; break; }
                    if (t > maxnm) { status = 4; result = t; break; }
                    if (t >= lr) break;
                    ++t;
                    int32_t* drow = (P.dump && static_cast<int64_t>(t + 1) * (t + 1) <= P.dump_cap)
                                        ? P.dump + static_cast<int64_t>(t) * t : nullptr;
                    if (do_round(en, t, la, lb, 0, 2 * t + 5, tid, nthr, drow, cnt)) L.flag = 1;
                    int32_t* tmp = la;
                    la = lb;
                    lb = tmp;
                    __syncthreads();
                }
                if (status == 0) {
                    for (int32_t e = tid; e < 2 * t + 5; e += nthr) gp[e - (t + 2)] = la[e - (t + 2)];
                }
                __syncthreads();
                if (tid == 0) {
                    if (status != 0) {
                        ctl->result_t = result;
                        __hip_atomic_store(&ctl->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    } else {
                        ctl->phase_t = t;
                    }
                    __hip_atomic_store(&ctl->phase, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
                finished = status != 0;
            } else {
                if (tid == 0) {
                    while (__hip_atomic_load(&ctl->phase, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0)
                        __builtin_amdgcn_s_sleep(8);
                    L.flag = __hip_atomic_load(&ctl->status, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                }
                __syncthreads();
                finished = L.flag != 0;
                // workgroup 0 wrote phase_t before its release of `phase`
                if (!finished) t = __hip_atomic_load(&ctl->phase_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        } else {
            // round 0 grid-wide (only workgroup 0 holds the entries)
            int32_t* drow = P.dump && P.dump_cap >= 1 ? P.dump : nullptr;
            if (blockIdx.x == 0) {
                if (do_round(en, 0, gp, gp, 0, 5, tid, nthr, drow, cnt))
                    __hip_atomic_store(&ctl->found_t, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            grid_barrier(ctl);
        }
    }

    // ---------------- phase B: all workgroups, rows in global memory ----------------
    if (!finished) {
        const int G = gridDim.x;
        for (;;) {
            // found_t is written during a round and read after that round's
            // barrier; a value above t was written by a workgroup already in
            // round t+1 and is acted on after the next barrier
            const int32_t ft = __hip_atomic_load(&ctl->found_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int32_t status = 0, result = 0;
            if (ft >= 0 && ft <= t) { status = 1; result = ft; }
            else if (P.kmax >= 0 && t >= P.kmax) { status = 2; result = P.kmax + 1; }
            else if (t > maxnm) { status = 4; result = t; }
            else if (t >= K) { status = 3; result = t; }
            if (status != 0) {
                if (blockIdx.x == 0 && tid == 0) {
                    ctl->result_t = result;
                    ctl->wbuf = gp == P.f0 + K + 2 ? 0 : 1;
                    __hip_atomic_store(&ctl->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
                break;
            }
            ++t;
            const int32_t total = 2 * t + 5;
            const int32_t chunk = (total + G - 1) / G;
            const int32_t eb = imin(total, static_cast<int32_t>(blockIdx.x) * chunk);
            const int32_t ee = imin(total, eb + chunk);
            int32_t* drow = (P.dump && static_cast<int64_t>(t + 1) * (t + 1) <= P.dump_cap)
                                ? P.dump + static_cast<int64_t>(t) * t : nullptr;
            if (do_round(en, t, gp, gc, eb, ee, tid, nthr, drow, cnt))
                __hip_atomic_store(&ctl->found_t, t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            grid_barrier(ctl);
            int32_t* tmp = gp;
            gp = gc;
            gc = tmp;
        }
    }
    flush_counters(cnt, P.counters);
}

__global__ __launch_bounds__(kFrontierThreads) void batch_kernel(BatchParams P) {
    __shared__ LdsState L;
    const int tid = threadIdx.x;
    CountersDev cnt = {};
    if (P.engine == 1) build_lut4(L.lut4, P.h.r, tid, blockDim.x);
    for (;;) {
        __syncthreads();
        if (tid == 0) L.pair = static_cast<int32_t>(atomicAdd(P.ticket, 1u));
        __syncthreads();
        const int32_t idx = L.pair;
        if (idx >= P.count) break;
        const int32_t pi = P.order[idx];
        const BatchItem item = P.items[pi];
        const Engine en = make_engine(item.p, P.h, P.engine, P.lane_words, L.lut4);
        const int32_t k = pair_in_workgroup(en, L, P.lds_rounds, P.kmax, item.f0, item.f1, item.K, cnt);
        if (tid == 0) P.k_out[pi] = k;
    }
    flush_counters(cnt, P.counters);
}

__global__ __launch_bounds__(256) void lcp_query_kernel(LcpQueryParams Q) {
    __shared__ uint64_t lut4[256];
    CountersDev cnt = {};
    if (Q.engine == 1) build_lut4(lut4, Q.h.r, threadIdx.x, blockDim.x);
    __syncthreads();
    const Engine en = make_engine(Q.p, Q.h, Q.engine, Q.lane_words, lut4);
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    for (int64_t qi = wave; qi < Q.count; qi += nwaves) {
        const int32_t x = static_cast<int32_t>(Q.x[qi]);
        const int32_t y = static_cast<int32_t>(Q.y[qi]);
        const int32_t l = slide(en, lane_id() == 0, x, y, cnt);
        if (lane_id() == 0) Q.out[qi] = l;
    }
    flush_counters(cnt, Q.counters);
}

hipError_t launch_ctl_init(FrontierCtl* ctl, CountersDev* cnt, hipStream_t s) {
    hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(64), 0, s, ctl, cnt);
    return hipGetLastError();
}

hipError_t frontier_max_grid(int device, int* grid_out) {
    int cus = 0, per = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(frontier_kernel),
                                                     kFrontierThreads, 0);
    if (e != hipSuccess) return e;
    if (per < 1) per = 1;
    *grid_out = cus * per;
    return hipSuccess;
}

hipError_t launch_frontier(const FrontierParams& fp, int grid, hipStream_t s) {
    FrontierParams arg = fp;
    void* args[] = {&arg};
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(frontier_kernel), dim3(grid),
                                      dim3(kFrontierThreads), args, 0, s);
}

hipError_t launch_batch(const BatchParams& bp, int grid, hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(kFrontierThreads), 0, s, bp);
    return hipGetLastError();
}

hipError_t launch_lcp_queries(const LcpQueryParams& qp, hipStream_t s) {
    int64_t waves = qp.count < 1 ? 1 : qp.count;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(lcp_query_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, qp);
    return hipGetLastError();
}

}  // namespace ed
