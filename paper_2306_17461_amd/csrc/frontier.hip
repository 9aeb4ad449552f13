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
//   frontier_kernel  one pair, all rounds in one persistent launch.
//                    Phase A: workgroup 0 runs the first rounds alone with
//                    both rows in LDS (workgroup barriers only).
//                    Phase B: every workgroup owns a slice of the diagonals;
//                    it loads its slice plus a halo of H diagonals per side,
//                    advances H rounds in LDS (the halo shrinks by one
//                    diagonal per round, so every value it computes is
//                    exact), writes its slice back, and meets the others at a
//                    device-wide barrier: one barrier per H rounds.
//   task_kernel      many pairs in one persistent launch, work stealing over
//                    (pair, diagonal-chunk) tasks (batch and serving).
//   lcp_query_kernel one LCP query per wavefront (tests of the engines).
//
// Inside a round every thread takes up to kU diagonals and issues the first
// word loads of all of them before comparing (one memory latency per pass).
// LCPs that run past the lane and wavefront tiers go to a job list in LDS
// and the whole workgroup extends each job (4 words per thread per step);
// the hash engine follows its direct steps with a wavefront's hash search.
#include <climits>

#include "device.h"

namespace ed {

namespace {

constexpr int kU = 2;          // diagonals per thread per pass
constexpr int kJobHalf = kGridJobs;  // queued LCPs per round (a ring of two halves)
constexpr int kWaveSteps = 2;  // wavefront steps before the hash search / workgroup tier
constexpr int kWgWords = 8;      // words per thread per workgroup-tier step (single pair)
constexpr int kWgWordsTask = 4;  // ... in the many-pair kernel (register budget)

struct RoundShared {
    int32_t ji[2 * kJobHalf];
    int32_t jx[2 * kJobHalf];
    int32_t jy[2 * kJobHalf];
    int32_t jlim[2 * kJobHalf];
    int32_t jl[2 * kJobHalf];
    int32_t jcount[2];  // monotonic job counters, one per round parity
    int32_t wmin;       // workgroup-tier reduction slot
    int32_t gmin;       // grid rounds: this workgroup's first mismatch of a job
    int32_t jorder[kJobHalf];  // grid rounds: queued jobs in increasing diagonal order
    int32_t hres;       // hash engine: result of wavefront 0's search for the workgroup
    int32_t hskip;      // hash engine: the last searched LCP outran the direct steps
    int32_t flag;
    int32_t pair;
    long long task;
    int32_t sched;                // task kernel: this workgroup schedules a super-step
    int32_t nsched;               // ... of this many chunk tasks
    unsigned long long qbase;     // ... from this position of the ring
};

struct LdsState {
    int32_t row[2][kLdsRowLen];
    uint64_t lut32[8][256];
    RoundShared rs;
    CountersDev cnt;
};

// Per-workgroup cursor into the job counters (uniform, kept in registers).
struct JobCursor {
    int32_t start[2];
};

__device__ __forceinline__ int32_t imax(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ __forceinline__ int32_t imin(int32_t a, int32_t b) { return a < b ? a : b; }

__device__ __forceinline__ void rs_init(RoundShared& RS, JobCursor& jc) {
    if (threadIdx.x == 0) {
        RS.jcount[0] = 0;
        RS.jcount[1] = 0;
        RS.flag = 0;
        RS.hskip = 0;
    }
    jc.start[0] = 0;
    jc.start[1] = 0;
}

// Engine (a), workgroup tier: every thread of the workgroup compares 4 words in
// the first step and W in each later one (W = 8: 262144 characters per step at
// 2 bits, 65536 at 8 bits); the first mismatch is the minimum over
// wavefronts.  Uniform arguments; returns the LCP.
// One workgroup step of W words per thread from offset l: the first mismatch
// below lim (INT_MAX if none).  Every thread calls it.
template <int W>
__device__ __forceinline__ int32_t wg_step(const SView& A, const SView& B, int32_t x, int32_t y, int32_t lim,
                                           int32_t l, int32_t& wmin) {
    const int tid = threadIdx.x;
    constexpr int nthr = kFrontierThreads;  // every launch of these kernels
    if (tid == 0) wmin = INT_MAX;
    __syncthreads();
    // every word first (all loads in flight together), then this lane's
    // first mismatch (the smallest word wins), the wavefront's and the
    // workgroup's
    uint64_t d[W];
#pragma unroll
    for (int w = 0; w < W; ++w) {
        const int32_t p = l + ((w * nthr + tid) << A.lcpw);
        const int32_t q = p < lim ? p : 0;
        d[w] = fetch(A, x + q) ^ fetch(B, y + q);
    }
    int32_t first = INT_MAX;
#pragma unroll
    for (int w = W - 1; w >= 0; --w) {
        const int32_t p = l + ((w * nthr + tid) << A.lcpw);
        if (p < lim && d[w]) first = p + (ctz64(d[w]) >> A.lbpc);
    }
    first = wave_min(first);
    if (lane_id() == 0 && first != INT_MAX) atomicMin(&wmin, first);
    __syncthreads();
    const int32_t m = wmin;
    __syncthreads();
    return m;
}

// The first step takes 4 words per thread (most LCPs that reach this tier end
// there), later steps W words per thread.
template <int W>
__device__ __forceinline__ int32_t lcp_wg_direct(const SView& A, const SView& B, int32_t x, int32_t y,
                                                 int32_t lim, int32_t l, int32_t& wmin) {
    constexpr int32_t nthr = kFrontierThreads;
    if (l < lim) {
        const int32_t m = wg_step<4>(A, B, x, y, lim, l, wmin);
        if (m != INT_MAX) return m < lim ? m : lim;
        l += (4 * nthr) << A.lcpw;
    }
    while (l < lim) {
        const int32_t m = wg_step<W>(A, B, x, y, lim, l, wmin);
        if (m != INT_MAX) return m < lim ? m : lim;
        l += (W * nthr) << A.lcpw;
    }
    return lim;
}

// Hash engine, workgroup tier: direct steps of the workgroup first (4 words
// per thread, then W), then, for an LCP that runs past them, the
// wavefront-parallel hash search by wavefront 0.  A direct step costs about 5
// us here; the search, several rounds of dependent probes, about 9 us on 2-bit
// strings (the masked block hash) and 30 us on 8-bit ones.  Hence one step at
// 2 bits (131072 characters) and kWgHashSteps8 at 8 bits (32768 + 3 x 65536),
// and none while the workgroup's last searched LCP ran on past their reach
// (the LCPs of a pair tend to be alike: about n/k characters on the path).
constexpr int kWgHashSteps8 = 4;
template <int W>
__device__ __forceinline__ int32_t lcp_wg_hash(const Engine& en, int32_t x, int32_t y, int32_t lim, int32_t l,
                                               RoundShared& RS, Cnt& cnt) {
    constexpr int32_t nthr = kFrontierThreads;
    // (the many-pair kernel, at its register limit, takes the first step only)
    const int steps = (W == kWgWords && en.A.bpc == 8) ? kWgHashSteps8 : 1;
    const int32_t reach = (4 * nthr + (steps - 1) * W * nthr) << en.A.lcpw;
    const int32_t l0 = l;
    if (!RS.hskip) {
        if (l < lim) {
            const int32_t m = wg_step<4>(en.A, en.B, x, y, lim, l, RS.wmin);
            if (m != INT_MAX) return m < lim ? m : lim;
            l += (4 * nthr) << en.A.lcpw;
        }
        for (int st = 1; st < steps && l < lim; ++st) {
            const int32_t m = wg_step<W>(en.A, en.B, x, y, lim, l, RS.wmin);
            if (m != INT_MAX) return m < lim ? m : lim;
            l += (W * nthr) << en.A.lcpw;
        }
        if (l >= lim) return lim;
    }
    if ((threadIdx.x >> 6) == 0) {
        const int32_t r = lcp_wave_hash(en.A, en.B, en.TA, en.TB, en.q, x, y, lim, l, cnt);
        if (threadIdx.x == 0) RS.hres = r;
    }
    __syncthreads();
    const int32_t r = RS.hres;
    // every thread read hskip before the barrier above
    if (threadIdx.x == 0) RS.hskip = r - l0 > reach ? 1 : 0;
    __syncthreads();  // hres and hskip are written again by the next job
    return r;
}

// Tiers (2)/(3) for one slot of diagonals of a wavefront: every lane with a
// pending LCP is extended in turn by the whole wavefront.  Arguments are the
// calling lane's own values; `l` and `queued` are updated in that lane.
__device__ __forceinline__ void wave_extend(const Engine& en, bool pend, int32_t c, int32_t i,
                                            int32_t lim, int32_t& l, bool& queued, RoundShared& RS,
                                            int par, int half, int32_t jstart, int lane,
                                            Cnt& cnt) {
    uint64_t pm = ballot(pend);
    while (pm) {
        const int src = ctz64(pm);
        pm &= pm - 1;
        const int32_t jx = shfl_i32(c, src), jy = shfl_i32(c - i, src);
        const int32_t jlim = shfl_i32(lim, src), jl = shfl_i32(l, src);
        bool done = false;
        int32_t r;
        if (en.kind == 1 && en.hash_first) {
            // long-LCP form: the wavefront's hash search, no direct steps
            r = lcp_wave_hash(en.A, en.B, en.TA, en.TB, en.q, jx, jy, jlim, jl, cnt);
            done = true;
        } else {
            r = lcp_wave_steps(en.A, en.B, jx, jy, jlim, jl, kWaveSteps, done);
        }
        if (lane == 0) atomicAdd(&cnt.sh->wave_lcps, 1ull);
        if (!done) {
            // the workgroup tier takes it after the round's barrier
            int32_t s = 0;
            if (lane == 0) s = atomicAdd(&RS.jcount[par], 1) - jstart;
            s = shfl_i32(s, 0);
            if (s < kJobHalf) {
                if (lane == src) {
                    RS.ji[half + s] = i;
                    RS.jx[half + s] = jx;
                    RS.jy[half + s] = jy;
                    RS.jlim[half + s] = jlim;
                    RS.jl[half + s] = r;
                    queued = true;
                }
                continue;
            }
            // queue full: the wavefront finishes it
            r = lcp_wave_direct(en.A, en.B, jx, jy, jlim, r);
        }
        if (lane == src) l = r;
    }
}

// Grid tier of engine (a): one long LCP shared by every wavefront of a launch.  Wavefront
// w of `nw` takes the segments w, w + nw, w + 2 nw, ... of 64 x kGridWords
// words (every load instruction covers 64 consecutive words), in increasing
// order, and lowers *result with the first mismatch it finds; it stops at its
// first segment that starts at or beyond min(lim, *result), so once every
// wavefront has stopped, every segment below the answer has been compared.
// Positions are offsets from l0 (the first l0 characters are known to
// match).  Segments are assigned statically: a shared ticket would serialise
// thousands of atomics on one address.  Uniform arguments; no barrier inside.
template <int kGridWords>
__device__ __forceinline__ void grid_segments(const SView& A, const SView& B, int32_t x, int32_t y, int32_t lim,
                                           int32_t l0, int32_t w0, int32_t nw, int32_t* result) {
    const int lane = lane_id();
    const int32_t cpw = 1 << A.lcpw;
    const int64_t span = static_cast<int64_t>(64) * kGridWords * cpw;
    for (int64_t seg = w0;; seg += nw) {
        const int64_t start = l0 + seg * span;
        if (start >= lim) break;
        int32_t best = 0;
        if (lane == 0) best = __hip_atomic_load(result, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        best = shfl_i32(best, 0);
        if (start >= best) break;
        // this lane's first mismatch in the segment (the smallest word wins),
        // then the wavefront's
        int32_t first = INT_MAX;
#pragma unroll
        for (int w = kGridWords - 1; w >= 0; --w) {
            const int32_t rel = (w * 64 + lane) << A.lcpw;
            const int64_t pp = start + rel;
            const bool ok = pp < lim;
            const int32_t q = ok ? static_cast<int32_t>(pp) : 0;
            const uint64_t v = fetch(A, x + q) ^ fetch(B, y + q);
            if (ok && v) first = rel + (ctz64(v) >> A.lbpc);
        }
        first = wave_min(first);
        const bool hit = first != INT_MAX;
        if (hit && lane == 0) atomicMin(result, static_cast<int32_t>(start + first));
        if (hit) break;  // later segments of this wavefront start beyond m
    }
}

// One round over diagonals [i_begin, i_end) (any i outside [max(-t,-m),
// min(t,n)] is written as kNone).  Diagonal i of a row lives at
// row[i + ofs]; every index formed here is inside the row, so no pointer
// ever points before an array (rows in LDS stay LDS addresses).  Called by
// every thread of the workgroup; ends with a workgroup barrier, after which
// `cur` is complete and RS.flag is 1 if f_t[n-m] = n was found.  Diagonals in
// [dlo, dhi] are also copied to dump_row[i + t].  Returns true in the thread
// that found the target.
//
// Tiers of the slide: (1) each lane compares the first cpw characters of each
// of its diagonals (one 64-bit window from two words), all loads in flight
// together; (2) a lane whose LCP runs on
// is extended by its own wavefront, kWaveSteps steps of 4 words per lane;
// (3) the hash engine then finishes with its wavefront-parallel search, the
// direct engine queues the LCP and the whole workgroup extends it after the
// round barrier (the queue and its counter alternate with the round parity,
// so the next round's pushes never meet this round's reads).
template <int WGW, int KU = kU, typename PrevPtr, typename CurPtr>
__device__ __forceinline__ bool round_range(const Engine& en, int32_t t, PrevPtr prev, CurPtr cur,
                                            int32_t ofs, int32_t i_begin, int32_t i_end, RoundShared& RS,
                                            JobCursor& jc, int32_t* dump_row, int32_t dlo, int32_t dhi,
                                            Cnt& cnt, int32_t* deferred = nullptr) {
    const int tid = threadIdx.x;
    constexpr int nthr = kFrontierThreads;  // every launch of the round kernels
    const int lane = tid & 63;
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t lo = imax(-t, -m), hi = imin(t, n);
    const int32_t target = n - m;
    const int32_t cpw = 1 << en.A.lcpw;
    const int par = t & 1;
    const int half = par * kJobHalf;
    const int32_t jstart = jc.start[par];
    bool found = false;
    // first thread of this wavefront, as a uniform value: a slot whose
    // diagonals all lie past i_end is skipped by the whole wavefront
    const int32_t wbase = __builtin_amdgcn_readfirstlane(tid & ~63);
    const int32_t qmask = (1 << en.A.lcpw) - 1;
    for (int32_t base = i_begin; base < i_end; base += nthr * KU) {
        int32_t iv[KU], c[KU], l[KU], lim[KU];
        bool val[KU], act[KU], pend[KU], queued[KU], slot[KU];
        uint64_t wa[KU][2], wb[KU][2];
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            slot[u] = base + u * nthr + wbase < i_end;
            const int32_t i = base + u * nthr + tid;
            iv[u] = i;
            if (!slot[u]) {  // no diagonal of this wavefront (a uniform branch)
                act[u] = val[u] = false;
                c[u] = -1;
                lim[u] = 0;
                continue;
            }
            act[u] = i < i_end;
            const bool inr = act[u] && i >= lo && i <= hi;
            int32_t cc = -1;
            if (inr) {
                if (t == 0) {
                    cc = 0;
                } else {
                    const int32_t a = prev[i + ofs], b = prev[i + ofs - 1], e = prev[i + ofs + 1];
                    cc = imax(imax(a + 1, b + 1), e);  // kNone + 1 stays negative
                    if (cc >= 0) cc = imin(imin(cc, n), m + i);
                }
            }
            c[u] = cc;
            val[u] = inr && cc >= 0;
            lim[u] = val[u] ? imin(n - cc, m - (cc - i)) : 0;
        }
        // (1) two words of A and of B per diagonal (the first cpw characters
        // from any offset), issued for every slot before any use: one memory
        // latency per pass.  Idle lanes read word 0 (always there).
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (!slot[u]) continue;
            const bool go = lim[u] > 0;
            const int32_t qa = go ? c[u] >> en.A.lcpw : 0;
            const int32_t qb = go ? (c[u] - iv[u]) >> en.A.lcpw : 0;
            wa[u][0] = en.A.w[qa];
            wa[u][1] = en.A.w[qa + 1];
            wb[u][0] = en.B.w[qb];
            wb[u][1] = en.B.w[qb + 1];
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            l[u] = 0;
            pend[u] = false;
            queued[u] = false;
            if (!slot[u]) continue;
            const bool go = lim[u] > 0;
            const uint32_t sa = go ? static_cast<uint32_t>(c[u] & qmask) << en.A.lbpc : 0;
            const uint32_t sb = go ? static_cast<uint32_t>((c[u] - iv[u]) & qmask) << en.A.lbpc : 0;
            // (hi << 1) << (63 - sh) equals hi << (64 - sh) and is 0 for sh = 0
            const uint64_t a0 = (wa[u][0] >> sa) | ((wa[u][1] << 1) << (63 - sa));
            const uint64_t b0 = (wb[u][0] >> sb) | ((wb[u][1] << 1) << (63 - sb));
            const uint64_t d = a0 ^ b0;
            // the first mismatch (cpw when none), without branches: every
            // lane takes the same instructions
            const int32_t m0 = d ? (ctz64(d) >> en.A.lbpc) : cpw;
            l[u] = go ? imin(m0, lim[u]) : 0;
            pend[u] = go && m0 == cpw && lim[u] > cpw;
        }
        // (2)/(3) the wavefront extends its lanes' long LCPs
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (!slot[u]) continue;
            wave_extend(en, pend[u], c[u], iv[u], lim[u], l[u], queued[u], RS, par, half, jstart, lane, cnt);
        }
#pragma unroll
        for (int u = 0; u < KU; ++u) {
            if (!slot[u]) continue;
            // (a queued diagonal is written by the workgroup tier)
            const int32_t f = val[u] ? c[u] + l[u] : kNone;
            if (act[u] && !queued[u]) {
                cur[iv[u] + ofs] = f;
                if (dump_row && iv[u] >= dlo && iv[u] <= dhi) dump_row[iv[u] + t] = f;
            }
            // counters and the target test as selects (no branch)
            const bool done = val[u] && !queued[u];
            cnt.updates += done ? 1ull : 0ull;
            cnt.lcp_chars += done ? static_cast<unsigned long long>(l[u]) : 0ull;
            found = found || (done && iv[u] == target && f == n);
        }
    }
    if (found) RS.flag = 1;
    __syncthreads();
    // workgroup tier for the queued LCPs of this round
    const int32_t jend = RS.jcount[par];
    const int32_t nj = imin(jend - jstart, kJobHalf);
    jc.start[par] = jend;
    if (deferred) {
        // the caller extends the queued LCPs (entries [half, half + nj) of the
        // queue), unless the queue overflowed: then which LCPs it holds depends
        // on the order the wavefronts pushed them, and the workgroup tier
        // takes them here
        *deferred = jend - jstart <= kJobHalf ? nj : 0;
        if (*deferred) return found;
    }
    if (nj > 0) {
        for (int j = 0; j < nj; ++j) {
            const int32_t jx = RS.jx[half + j];
            const int32_t jy = RS.jy[half + j], jlim = RS.jlim[half + j], jl = RS.jl[half + j];
            const int32_t r = en.kind == 0 ? lcp_wg_direct<WGW>(en.A, en.B, jx, jy, jlim, jl, RS.wmin)
                                           : lcp_wg_hash<WGW>(en, jx, jy, jlim, jl, RS, cnt);
            if (tid == 0) {
                const int32_t i = RS.ji[half + j];
                const int32_t f = jx + r;
                cur[i + ofs] = f;
                if (dump_row && i >= dlo && i <= dhi) dump_row[i + t] = f;
                cnt.updates++;
                atomicAdd(&cnt.sh->wg_lcps, 1ull);
                cnt.lcp_chars += static_cast<unsigned long long>(r);
                if (i == target && f == n) {
                    found = true;
                    RS.flag = 1;
                }
            }
        }
        __syncthreads();
    }
    return found;
}

// Device-wide barrier: workgroup g > 0 raises its flag to `epoch`; workgroup 0
// waits for every flag, then publishes `epoch` in ctl->release.  Waiting
// loops poll with relaxed loads (no cache invalidation per poll) and take one
// acquire fence once the value arrived.
// Every wait has a deadline of `ticks` s_memrealtime ticks: a waiter that
// reaches it sets ctl->status = 4 and goes on, so that the launch ends (with
// that status, which the host reports as an internal error) whatever happened
// to the workgroup it waited for.
__device__ __forceinline__ void set_wait_error(FrontierCtl* ctl) {
    __hip_atomic_store(&ctl->status, 4, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void grid_sync(FrontierCtl* ctl, unsigned int* bar, unsigned int epoch, uint64_t ticks) {
    __syncthreads();
    const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
    if (blockIdx.x == 0) {
        for (int g = threadIdx.x + 1; g < static_cast<int>(gridDim.x); g += blockDim.x)
            while (__hip_atomic_load(bar + g * kBarStride, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
                if (__builtin_amdgcn_s_memrealtime() - t0 > ticks) {
                    set_wait_error(ctl);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&ctl->release, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else if (threadIdx.x == 0) {
        __hip_atomic_store(bar + blockIdx.x * kBarStride, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(&ctl->release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            if (__builtin_amdgcn_s_memrealtime() - t0 > ticks) {
                set_wait_error(ctl);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// Values every lane holds alike, marked uniform so that they live in scalar
// registers (fields loaded from device memory would otherwise take vector
// registers in every lane).
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni(uint64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(v >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}
template <typename T>
__device__ __forceinline__ const T* uni(const T* p) {
    return reinterpret_cast<const T*>(uni(reinterpret_cast<uint64_t>(p)));
}
__device__ __forceinline__ gword* uni(gword* p) { return (gword*)uni(reinterpret_cast<uint64_t>(p)); }

// KIND (0 direct, 1 hash) is a compile-time constant in every kernel that
// runs rounds, so the other engine's code and fields drop out of it.
template <int KIND>
__device__ __forceinline__ Engine make_engine(const PairDev& p, const HashDev& h, int lane_words,
                                              const uint64_t (*lut32)[256]) {
    Engine en;
    const uint32_t alpha = *p.alpha;
    pair_views(p, alpha, en.A, en.B);
    en.A.w = uni(en.A.w);
    en.B.w = uni(en.B.w);
    en.A.len = uni(en.A.len);
    en.B.len = uni(en.B.len);
    en.A.lcpw = en.B.lcpw = uni(en.A.lcpw);
    en.A.bpc = en.B.bpc = uni(en.A.bpc);
    en.A.lbpc = en.B.lbpc = uni(en.A.lbpc);
    if (KIND == 1) {
        en.TA = uni((gword*)p.a.tab);
        en.TB = uni((gword*)p.b.tab);
        en.q.h.r = uni(h.r);
        en.q.h.pow0 = en.q.h.pow1 = nullptr;
        en.q.pow0 = uni((gword*)h.pow0);
        en.q.pow1 = uni((gword*)h.pow1);
        en.q.r4 = mp_mul(mp_mul(en.q.h.r, en.q.h.r), mp_mul(en.q.h.r, en.q.h.r));
        en.q.r32 = uni(h.pow0[32]);
        en.q.rinv = uni((gword*)(h.rtab + kRtabRinv32));
        en.q.lut32 = lut32;
        en.q.log2b = uni(p.log2b);
    } else {
        en.TA = en.TB = nullptr;
        en.q.h.r = 0;
        en.q.h.pow0 = en.q.h.pow1 = nullptr;
        en.q.pow0 = en.q.pow1 = nullptr;
        en.q.r4 = en.q.r32 = 0;
        en.q.rinv = nullptr;
        en.q.lut32 = nullptr;
        en.q.log2b = 0;
    }
    en.kind = KIND;
    en.lane_words = uni(lane_words);
    en.hash_first = 0;
    return en;
}

// Where round t's row goes in the dump: entry for diagonal i at row[i + t],
// for i in [lo, hi] (the caller's range cut to the dump's window); row is
// nullptr before the dump's first round, past its capacity, or without a dump.
struct DumpAt {
    int32_t* row;
    int32_t lo, hi;
};

__device__ __forceinline__ DumpAt dump_at(const FrontierParams& P, int32_t* dump, int32_t t, int32_t lo,
                                          int32_t hi) {
    DumpAt d{nullptr, lo, hi};
    if (!dump || t < P.dump_t0) return d;
    if (P.dump_cone) {
        if (t > P.dump_kend || cone_off(t + 1, P.dump_kend) > P.dump_cap) return d;
        const KeepLayout L{1, P.dump_t0, 0, 0, P.dump_iend, P.dump_kend};
        int32_t klo, khi;
        int64_t off;
        keep_row(L, t, klo, khi, off);
        d.lo = imax(lo, klo);
        d.hi = imin(hi, khi);
        // row[i + t] = dump[off + i - klo] for i in [lo, hi]
        d.row = dump + (off - klo - t);
    } else if (P.dump_w > 0) {
        const int64_t r = t - P.dump_t0;
        if ((r + 1) * P.dump_w > P.dump_cap) return d;
        d.lo = imax(lo, P.dump_lo);
        d.hi = imin(hi, P.dump_lo + P.dump_w - 1);
        // row[i + t] = dump[r * w + i - lo] for i in [lo, hi]
        d.row = dump + (r * P.dump_w - P.dump_lo - t);
    } else {
        const int64_t base = static_cast<int64_t>(P.dump_t0) * P.dump_t0;
        if (static_cast<int64_t>(t + 1) * (t + 1) - base > P.dump_cap) return d;
        d.row = dump + (static_cast<int64_t>(t) * t - base);
    }
    // the same for every lane: kept in scalar registers
    d.row = reinterpret_cast<int32_t*>(uni(reinterpret_cast<uint64_t>(d.row)));
    d.lo = uni(d.lo);
    d.hi = uni(d.hi);
    return d;
}

// ---------------------------------------------------------------------------
// Work stealing over (pair, diagonal-chunk) tasks.
//
// A pair starts as a whole-pair task: one workgroup runs its rounds with both
// rows in LDS.  When its frontier outgrows `solo_rounds` the workgroup writes
// the row to the pair's global rows and schedules a super-step: the 2T+5
// entries of round T = t + H are cut into chunks of `chunk_diags` diagonals,
// one task each.  A chunk task loads its diagonals plus a halo of H per side,
// runs H rounds in LDS and writes its diagonals back; the workgroup that
// finishes the last chunk of a super-step schedules the next one (or records
// the result).  Tasks travel through a bounded multi-producer multi-consumer
// ring: position p lives in slot p mod cap, whose sequence number is p while
// the slot waits for the push of p and p + 1 once it holds that task.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void q_push(const TaskParams& P, long long task, unsigned long long pos) {
    const uint32_t slot = static_cast<uint32_t>(pos % P.qcap);
    while (__hip_atomic_load(P.qseq + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != pos)
        __builtin_amdgcn_s_sleep(1);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __hip_atomic_store(P.qtask + slot, task, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(P.qseq + slot, pos + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// One thread: the next task, or -1 once no pair of the launch is active.
__device__ __forceinline__ long long q_pop(const TaskParams& P) {
    const unsigned long long pos = atomicAdd(P.qhead, 1ull);
    const uint32_t slot = static_cast<uint32_t>(pos % P.qcap);
    for (;;) {
        if (__hip_atomic_load(P.qseq + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == pos + 1) break;
        if (__hip_atomic_load(P.remaining, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) <= 0) return -1;
        __builtin_amdgcn_s_sleep(2);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const long long task = __hip_atomic_load(P.qtask + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(P.qseq + slot, pos + P.qcap, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    return task;
}

__device__ __forceinline__ void pair_finish(const TaskParams& P, TaskPair* S, int32_t status, int32_t result) {
    S->status = status;
    S->result = result;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_fetch_add(P.remaining, -1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The next super-step of pair pi (f_t in row S->cur), or its result.  Every
// thread of the workgroup calls it: thread 0 takes the decision and reserves
// the ring positions, then the threads push the chunk tasks side by side (one
// position each), so that a super-step of many chunks costs one round trip to
// the ring rather than one per chunk.
__device__ void schedule_superstep(const TaskParams& P, TaskPair* S, int32_t pi, RoundShared& RS) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        RS.nsched = 0;
        const int32_t t = S->t;
        int32_t H = imin(P.block_rounds, S->K - t);
        H = imin(H, (kLdsRowLen - P.chunk_diags) / 2);  // window of a chunk must fit an LDS row
        const int32_t kmax = S->kmax;
        if (kmax >= 0) H = imin(H, kmax - t);
        H = imin(H, S->t_limit - t);
        if (H <= 0) {
            if (kmax >= 0 && t >= kmax) pair_finish(P, S, 2, kmax + 1);
            else if (t >= S->t_limit) pair_finish(P, S, 5, 0);
            else pair_finish(P, S, 3, t);
        } else {
            const int32_t T = t + H;
            const int32_t total = 2 * T + 5;
            const int32_t C = P.chunk_diags;
            const int32_t nch = (total + C - 1) / C;
            S->H = H;
            S->T = T;
            S->chunk = C;
            S->nchunks = nch;
            S->chunks_left = nch;
            S->found_t = INT_MAX;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            RS.qbase = atomicAdd(P.qtail, static_cast<unsigned long long>(nch));
            RS.nsched = nch;
        }
    }
    __syncthreads();
    const int32_t nch = RS.nsched;
    const unsigned long long base = RS.qbase;
    for (int32_t c = tid; c < nch; c += static_cast<int32_t>(blockDim.x))
        q_push(P, static_cast<long long>(static_cast<uint32_t>(pi)) | (static_cast<long long>(c + 1) << 32),
               base + static_cast<unsigned long long>(c));
    __syncthreads();
}

template <int KIND>
__device__ void solo_task(const TaskParams& P, int32_t pi, LdsState& L, JobCursor& jc, Cnt& cnt) {
    TaskPair* S = P.pairs + pi;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const Engine en = make_engine<KIND>(S->p, P.h, P.lane_words, L.lut32);
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t maxnm = imax(n, m);
    const int32_t off = kLdsRoundsMax + 2;  // diagonal i at row[i + off]
    int32_t* la = L.row[0];
    int32_t* lb = L.row[1];
    RoundShared& RS = L.rs;
    int32_t t = uni(S->t);
    const int32_t K = uni(S->K), cur = uni(S->cur), t_limit = uni(S->t_limit), kmax = uni(S->kmax);
    int32_t* g = const_cast<int32_t*>(uni(static_cast<const int32_t*>(cur ? S->f1 : S->f0)));
    if (tid == 0) RS.flag = 0;
    __syncthreads();
    if (t == 0) {
        round_range<kWgWordsTask>(en, 0, la, la, off, -2, 3, RS, jc, nullptr, 0, -1, cnt);
    } else {
        for (int32_t e = tid; e < 2 * t + 5; e += nthr) la[off + e - (t + 2)] = g[K + 2 + e - (t + 2)];
        __syncthreads();
    }
    const int32_t lr = imin(P.solo_rounds, kLdsRoundsMax);
    int32_t status = 0, result = 0;
    for (;;) {
        if (RS.flag) { status = 1; result = t; break; }
        if (kmax >= 0 && t >= kmax) { status = 2; result = kmax + 1; break; }
        if (t > maxnm) { status = 4; result = t; break; }
        if (t >= t_limit) { status = 5; break; }
        if (t >= lr) break;
        ++t;
        round_range<kWgWordsTask>(en, t, la, lb, off, -(t + 2), t + 3, RS, jc, nullptr, 0, -1, cnt);
        int32_t* tmp = la;
        la = lb;
        lb = tmp;
    }
    if (status == 0 || status == 5) {
        // the frontier continues later: it goes to the global row
        if (K < t || g == nullptr) {
            status = 3;
            result = t;
        } else {
            for (int32_t e = tid; e < 2 * t + 5; e += nthr) g[K + 2 + e - (t + 2)] = la[off + e - (t + 2)];
        }
    }
    __syncthreads();
    if (tid == 0) S->t = t;
    if (status != 0) {
        if (tid == 0) pair_finish(P, S, status, result);
    } else {
        schedule_superstep(P, S, pi, RS);
    }
}

template <int KIND>
__device__ void chunk_task(const TaskParams& P, int32_t pi, int32_t c, LdsState& L, JobCursor& jc,
                           Cnt& cnt) {
    TaskPair* S = P.pairs + pi;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const Engine en = make_engine<KIND>(S->p, P.h, P.lane_words, L.lut32);
    RoundShared& RS = L.rs;
    const int32_t t = uni(S->t), H = uni(S->H), T = uni(S->T), C = uni(S->chunk), K = uni(S->K),
                  cur = uni(S->cur);
    const int32_t gofs = K + 2;
    const int32_t* gp = uni(static_cast<const int32_t*>(cur ? S->f1 : S->f0));
    int32_t* gc = const_cast<int32_t*>(uni(static_cast<const int32_t*>(cur ? S->f0 : S->f1)));
    const int32_t total = 2 * T + 5;
    const int32_t eb = c * C;
    const int32_t ee = imin(total, eb + C);
    const int32_t a = eb - (T + 2), b = ee - 1 - (T + 2);
    const int32_t W = (ee - eb) + 2 * H;
    const int32_t wofs = H - a;  // diagonal i of the window at row[i + wofs]
    int32_t* r0 = L.row[0];
    for (int32_t li = tid; li < W; li += nthr) {
        const int32_t i = a - H + li;
        r0[li] = (i >= -(t + 2) && i <= t + 2) ? gp[i + gofs] : kNone;
    }
    __syncthreads();
    int32_t* rp = L.row[0];
    int32_t* rc = L.row[1];
    for (int32_t s = 1; s <= H; ++s) {
        const int32_t tt = t + s;
        if (round_range<kWgWordsTask>(en, tt, rp, rc, wofs, a - (H - s), b + (H - s) + 1, RS, jc, nullptr, 0, -1, cnt))
            atomicMin(&S->found_t, tt);
        int32_t* tmp = rp;
        rp = rc;
        rc = tmp;
    }
    for (int32_t i = a + tid; i <= b; i += nthr) gc[i + gofs] = rp[i + wofs];
    __syncthreads();
    if (tid == 0) {
        int32_t next = 0;
        const int32_t left = __hip_atomic_fetch_add(&S->chunks_left, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (left == 1) {
            // every chunk of the super-step is in: f_T is in row cur ^ 1
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            S->t = T;
            S->cur = cur ^ 1;
            const int32_t ft = __hip_atomic_load(&S->found_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (ft <= T)
                pair_finish(P, S, 1, ft);
            else
                next = 1;
        }
        RS.sched = next;
    }
    __syncthreads();
    if (RS.sched) schedule_superstep(P, S, pi, RS);
}

__device__ __forceinline__ uint64_t clock_now() { return __builtin_amdgcn_s_memrealtime(); }

// ---------------------------------------------------------------------------
// Grid rounds (direct engine): for pairs whose slides run far past a
// workgroup step (a pair within few edits of identity), the first rounds run
// on every workgroup at once.  Each workgroup computes the whole (narrow)
// frontier in its LDS, the same values in every one; the slides that run past
// the wavefront steps are queued, and every workgroup takes its static share
// of the segments of each queued slide (grid_segments over the wavefronts of
// the launch), keeps its own first mismatch and stores it in its slot of
// `part`.  One device-wide barrier later every workgroup reduces the slots of
// each job and completes the same row.  No workgroup waits on another except
// at that barrier, and only rounds with queued slides pay it.
// ---------------------------------------------------------------------------
template <typename CurPtr>
__device__ __forceinline__ bool grid_round_jobs(const Engine& en, int32_t t, CurPtr cur, int32_t ofs, int32_t nj,
                                                RoundShared& RS, int32_t* part, int32_t active_waves,
                                                const DumpAt& dump, FrontierCtl* ctl, unsigned int* bar,
                                                unsigned int& epoch, uint64_t ticks, Cnt& cnt, int32_t& longest) {
    const int tid = threadIdx.x;
    const int G = static_cast<int>(gridDim.x);
    const int32_t n = en.A.len, m = en.B.len, target = n - m;
    const int half = (t & 1) * kJobHalf;
    // this wavefront's place among the wavefronts of the launch, workgroups
    // first, so that the active ones spread over the compute units
    const int32_t wg = (tid >> 6) * G + static_cast<int32_t>(blockIdx.x);
    // the jobs in increasing diagonal order: every workgroup queued the same
    // LCPs, in an order that depends on its wavefronts' timing
    if (tid < nj) {
        const int32_t mine = RS.ji[half + tid];
        int32_t rank = 0;
        for (int k = 0; k < nj; ++k) rank += RS.ji[half + k] < mine ? 1 : 0;
        RS.jorder[rank] = tid;
    }
    __syncthreads();
    // two sets of slots, by the parity of the barrier: a workgroup writes the
    // set of the next barrier only after passing the previous one, which
    // every workgroup reaches only after reading the set it wrote before
    part += ((epoch + 1) & 1) * kGridJobs * kMaxGrid;
    for (int j = 0; j < nj; ++j) {
        const int q = half + RS.jorder[j];
        const int32_t jx = RS.jx[q], jy = RS.jy[q], jlim = RS.jlim[q], jl = RS.jl[q];
        if (tid == 0) RS.gmin = INT_MAX;
        __syncthreads();
        if (wg < active_waves) grid_segments<16>(en.A, en.B, jx, jy, jlim, jl, wg, active_waves, &RS.gmin);
        __syncthreads();
        if (tid == 0) part[j * kMaxGrid + static_cast<int>(blockIdx.x)] = RS.gmin;
    }
    grid_sync(ctl, bar, ++epoch, ticks);
    bool found = false;
    int32_t lmax = 0;
    for (int j = 0; j < nj; ++j) {
        // the first mismatch over every workgroup's share
        int32_t v = INT_MAX;
        for (int g = tid; g < G; g += kFrontierThreads) v = imin(v, part[j * kMaxGrid + g]);
        v = wave_min(v);
        if (tid == 0) RS.gmin = INT_MAX;
        __syncthreads();
        if ((tid & 63) == 0 && v != INT_MAX) atomicMin(&RS.gmin, v);
        __syncthreads();
        const int q = half + RS.jorder[j];
        const int32_t jx = RS.jx[q], jlim = RS.jlim[q];
        const int32_t r = imin(RS.gmin, jlim);
        lmax = imax(lmax, r);
        if (tid == 0) {
            const int32_t i = RS.ji[q];
            const int32_t f = jx + r;
            cur[i + ofs] = f;
            if (dump.row && i >= dump.lo && i <= dump.hi) dump.row[i + t] = f;
            cnt.updates++;
            atomicAdd(&cnt.sh->grid_lcps, 1ull);
            cnt.lcp_chars += static_cast<unsigned long long>(r);
            if (i == target && f == n) {
                found = true;
                RS.flag = 1;
            }
        }
        __syncthreads();
    }
    longest = lmax;
    return found;
}

}  // namespace

__global__ void ctl_init_kernel(FrontierCtl* ctl, CountersDev* cnt, unsigned int* bar) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        ctl->release = 0;
        ctl->phase = 0;
        ctl->phase_t = 0;
        ctl->found_t = INT_MAX;
        ctl->status = 0;
        ctl->result_t = 0;
        ctl->wbuf = 0;
        ctl->clk_begin = 0;
        ctl->clk_switch = 0;
        ctl->clk_end = 0;
    }
    if (cnt)
        for (int i = tid; i < static_cast<int>((kMaxGrid + 1) * sizeof(CountersDev) / 8); i += blockDim.x)
            reinterpret_cast<unsigned long long*>(cnt)[i] = 0;
    if (bar)
        for (int g = tid; g < kMaxGrid; g += blockDim.x) bar[g * kBarStride] = 0;
}

template <int KIND, bool DUMP>
__global__ __launch_bounds__(kFrontierThreads) void frontier_kernel(FrontierParams P) {
    __shared__ LdsState L;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int G = gridDim.x;
    Cnt cnt;
    cnt_bind(cnt, &L.cnt);
    cnt_init_shared(&L.cnt);
    JobCursor jc;
    rs_init(L.rs, jc);
    if (KIND == 1) load_lut32(L.lut32, P.h.rtab, tid, nthr);
    __syncthreads();
    Engine en = make_engine<KIND>(P.p, P.h, P.lane_words, L.lut32);
    en.hash_first = KIND == 1 ? uni(P.hash_first) : 0;
    int32_t* const dump = DUMP ? P.dump : nullptr;
    RoundShared& RS = L.rs;
    const int32_t n = en.A.len, m = en.B.len;
    const int32_t maxnm = imax(n, m);
    FrontierCtl* ctl = P.ctl;
    const int32_t K = P.K;
    int32_t t = P.t0;
    const int32_t gofs = K + 2;  // diagonal i of a global row at row[i + gofs]
    int32_t* gp = P.f0;          // holds f_t
    int32_t* gc = P.f1;
    bool finished = false;
    unsigned int epoch = 0;
    if (blockIdx.x == 0 && tid == 0) ctl->clk_begin = clock_now();

    if (P.t0 == 0) {
        const int32_t off = kLdsRoundsMax + 2;  // diagonal i at row[i + off]
        int32_t* la = L.row[0];
        int32_t* lb = L.row[1];
        const int32_t lr = imin(imin(P.lds_rounds, kLdsRoundsMax), K);
        int32_t status = 0, result = 0;
        bool started = false;  // round 0 done by the grid rounds
        bool to_b = false;     // the grid rounds reached the end of the LDS phase
        // ---------------- grid rounds: every workgroup, rows in LDS ----------------
        if (KIND == 0 && P.grid_rounds) {
            // slides longer than this keep the grid rounds going: about 16
            // workgroup-tier steps (4M characters at 2 bits), where a round of
            // the grid tier (one pass of segments, one barrier, the
            // reduction; about 15-30 us here) beats the workgroup's dependent
            // steps (about 3.5 us each)
            const int32_t big = (128 * kFrontierThreads) << en.A.lcpw;
            const int32_t span = (64 * 16) << en.A.lcpw;  // one wavefront's segment
            const int32_t all_waves = G * (kFrontierThreads >> 6);
            int32_t* const dump0 = blockIdx.x == 0 ? dump : nullptr;
            int32_t nj = 0, longest = 0, quiet = 0, est = INT_MAX;
            auto resolve = [&](int32_t tt, int32_t* cur, const DumpAt& drow) {
                longest = 0;
                if (nj > 0) {
                    // wavefronts for about twice the longest slide of the last round
                    const int64_t need = est == INT_MAX ? all_waves : 2 * (static_cast<int64_t>(est) / span + 1);
                    const int32_t aw = static_cast<int32_t>(need < 64 ? 64 : (need > all_waves ? all_waves : need));
                    grid_round_jobs(en, tt, cur, off, nj, RS, P.gpart, aw, drow, ctl, P.bar, epoch, P.wait_ticks,
                                    cnt, longest);
                    est = longest;
                }
            };
            {
                const DumpAt d = dump_at(P, dump0, 0, 0, 0);
                round_range<kWgWords>(en, 0, la, la, off, -2, 3, RS, jc, d.row, d.lo, d.hi, cnt, &nj);
                resolve(0, la, d);
            }
            started = true;
            for (;;) {
                if (RS.flag) { status = 1; result = t; break; }
                if (P.kmax >= 0 && t >= P.kmax) { status = 2; result = P.kmax + 1; break; }
                if (t > maxnm) { status = 4; result = t; break; }
                if (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 4) {
                    status = 4;
                    result = t;
                    break;
                }
                quiet = longest >= big ? 0 : quiet + 1;
                if (t == 0 ? quiet > 0 : quiet >= 8) break;  // back to one workgroup
                if (t >= lr) {
                    to_b = true;
                    break;
                }
                ++t;
                const DumpAt d = dump_at(P, dump0, t, -t, t);
                round_range<kWgWords>(en, t, la, lb, off, -(t + 2), t + 3, RS, jc, d.row, d.lo, d.hi, cnt, &nj);
                resolve(t, lb, d);
                int32_t* tmp = la;
                la = lb;
                lb = tmp;
            }
            if (blockIdx.x != 0) {
                // the same rounds as workgroup 0: counted there only
                __syncthreads();
                cnt.updates = cnt.lcp_chars = cnt.ne_len = 0;
                cnt_init_shared(&L.cnt);
                __syncthreads();
            }
            if (status != 0 || to_b) {
                if ((to_b || status == 2) && blockIdx.x == 0)
                    for (int32_t e = tid; e < 2 * t + 5; e += nthr) gp[gofs + e - (t + 2)] = la[off + e - (t + 2)];
                if (blockIdx.x == 0 && tid == 0) {
                    ctl->clk_switch = clock_now();
                    ctl->wbuf = 0;
                    ctl->phase_t = t;
                    if (status != 0) {
                        ctl->result_t = result;
                        __hip_atomic_store(&ctl->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                    }
                }
                finished = status != 0;
                // the row of round t is read by every workgroup in phase B
                if (to_b) grid_sync(ctl, P.bar, ++epoch, P.wait_ticks);
            }
        }
        if (status != 0 || to_b) {
            // (decided alike by every workgroup in the grid rounds)
        } else if (blockIdx.x == 0) {
            // ---------------- phase A: workgroup 0, rows in LDS ----------------
            if (!started) {
                const DumpAt d = dump_at(P, dump, 0, 0, 0);
                round_range<kWgWords>(en, 0, la, la, off, -2, 3, RS, jc, d.row, d.lo, d.hi, cnt);
            }
            for (;;) {
                if (RS.flag) { status = 1; result = t; break; }
                if (P.kmax >= 0 && t >= P.kmax) { status = 2; result = P.kmax + 1; break; }
                if (t > maxnm) { status = 4; result = t; break; }
                if (t >= lr) break;
                ++t;
                const DumpAt d = dump_at(P, dump, t, -t, t);
                round_range<kWgWords>(en, t, la, lb, off, -(t + 2), t + 3, RS, jc, d.row, d.lo, d.hi, cnt);
                int32_t* tmp = la;
                la = lb;
                lb = tmp;
            }
            // (also when k_max stopped the rounds: the state a later launch resumes from)
            if (status == 0 || status == 2)
                for (int32_t e = tid; e < 2 * t + 5; e += nthr) gp[gofs + e - (t + 2)] = la[off + e - (t + 2)];
            __syncthreads();
            if (tid == 0) {
                ctl->clk_switch = clock_now();
                ctl->wbuf = 0;
                if (status != 0) {
                    ctl->result_t = result;
                    ctl->phase_t = t;
                    __hip_atomic_store(&ctl->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    ctl->phase_t = t;
                }
                __hip_atomic_store(&ctl->phase, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            finished = status != 0;
        } else {
            if (tid == 0) {
                // relaxed polling (no cache invalidation per poll), one acquire fence
                const uint64_t t0 = clock_now();
                while (__hip_atomic_load(&ctl->phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
                    if (clock_now() - t0 > P.wait_ticks) {
                        set_wait_error(ctl);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(64);
                }
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
            if (tid == 0)
                RS.flag = __hip_atomic_load(&ctl->status, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            finished = RS.flag != 0;
            if (!finished) t = __hip_atomic_load(&ctl->phase_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (blockIdx.x == 0 && tid == 0) {
        ctl->clk_switch = ctl->clk_begin;
        ctl->phase_t = t;
    }

    // ---------------- phase B: every workgroup, H rounds per barrier ----------------
    if (!finished) {
        for (;;) {
            // a wait gave up somewhere (set before the last barrier): every workgroup stops here
            if (__hip_atomic_load(&ctl->status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 4) {
                if (blockIdx.x == 0 && tid == 0) ctl->result_t = t;
                break;
            }
            // found_t only holds rounds of finished blocks once everyone passed the barrier
            const int32_t ft = __hip_atomic_load(&ctl->found_t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            int32_t status = 0, result = 0;
            if (ft <= t) { status = 1; result = ft; }
            else if (P.kmax >= 0 && t >= P.kmax) { status = 2; result = P.kmax + 1; }
            else if (t > maxnm) { status = 4; result = t; }
            else if (t >= K) { status = 3; result = t; }
            if (status != 0) {
                if (blockIdx.x == 0 && tid == 0) {
                    ctl->result_t = result;
                    ctl->wbuf = gp == P.f0 ? 0 : 1;
                    __hip_atomic_store(&ctl->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
                break;
            }
            int32_t H = imin(imax(P.block_rounds, 1), K - t);
            if (P.kmax >= 0) H = imin(H, P.kmax - t);
            const int32_t T = t + H;
            const int32_t total = 2 * T + 5;
            const int32_t chunk = (total + G - 1) / G;
            const int32_t eb = imin(total, static_cast<int32_t>(blockIdx.x) * chunk);
            const int32_t ee = imin(total, eb + chunk);
            const int32_t a = eb - (T + 2), b = ee - 1 - (T + 2);  // owned diagonals
            const bool in_lds = chunk + 2 * H <= kLdsRowLen;
            if (!in_lds) {
                // slices too wide for LDS: one round per barrier on the global rows
                const int32_t t1 = t + 1;
                const int32_t total1 = 2 * t1 + 5;
                const int32_t c1 = (total1 + G - 1) / G;
                const int32_t e0 = imin(total1, static_cast<int32_t>(blockIdx.x) * c1);
                const int32_t e1 = imin(total1, e0 + c1);
                const DumpAt d = dump_at(P, dump, t1, -t1, t1);
                if (e0 < e1 && round_range<kWgWords>(en, t1, gp, gc, gofs, e0 - (t1 + 2), e1 - (t1 + 2), RS, jc,
                                                     d.row, d.lo, d.hi, cnt))
                    atomicMin(&ctl->found_t, t1);
                grid_sync(ctl, P.bar, ++epoch, P.wait_ticks);
                int32_t* tmp = gp;
                gp = gc;
                gc = tmp;
                t = t1;
                continue;
            }
            if (eb < ee) {
                // window [a - H, b + H] in LDS: diagonal i at row[i + wofs],
                // wofs = H - a, so every index used is in [0, W)
                const int32_t W = (b - a + 1) + 2 * H;
                const int32_t wofs = H - a;
                int32_t* r0 = L.row[0];
                for (int32_t li = tid; li < W; li += nthr) {
                    const int32_t i = a - H + li;
                    r0[li] = (i >= -(t + 2) && i <= t + 2) ? gp[i + gofs] : kNone;
                }
                __syncthreads();
                int32_t* rp = L.row[0];
                int32_t* rc = L.row[1];
                for (int32_t s = 1; s <= H; ++s) {
                    const int32_t tt = t + s;
                    const DumpAt d = dump_at(P, dump, tt, imax(a, -tt), imin(b, tt));
                    // one diagonal per thread when the window fits the workgroup
                    const bool one = (b - a + 1) + 2 * (H - s) <= kFrontierThreads;
                    const bool hit =
                        one ? round_range<kWgWords, 1>(en, tt, rp, rc, wofs, a - (H - s), b + (H - s) + 1, RS, jc,
                                                       d.row, d.lo, d.hi, cnt)
                            : round_range<kWgWords, kU>(en, tt, rp, rc, wofs, a - (H - s), b + (H - s) + 1, RS, jc,
                                                        d.row, d.lo, d.hi, cnt);
                    if (hit) atomicMin(&ctl->found_t, tt);
                    int32_t* tmp = rp;
                    rp = rc;
                    rc = tmp;
                }
                for (int32_t i = a + tid; i <= b; i += nthr) gc[i + gofs] = rp[i + wofs];
            }
            grid_sync(ctl, P.bar, ++epoch, P.wait_ticks);
            int32_t* tmp = gp;
            gp = gc;
            gc = tmp;
            t = T;
        }
    }
    if (blockIdx.x == 0 && tid == 0) ctl->clk_end = clock_now();
    flush_counters(cnt, P.counters);
}

template <int KIND>
__global__ __launch_bounds__(kFrontierThreads) void task_kernel(TaskParams P) {
    __shared__ LdsState L;
    const int tid = threadIdx.x;
    Cnt cnt;
    cnt_bind(cnt, &L.cnt);
    cnt_init_shared(&L.cnt);
    JobCursor jc;
    rs_init(L.rs, jc);
    if (KIND == 1) load_lut32(L.lut32, P.h.rtab, tid, blockDim.x);
    for (;;) {
        __syncthreads();
        if (tid == 0) L.rs.task = q_pop(P);
        __syncthreads();
        const long long task = static_cast<long long>(uni(static_cast<uint64_t>(L.rs.task)));
        if (task < 0) break;
        const int32_t pi = static_cast<int32_t>(task & 0xFFFFFFFFll);
        const uint32_t c = static_cast<uint32_t>(static_cast<unsigned long long>(task) >> 32);
        if (c == kTaskSolo)
            solo_task<KIND>(P, pi, L, jc, cnt);
        else
            chunk_task<KIND>(P, pi, static_cast<int32_t>(c - 1), L, jc, cnt);
    }
    flush_counters(cnt, P.counters);
}

__global__ __launch_bounds__(256) void lcp_query_kernel(LcpQueryParams Q) {
    __shared__ uint64_t lut32[8][256];
    __shared__ CountersDev sh;
    Cnt cnt;
    cnt_bind(cnt, &sh);
    cnt_init_shared(&sh);
    if (Q.engine == 1) load_lut32(lut32, Q.h.rtab, threadIdx.x, blockDim.x);
    __syncthreads();
    const Engine en = Q.engine == 1 ? make_engine<1>(Q.p, Q.h, Q.lane_words, lut32)
                                    : make_engine<0>(Q.p, Q.h, Q.lane_words, lut32);
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

// Grid tier queries: one launch per query, every workgroup of the grid on it.
__global__ __launch_bounds__(kFrontierThreads) void lcp_grid_kernel(LcpQueryParams Q) {
    const Engine en = make_engine<0>(Q.p, Q.h, Q.lane_words, nullptr);
    const int64_t qi = Q.query;
    const int32_t x = static_cast<int32_t>(Q.x[qi]);
    const int32_t y = static_cast<int32_t>(Q.y[qi]);
    const int32_t lim = imin(en.A.len - x, en.B.len - y);
    const int32_t waves = blockDim.x >> 6;
    grid_segments<16>(en.A, en.B, x, y, lim, 0, static_cast<int32_t>(blockIdx.x) * waves + (threadIdx.x >> 6),
                      static_cast<int32_t>(gridDim.x) * waves, Q.result + qi);
}

// Workgroup-tier LCP queries: one workgroup per query (tests of the tier).
__global__ __launch_bounds__(kFrontierThreads) void lcp_query_wg_kernel(LcpQueryParams Q) {
    __shared__ int32_t wmin;
    const Engine en = make_engine<0>(Q.p, Q.h, Q.lane_words, nullptr);
    for (int64_t qi = blockIdx.x; qi < Q.count; qi += gridDim.x) {
        const int32_t x = static_cast<int32_t>(Q.x[qi]);
        const int32_t y = static_cast<int32_t>(Q.y[qi]);
        const int32_t la = en.A.len - x, lb = en.B.len - y;
        const int32_t lim = la < lb ? la : lb;
        const int32_t l = lcp_wg_direct<kWgWords>(en.A, en.B, x, y, lim, 0, wmin);
        if (threadIdx.x == 0) Q.out[qi] = l;
    }
}

// Sums the per-workgroup counter slots into slot kMaxGrid.
__global__ __launch_bounds__(1024) void counters_sum_kernel(CountersDev* cnt) {
    constexpr int F = sizeof(CountersDev) / 8;
    __shared__ unsigned long long acc[F];
    if (threadIdx.x < F) acc[threadIdx.x] = 0;
    __syncthreads();
    const unsigned long long* slot = reinterpret_cast<const unsigned long long*>(cnt + threadIdx.x);
    for (int f = 0; f < F; ++f)
        if (slot[f]) atomicAdd(&acc[f], slot[f]);
    __syncthreads();
    if (threadIdx.x < F) reinterpret_cast<unsigned long long*>(cnt + kMaxGrid)[threadIdx.x] = acc[threadIdx.x];
}

hipError_t launch_counters_sum(CountersDev* cnt, hipStream_t s) {
    hipLaunchKernelGGL(counters_sum_kernel, dim3(1), dim3(kMaxGrid), 0, s, cnt);
    return hipGetLastError();
}

hipError_t launch_ctl_init(FrontierCtl* ctl, CountersDev* cnt, unsigned int* bar, hipStream_t s) {
    hipLaunchKernelGGL(ctl_init_kernel, dim3(1), dim3(256), 0, s, ctl, cnt, bar);
    return hipGetLastError();
}

hipError_t frontier_max_grid(int device, int* grid_out) {
    int cus = 0, per = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    // the smallest occupancy over the instantiations (all run the same grid)
    const void* kernels[] = {reinterpret_cast<const void*>(frontier_kernel<0, false>),
                             reinterpret_cast<const void*>(frontier_kernel<0, true>),
                             reinterpret_cast<const void*>(frontier_kernel<1, false>),
                             reinterpret_cast<const void*>(frontier_kernel<1, true>)};
    per = 1 << 30;
    for (const void* k : kernels) {
        int q = 0;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&q, k, kFrontierThreads, 0);
        if (e != hipSuccess) return e;
        per = q < per ? q : per;
    }
    if (per < 1) per = 1;
    int g = cus * per;
    *grid_out = g < kMaxGrid ? g : kMaxGrid;
    return hipSuccess;
}

hipError_t launch_frontier(const FrontierParams& fp, int grid, hipStream_t s) {
    FrontierParams arg = fp;
    void* args[] = {&arg};
    const void* k = fp.engine == 1 ? (fp.dump ? reinterpret_cast<const void*>(frontier_kernel<1, true>)
                                              : reinterpret_cast<const void*>(frontier_kernel<1, false>))
                                   : (fp.dump ? reinterpret_cast<const void*>(frontier_kernel<0, true>)
                                              : reinterpret_cast<const void*>(frontier_kernel<0, false>));
    return hipLaunchCooperativeKernel(k, dim3(grid), dim3(kFrontierThreads), args, 0, s);
}

hipError_t task_max_grid(int device, int* grid_out) {
    int cus = 0, per = 0;
    hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) return e;
    int per1 = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(task_kernel<0>),
                                                     kFrontierThreads, 0);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, reinterpret_cast<const void*>(task_kernel<1>),
                                                     kFrontierThreads, 0);
    if (e != hipSuccess) return e;
    per = per1 < per ? per1 : per;
    if (per < 1) per = 1;
    *grid_out = cus * per;
    return hipSuccess;
}

hipError_t launch_tasks(const TaskParams& tp, int grid, hipStream_t s) {
    if (tp.engine == 1)
        hipLaunchKernelGGL(task_kernel<1>, dim3(grid), dim3(kFrontierThreads), 0, s, tp);
    else
        hipLaunchKernelGGL(task_kernel<0>, dim3(grid), dim3(kFrontierThreads), 0, s, tp);
    return hipGetLastError();
}

__global__ void lcp_grid_finish_kernel(LcpQueryParams Q) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < Q.count) {
        const int32_t lim = imin(Q.p.a.len - static_cast<int32_t>(Q.x[i]), Q.p.b.len - static_cast<int32_t>(Q.y[i]));
        Q.out[i] = imin(Q.result[i], lim);
    }
}

hipError_t launch_lcp_grid_finish(const LcpQueryParams& qp, hipStream_t s) {
    const int64_t blocks = (qp.count + 255) / 256;
    hipLaunchKernelGGL(lcp_grid_finish_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, qp);
    return hipGetLastError();
}

hipError_t launch_lcp_grid(const LcpQueryParams& qp, int grid, hipStream_t s) {
    hipLaunchKernelGGL(lcp_grid_kernel, dim3(grid), dim3(kFrontierThreads), 0, s, qp);
    return hipGetLastError();
}

hipError_t launch_lcp_queries(const LcpQueryParams& qp, hipStream_t s) {
    if (qp.engine == 2) {
        int64_t blocks = qp.count < 1 ? 1 : qp.count;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(lcp_query_wg_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kFrontierThreads), 0, s, qp);
        return hipGetLastError();
    }
    int64_t waves = qp.count < 1 ? 1 : qp.count;
    int64_t blocks = (waves + 3) / 4;
    if (blocks > 2048) blocks = 2048;
    hipLaunchKernelGGL(lcp_query_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, qp);
    return hipGetLastError();
}

}  // namespace ed
