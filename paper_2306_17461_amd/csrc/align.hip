// Alignment output and its check (the certificate for the hash engine).
//
// The frontier rows f_t of every round (the per-round dump of the frontier
// kernel) determine an optimal alignment: at round t the path's diagonal i
// holds f_t[i] = slide(c) with c the clamped maximum of f_{t-1}[i] + 1,
// f_{t-1}[i-1] + 1 and f_{t-1}[i+1] (Algorithm 1, section 3.1); the candidate
// that produced c names the edit and the diagonal of round t - 1.  Walking
// from (t = k, i = n - m) back to round 0 gives k + 1 runs of matches joined
// by single edits.  Re-comparing every run's characters directly turns a
// hash-engine distance into a checked one: a collision can only make an LCP
// too long (so k too small), and a path of cost <= k whose runs all match
// shows that the edit distance is at most k (section 3.3 notes that the
// hash-based method is Monte Carlo; this check removes the error).
#include "device.h"

namespace ed {

namespace {
__device__ __forceinline__ int32_t amax(int32_t a, int32_t b) { return a > b ? a : b; }
__device__ __forceinline__ int32_t amin(int32_t a, int32_t b) { return a < b ? a : b; }
}  // namespace

// The path moves by at most one diagonal per round, so the next kTbRows
// rounds of the walk stay within kTbRows + 1 diagonals of the current one:
// the wavefront loads that band of the next kTbRows rows into LDS (one load
// per lane and row, all in flight together), then one lane takes the steps.
// The rows are those of rounds tb .. te in layout L (row u holds diagonals
// [lo(u), hi(u)]); the walk starts on diagonal i_end of round te, and every
// cell it reads lies within te - u + 1 diagonals of i_end at row u, which
// the layout keeps.  It ends at round tb, whose diagonal and row value it
// leaves in state[1], state[2] (state[0]: 0 ok, 1 the walk did not end at
// (0, 0), 2 no candidate).
constexpr int kTbRows = 30;

__global__ __launch_bounds__(64) void traceback_kernel(const int32_t* dump, KeepLayout L, int32_t tb, int32_t te,
                                                       int32_t i_end, int32_t n, int32_t m, PathStep* out,
                                                       int32_t* state) {
    __shared__ int32_t band[kTbRows][64];  // band[r][l]: row t0 - 1 - r, diagonal ic - 32 + l
    __shared__ int32_t sh[4];              // i, f, t, finished
    const int lane = threadIdx.x;
    if (lane == 0) {
        int32_t lo, hi;
        int64_t off;
        keep_row(L, te, lo, hi, off);
        sh[0] = i_end;
        sh[1] = dump[off + (i_end - lo)];
        sh[2] = te;
        sh[3] = 0;
        state[0] = 0;
    }
    __syncthreads();
    for (;;) {
        const int32_t ic = sh[0], t0 = sh[2];
        if (t0 == tb) {
            if (lane == 0) {
                if (tb == 0) {
                    out[0] = PathStep{sh[0], 0, sh[1], kStepStart};
                    if (sh[0] != 0) state[0] = 1;
                }
                state[1] = sh[0];
                state[2] = sh[1];
            }
            return;
        }
        const int32_t R = amin(kTbRows, t0 - tb);
        // every row's load issued before any is stored to LDS (one memory
        // latency per band, not one per row)
        int32_t v[kTbRows];
#pragma unroll
        for (int32_t r = 0; r < kTbRows; ++r) {
            const int32_t u = t0 - 1 - r;
            const int32_t j = ic - 32 + lane;
            int32_t lo, hi;
            int64_t off = 0;
            if (r < R) keep_row(L, u, lo, hi, off);
            const bool in = r < R && j >= -u && j <= u && j >= lo && j <= hi;
            v[r] = in ? dump[off + (j - lo)] : kNone;
        }
#pragma unroll
        for (int32_t r = 0; r < kTbRows; ++r) band[r][lane] = v[r];
        __syncthreads();
        if (lane == 0) {
            int32_t i = ic, f = sh[1];
            bool failed = false;
            for (int32_t r = 0; r < R && !failed; ++r) {
                const int32_t t = t0 - r;  // round of the current state; row t - 1 is band[r]
                const int32_t* row = band[r] + (32 - ic);
                const int32_t fa = row[i], fb = row[i - 1], fe = row[i + 1];
                int32_t C = amax(amax(fa + 1, fb + 1), fe);  // kNone + 1 stays negative
                C = amin(amin(C, n), m + i);
                int32_t kind, j, fj;
                if (fa >= 0 && fa + 1 == C) {
                    kind = kStepSub, j = i, fj = fa;
                } else if (fb >= 0 && fb + 1 == C) {
                    kind = kStepDel, j = i - 1, fj = fb;
                } else if (fe >= 0 && fe == C) {
                    kind = kStepIns, j = i + 1, fj = fe;
                } else if (fa >= 0 && fa == C) {
                    kind = kStepNone, j = i, fj = fa;
                } else {
                    out[t] = PathStep{i, C, f, kStepFail};
                    state[0] = 2;
                    failed = true;
                    break;
                }
                out[t] = PathStep{i, C, f, kind};
                i = j;
                f = fj;
            }
            sh[0] = i;
            sh[1] = f;
            sh[2] = failed ? tb : t0 - R;
            sh[3] = failed ? 1 : 0;
        }
        __syncthreads();
        if (sh[3]) return;
    }
}

// Each wavefront takes segments w, w + W, ...; lane l compares words l,
// l + 64, ... of its segment (characters from any offset, the last word
// masked to the segment's end).
__global__ __launch_bounds__(256) void verify_kernel(PairDev p, const VerifySeg* segs, int64_t count, uint32_t* bad) {
    SView A, B;
    pair_views(p, *p.alpha, A, B);
    const int lane = threadIdx.x & 63;
    const int64_t wave = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) >> 6;
    const int64_t nwaves = (static_cast<int64_t>(gridDim.x) * blockDim.x) >> 6;
    const int32_t cpw = 1 << A.lcpw;
    uint64_t diff = 0;
    for (int64_t sidx = wave; sidx < count; sidx += nwaves) {
        const VerifySeg sg = segs[sidx];
        for (int32_t o = lane * cpw; o < sg.len; o += 64 * cpw) {
            uint64_t d = fetch(A, sg.x + o) ^ fetch(B, sg.y + o);
            const int32_t rest = sg.len - o;
            if (rest < cpw) d &= (1ull << (rest << A.lbpc)) - 1;
            diff |= d;
        }
    }
    if (ballot(diff != 0) && lane == 0) atomicOr(bad, 1u);
}

hipError_t launch_traceback(const int32_t* dump, const KeepLayout& L, int32_t tb, int32_t te, int32_t i_end,
                            int32_t n, int32_t m, PathStep* out, int32_t* state, hipStream_t s) {
    hipLaunchKernelGGL(traceback_kernel, dim3(1), dim3(64), 0, s, dump, L, tb, te, i_end, n, m, out, state);
    return hipGetLastError();
}

hipError_t launch_verify(const PairDev& p, const VerifySeg* segs, int64_t count, uint32_t* bad, int grid,
                         hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t need = (count + 3) / 4;  // four wavefronts per workgroup
    if (grid > need) grid = static_cast<int>(need);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(verify_kernel, dim3(grid), dim3(256), 0, s, p, segs, count, bad);
    return hipGetLastError();
}

}  // namespace ed
