// ed_align and the check behind ED_FLAG_CERTIFY (host side): k from the
// frontier (or from the pair's last unbounded distance on the same engine),
// the frontier rounds again with every row kept in device memory,
// the path traced back on the device, its geometry checked here, and its runs
// of matches re-compared on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "../../include/ed.h"
#include "host.h"
#include "internal.h"

using namespace ed;

namespace {

// Device buffers of one call, freed on every exit.
struct DevBufs {
    std::vector<void*> held;
    void* get(size_t bytes) {
        void* q = nullptr;
        if (hipMalloc(&q, bytes) != hipSuccess) return nullptr;
        held.push_back(q);
        return q;
    }
    ~DevBufs() {
        for (void* q : held) (void)hipFree(q);
    }
};

// Every step is one edit (or none) from the previous one, the runs stay in
// the grid and the path ends at (n, m); returns the number of edits, or -1.
int64_t path_cost(const std::vector<PathStep>& path, int64_t n, int64_t m) {
    int64_t cost = 0;
    for (size_t t = 0; t < path.size(); ++t) {
        const PathStep& s = path[t];
        if (s.c < 0 || s.c > s.f || s.f > n || s.c - s.i < 0 || s.f - s.i > m) return -1;
        if (t == 0) {
            if (s.kind != kStepStart || s.i != 0 || s.c != 0) return -1;
            continue;
        }
        const PathStep& q = path[t - 1];
        switch (s.kind) {
            case kStepSub:
                if (s.i != q.i || s.c != q.f + 1) return -1;
                ++cost;
                break;
            case kStepDel:
                if (s.i != q.i + 1 || s.c != q.f + 1) return -1;
                ++cost;
                break;
            case kStepIns:
                if (s.i != q.i - 1 || s.c != q.f) return -1;
                ++cost;
                break;
            case kStepNone:
                if (s.i != q.i || s.c != q.f) return -1;
                break;
            default:
                return -1;
        }
    }
    const PathStep& e = path.back();
    if (e.i != n - m || e.f != n) return -1;
    return cost;
}

}  // namespace

int ed::align_locked(ed_ctx* c, ed_pair* p, uint64_t* k_out, std::vector<PathStep>& path, hipStream_t s) {
    uint64_t k = 0;
    int rc = ED_OK;
    if (p->known_k >= 0 && p->known_engine == p->engine)
        k = static_cast<uint64_t>(p->known_k);  // computed before on this pair and engine
    else
        rc = distance_locked(c, p, -1, &k, nullptr, 0, s);
    if (rc != ED_OK) return rc;
    const int64_t n = static_cast<int64_t>(p->len[0]), m = static_cast<int64_t>(p->len[1]);
    const uint64_t cap = (k + 1) * (k + 1);
    const size_t dump_bytes = cap * 4;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess || dump_bytes + (size_t(256) << 20) > free_b) {
        set_error("ed_align: the rows of %llu rounds need %zu bytes of device memory", (unsigned long long)(k + 1),
                  dump_bytes);
        return ED_ENOMEM;
    }
    DevBufs db;
    int32_t* d_dump = static_cast<int32_t*>(db.get(dump_bytes));
    PathStep* d_path = static_cast<PathStep*>(db.get((k + 1) * sizeof(PathStep) + 64));
    if (!d_dump || !d_path) {
        set_error("ed_align: device allocation failed");
        return ED_ENOMEM;
    }
    int32_t* d_status = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_path) + (k + 1) * sizeof(PathStep));
    uint64_t k2 = 0;
    rc = distance_locked(c, p, static_cast<int64_t>(k), &k2, nullptr, 0, s, d_dump, cap);
    if (rc != ED_OK) return rc;
    if (k2 != k) {
        set_error("ed_align: the second run gave %llu, the first %llu", (unsigned long long)k2,
                  (unsigned long long)k);
        return ED_EINTERNAL;
    }
    path.assign(k + 1, PathStep{});
    int32_t status = -1;
    hipError_t e = launch_traceback(d_dump, static_cast<int32_t>(k), static_cast<int32_t>(n),
                                    static_cast<int32_t>(m), d_path, d_status, s);
    if (e == hipSuccess) e = hipMemcpyAsync(path.data(), d_path, (k + 1) * sizeof(PathStep), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&status, d_status, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("ed_align: traceback failed: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    const int64_t cost = status == 0 ? path_cost(path, n, m) : -1;
    if (cost < 0 || cost > static_cast<int64_t>(k)) {
        set_error("ed_align: the traced path is not a valid alignment (status %d, cost %lld, k %llu)", status,
                  (long long)cost, (unsigned long long)k);
        return ED_EINTERNAL;
    }
    // the runs of matches, in segments of at most 2048 characters
    std::vector<VerifySeg> segs;
    for (const PathStep& st : path)
        for (int32_t x = st.c; x < st.f; x += 2048)
            segs.push_back(VerifySeg{x, x - st.i, std::min<int32_t>(2048, st.f - x), 0});
    uint32_t bad = 0;
    if (!segs.empty()) {
        VerifySeg* d_segs = static_cast<VerifySeg*>(db.get(segs.size() * sizeof(VerifySeg) + 64));
        if (!d_segs) {
            set_error("ed_align: device allocation failed");
            return ED_ENOMEM;
        }
        uint32_t* d_bad = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_segs) + segs.size() * sizeof(VerifySeg));
        e = hipMemsetAsync(d_bad, 0, 4, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_segs, segs.data(), segs.size() * sizeof(VerifySeg), hipMemcpyHostToDevice, s);
        if (e == hipSuccess)
            e = launch_verify(pair_dev(p), d_segs, static_cast<int64_t>(segs.size()), d_bad, c->num_cu * 8, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&bad, d_bad, 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("ed_align: check failed: %s", hipGetErrorString(e));
            return ED_EDEVICE;
        }
    }
    *k_out = k;
    if (bad) {
        set_error("ed_align: a run of matches on the traced path does not match (hash collision)");
        return ED_ECOLLISION;
    }
    return ED_OK;
}

int ed_align(ed_ctx* c, ed_pair* p, uint64_t* k_out, ed_op_run* runs, uint64_t runs_cap, uint64_t* n_runs,
             void* hip_stream) {
    if (!c || !p || !k_out || !n_runs || p->ctx != c || (runs_cap && !runs)) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) {
        set_error("ed_align: hipSetDevice failed");
        return ED_EDEVICE;
    }
    if (!p->script_kept) {
        std::vector<PathStep> path;
        const int rc = align_locked(c, p, &p->script_k, path, static_cast<hipStream_t>(hip_stream));
        if (rc != ED_OK) {
            *k_out = p->script_k;
            return rc;
        }
        // the edit script: the step's edit, then its run of matches (merged)
        std::vector<ed_op_run>& out = p->script;
        out.clear();
        auto push = [&](uint32_t op, uint64_t len) {
            if (!len) return;
            if (!out.empty() && out.back().op == op)
                out.back().len += len;
            else
                out.push_back(ed_op_run{op, 0, len});
        };
        for (const PathStep& st : path) {
            if (st.kind == kStepSub) push(ED_OP_SUB, 1);
            if (st.kind == kStepDel) push(ED_OP_DEL, 1);
            if (st.kind == kStepIns) push(ED_OP_INS, 1);
            push(ED_OP_MATCH, static_cast<uint64_t>(st.f - st.c));
        }
        p->script_kept = true;
    }
    *k_out = p->script_k;
    *n_runs = p->script.size();
    if (p->script.size() > runs_cap) {
        // kept: a call with a buffer this large returns it without recomputing
        set_error("ed_align: %llu runs do not fit in %llu", (unsigned long long)p->script.size(),
                  (unsigned long long)runs_cap);
        return ED_EINVAL;
    }
    if (!p->script.empty()) std::memcpy(runs, p->script.data(), p->script.size() * sizeof(ed_op_run));
    std::vector<ed_op_run>().swap(p->script);
    p->script_kept = false;
    return ED_OK;
}

int ed_debug_check_runs(ed_ctx* c, ed_pair* p, const int32_t* x, const int32_t* y, const int32_t* len, uint64_t count,
                        uint32_t* bad, void* hip_stream) {
    if (!c || !p || !bad || p->ctx != c || (count && (!x || !y || !len))) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return ED_EDEVICE;
    const int64_t n = static_cast<int64_t>(p->len[0]), m = static_cast<int64_t>(p->len[1]);
    std::vector<VerifySeg> segs;
    for (uint64_t i = 0; i < count; ++i) {
        if (x[i] < 0 || y[i] < 0 || len[i] < 0 || x[i] + int64_t(len[i]) > n || y[i] + int64_t(len[i]) > m) {
            set_error("ed_debug_check_runs: run %llu outside the strings", (unsigned long long)i);
            return ED_EINVAL;
        }
        for (int32_t o = 0; o < len[i]; o += 2048)
            segs.push_back(VerifySeg{x[i] + o, y[i] + o, std::min<int32_t>(2048, len[i] - o), 0});
    }
    *bad = 0;
    if (segs.empty()) return ED_OK;
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    DevBufs db;
    VerifySeg* d_segs = static_cast<VerifySeg*>(db.get(segs.size() * sizeof(VerifySeg) + 64));
    if (!d_segs) return ED_ENOMEM;
    uint32_t* d_bad = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(d_segs) + segs.size() * sizeof(VerifySeg));
    hipError_t e = hipMemsetAsync(d_bad, 0, 4, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_segs, segs.data(), segs.size() * sizeof(VerifySeg), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = launch_verify(pair_dev(p), d_segs, static_cast<int64_t>(segs.size()), d_bad, c->num_cu * 8, s);
    if (e == hipSuccess) e = hipMemcpyAsync(bad, d_bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("ed_debug_check_runs: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    return ED_OK;
}
