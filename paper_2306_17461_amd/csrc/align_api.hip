// ed_align and the check behind ED_FLAG_CERTIFY (host side).
//
// Forward: the frontier rounds run in segments of S rounds (one launch
// each, resumed from the previous segment's last row), and the row at each
// segment's end is kept; the last segment ends where the end cell is reached,
// which gives k.  Backward, last segment first: the segment's rounds run
// again from its kept first row with the rows kept for the diagonals that the
// path can reach from its known end (within one diagonal per round), and the
// path is traced back on the device through them to the segment's first
// round.  Device memory is about k^2 / S + 2 S^2 entries instead of the
// (k + 1)^2 of every row.  The path's geometry is checked here, its runs of
// matches re-compared on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
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

// Rounds per segment between kept rows.  The kept rows of a distance k take
// about k^2 / S entries and one segment's window of rows about 2 S^2, least
// for S near (k^2 / 4)^(1/3); S grows with the rounds when k is not known
// yet.  At least kMinSegment rounds, so that the launches (a few tens of
// microseconds each, with a traceback and a synchronisation per segment) stay
// few.
constexpr int64_t kMinSegment = 1024;

int64_t segment_rounds(int64_t k) {
    const double kk = static_cast<double>(std::max<int64_t>(k, 1));
    return std::max<int64_t>(kMinSegment, static_cast<int64_t>(std::llround(std::cbrt(kk * kk / 4.0))));
}

// A kept row: round t, diagonals -(t + 2) .. t + 2 at row[0 ..] (nullptr for
// round 0, which a launch from round 0 computes itself, and for round k).
struct Checkpoint {
    int64_t t;
    int32_t* row;
};

}  // namespace

int ed::align_locked(ed_ctx* c, ed_pair* p, uint64_t* k_out, std::vector<PathStep>& path, hipStream_t s) {
    FrontierParams fp;
    int rc = frontier_setup(c, p, fp);
    if (rc != ED_OK) return rc;
    const int64_t n = static_cast<int64_t>(p->len[0]), m = static_cast<int64_t>(p->len[1]);
    const int64_t maxnm = std::max(n, m);
    const int64_t known = (p->known_k >= 0 && p->known_engine == p->engine) ? p->known_k : -1;
    DevBufs db;
    // the two frontier rows (pooled), grown like the distance's
    int64_t K = std::max<int64_t>(1, std::min<int64_t>(maxnm, known >= 0 ? known : int64_t(1) << 17));
    struct Rows {
        ed_ctx* c;
        int32_t* r[2] = {nullptr, nullptr};
        ~Rows() {
            c->pool.put(r[0]);
            c->pool.put(r[1]);
        }
    } rows{c};
    rows.r[0] = static_cast<int32_t*>(c->pool.get(static_cast<size_t>(2 * K + 5) * 4));
    rows.r[1] = static_cast<int32_t*>(c->pool.get(static_cast<size_t>(2 * K + 5) * 4));
    if (!rows.r[0] || !rows.r[1]) {
        set_error("ed_align: device allocation failed");
        return ED_ENOMEM;
    }
    int cur = 0;  // rows.r[cur] holds the current round's row
    // checkpoint rows, bump-allocated from chunks: row of round t at
    // row[i + t + 2] for diagonals -(t + 2) .. t + 2
    std::vector<Checkpoint> ck{Checkpoint{0, nullptr}};
    int32_t* chunk = nullptr;
    int64_t chunk_left = 0;
    uint64_t ck_bytes = 0;
    auto ck_alloc = [&](int64_t len) -> int32_t* {
        if (len > chunk_left) {
            const int64_t sz = std::max<int64_t>(len, int64_t(1) << 24);
            chunk = static_cast<int32_t*>(db.get(static_cast<size_t>(sz) * 4));
            if (!chunk) return nullptr;
            chunk_left = sz;
            ck_bytes += static_cast<uint64_t>(sz) * 4;
        }
        int32_t* r = chunk;
        chunk += len;
        chunk_left -= len;
        return r;
    };
    double gpu_ns = 0;
    auto launch = [&](int64_t t0, int64_t t1) -> int {
        fp.f0 = rows.r[cur];
        fp.f1 = rows.r[1 - cur];
        fp.K = static_cast<int32_t>(K);
        fp.t0 = static_cast<int32_t>(t0);
        fp.kmax = static_cast<int32_t>(t1);
        return frontier_once(c, fp, s, &gpu_ns);
    };

    // with k known, one launch may keep every row the path can reach (the
    // cone of diagonals within k - u of the end at round u, about k^2 / 2
    // entries) when that fits an eighth of the free device memory: no kept
    // rows, no segments
    const int64_t iend = n - m;
    bool cone = false;
    if (known >= 0 && !(c->opt.flags & ED_FLAG_ALIGN_SEGMENTS)) {
        size_t free_b = 0, total_b = 0;
        cone = hipMemGetInfo(&free_b, &total_b) == hipSuccess &&
               static_cast<uint64_t>(cone_total(known)) * 4 <= free_b / 8;
    }

    // forward: the rounds in segments, the row at each segment's end kept
    // (with k unknown, these launches are the distance's)
    int64_t k = cone ? known : -1;
    CountersDev total;
    std::memset(&total, 0, sizeof total);
    int launches = 0;
    for (int64_t t = 0; k < 0;) {
        const int64_t t1 = std::min(maxnm, t + segment_rounds(known >= 0 ? known : t));
        if (known >= 0 && t1 >= known) {
            k = known;
            break;
        }
        if (t1 <= t && t > 0) {  // (t1 = t = 0 only for two empty strings)
            set_error("ed_align: no end found by round %lld", (long long)t);
            return ED_EINTERNAL;
        }
        if (t1 > K) {
            const int64_t K2 = std::min<int64_t>(maxnm, std::max<int64_t>(2 * K, t1));
            int32_t* g0 = static_cast<int32_t*>(c->pool.get(static_cast<size_t>(2 * K2 + 5) * 4));
            int32_t* g1 = static_cast<int32_t*>(c->pool.get(static_cast<size_t>(2 * K2 + 5) * 4));
            hipError_t e = (g0 && g1) ? hipSuccess : hipErrorOutOfMemory;
            if (e == hipSuccess && t > 0)
                e = hipMemcpyAsync(g0 + (K2 + 2) - (t + 2), rows.r[cur] + (K + 2) - (t + 2),
                                   static_cast<size_t>(2 * t + 5) * 4, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            c->pool.put(rows.r[0]);
            c->pool.put(rows.r[1]);
            rows.r[0] = g0;
            rows.r[1] = g1;
            cur = 0;
            if (e != hipSuccess) {
                set_error("ed_align: growing the rows failed: %s", hipGetErrorString(e));
                return e == hipErrorOutOfMemory ? ED_ENOMEM : ED_EDEVICE;
            }
            K = K2;
        }
        fp.dump = nullptr;
        rc = launch(t, t1);
        if (rc != ED_OK) return rc;
        ++launches;
        counters_add(total, *c->h_cnt);
        const FrontierCtl& st = *c->h_ctl;
        if (st.status == 1) {
            k = st.result_t;
            break;
        }
        if (st.status != 2) {
            set_error("ed_align: frontier kernel ended with status %d at t=%d", st.status, st.result_t);
            return ED_EINTERNAL;
        }
        if (st.wbuf != 0) cur = 1 - cur;  // the row of round t1
        int32_t* r = ck_alloc(2 * t1 + 5);
        if (!r) {
            set_error("ed_align: device allocation failed (checkpoint row of round %lld)", (long long)t1);
            return ED_ENOMEM;
        }
        const hipError_t e = hipMemcpyAsync(r, rows.r[cur] + (K + 2) - (t1 + 2), static_cast<size_t>(2 * t1 + 5) * 4,
                                            hipMemcpyDeviceToDevice, s);
        if (e != hipSuccess) {
            set_error("ed_align: checkpoint copy failed: %s", hipGetErrorString(e));
            return ED_EDEVICE;
        }
        ck.push_back(Checkpoint{t1, r});
        t = t1;
    }
    if (known < 0) {
        p->known_k = k;
        p->known_engine = p->engine;
        p->rounds = static_cast<uint64_t>(k);
        p->counters = total;
        p->launches_distance = launches;
        p->gpu_ns_frontier = gpu_ns;
        p->rounds_phase_a = 0;
        p->us_phase_a = p->us_phase_b = 0;
    }
    ck.push_back(Checkpoint{k, nullptr});

    PathStep* d_path = static_cast<PathStep*>(db.get((k + 1) * sizeof(PathStep) + 64));
    if (!d_path) {
        set_error("ed_align: device allocation failed");
        return ED_ENOMEM;
    }
    int32_t* d_state = reinterpret_cast<int32_t*>(reinterpret_cast<char*>(d_path) + (k + 1) * sizeof(PathStep));
    int32_t state[4] = {0, static_cast<int32_t>(iend), 0, 0};
    if (cone) {
        // one launch from round 0 with the cone of rows kept, one traceback
        const int64_t tot = cone_total(k);
        int32_t* d_keep = static_cast<int32_t*>(db.get(static_cast<size_t>(tot) * 4));
        if (!d_keep) {
            set_error("ed_align: device allocation failed");
            return ED_ENOMEM;
        }
        fp.dump = d_keep;
        fp.dump_cap = tot;
        fp.dump_cone = 1;
        fp.dump_t0 = 0;
        fp.dump_iend = static_cast<int32_t>(iend);
        fp.dump_kend = static_cast<int32_t>(k);
        rc = launch(0, k);
        if (rc != ED_OK) return rc;
        const FrontierCtl& st = *c->h_ctl;
        if (st.status != 1 || st.result_t != k) {
            set_error("ed_align: the rounds ended with status %d at t=%d, the distance is %lld", st.status,
                      st.result_t, (long long)k);
            return ED_EINTERNAL;
        }
        const KeepLayout L{1, 0, 0, 0, static_cast<int32_t>(iend), static_cast<int32_t>(k)};
        hipError_t e = launch_traceback(d_keep, L, 0, static_cast<int32_t>(k), static_cast<int32_t>(iend),
                             static_cast<int32_t>(n), static_cast<int32_t>(m), d_path, d_state, s);
        if (e == hipSuccess) e = hipMemcpyAsync(state, d_state, 3 * 4, hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            set_error("ed_align: traceback failed: %s", hipGetErrorString(e));
            return ED_EDEVICE;
        }
        p->align_bytes = static_cast<uint64_t>(tot) * 4 + (k + 1) * sizeof(PathStep) + 64;
        p->align_seg = static_cast<uint64_t>(k);
    } else {
        // backward: each segment's rounds again from its first row, the rows
        // kept for the diagonals the path can reach, and the path traced
        // through them
        int64_t seg_cap = 0;
        for (size_t j = 0; j + 1 < ck.size(); ++j) {
            const int64_t L = ck[j + 1].t - ck[j].t;
            seg_cap = std::max(seg_cap, (L + 1) * (2 * L + 5));
        }
        int32_t* d_seg = static_cast<int32_t*>(db.get(static_cast<size_t>(seg_cap) * 4));
        if (!d_seg) {
            set_error("ed_align: device allocation failed");
            return ED_ENOMEM;
        }
        p->align_bytes = ck_bytes + static_cast<uint64_t>(seg_cap) * 4 + (k + 1) * sizeof(PathStep) + 64;
        p->align_seg = static_cast<uint64_t>(segment_rounds(known >= 0 ? known : k));
        for (size_t j = ck.size() - 1; j-- > 0;) {
            const int64_t tb = ck[j].t, te = ck[j + 1].t, L = te - tb;
            const int64_t i_end = state[1];
            const int64_t wlo = i_end - L - 2, w = 2 * L + 5;
            hipError_t e = hipSuccess;
            if (tb > 0) {
                // the segment's first row: into the frontier row, and its window into the dump
                e = hipMemcpyAsync(rows.r[cur] + (K + 2) - (tb + 2), ck[j].row, static_cast<size_t>(2 * tb + 5) * 4,
                                   hipMemcpyDeviceToDevice, s);
                const int64_t d0 = std::max(wlo, -tb), d1 = std::min(wlo + w - 1, tb);
                if (e == hipSuccess && d0 <= d1)
                    e = hipMemcpyAsync(d_seg + (d0 - wlo), ck[j].row + (d0 + tb + 2),
                                       static_cast<size_t>(d1 - d0 + 1) * 4, hipMemcpyDeviceToDevice, s);
            }
            if (e != hipSuccess) {
                set_error("ed_align: row copy failed: %s", hipGetErrorString(e));
                return ED_EDEVICE;
            }
            fp.dump = d_seg;
            fp.dump_cap = (L + 1) * w;
            fp.dump_cone = 0;
            fp.dump_t0 = static_cast<int32_t>(tb);
            fp.dump_lo = static_cast<int32_t>(wlo);
            fp.dump_w = static_cast<int32_t>(w);
            rc = launch(tb, te);
            if (rc != ED_OK) return rc;
            const FrontierCtl& st = *c->h_ctl;
            const bool last = te == k;
            if (st.status != (last ? 1 : 2) || st.result_t != (last ? k : te + 1)) {
                set_error("ed_align: segment [%lld, %lld] ended with status %d at t=%d", (long long)tb, (long long)te,
                          st.status, st.result_t);
                return ED_EINTERNAL;
            }
            const KeepLayout Lw{0, static_cast<int32_t>(tb), static_cast<int32_t>(wlo), static_cast<int32_t>(w), 0, 0};
            e = launch_traceback(d_seg, Lw, static_cast<int32_t>(tb), static_cast<int32_t>(te),
                                 static_cast<int32_t>(i_end), static_cast<int32_t>(n), static_cast<int32_t>(m), d_path,
                                 d_state, s);
            if (e == hipSuccess) e = hipMemcpyAsync(state, d_state, 3 * 4, hipMemcpyDeviceToHost, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) {
                set_error("ed_align: traceback failed: %s", hipGetErrorString(e));
                return ED_EDEVICE;
            }
            if (state[0] != 0) break;
        }
    }
    path.assign(k + 1, PathStep{});
    hipError_t e = hipMemcpyAsync(path.data(), d_path, (k + 1) * sizeof(PathStep), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("ed_align: path copy failed: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    const int64_t cost = state[0] == 0 ? path_cost(path, n, m) : -1;
    if (cost < 0 || cost > k) {
        set_error("ed_align: the traced path is not a valid alignment (status %d, cost %lld, k %lld)", state[0],
                  (long long)cost, (long long)k);
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
    *k_out = static_cast<uint64_t>(k);
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
