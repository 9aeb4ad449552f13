// Serving: a request loop with continuous batching.
//
// Submitted requests wait in a host queue.  A worker thread repeats one step:
//   1. one launch of the work-stealing task kernel, on the server's stream,
//      advances every active slot by a round budget (whole-pair tasks in LDS,
//      chunked super-steps for wide frontiers); a slot's frontier is saved in
//      its rows when its budget is used up;
//   2. while that launch runs, admission: while a slot is free and the
//      request's device bytes (packed strings, 8-bit copies, tables, staging
//      and frontier rows) fit in the HBM budget, the request is copied and
//      prepared on the server's second stream, and its slot joins the next
//      launch; its strings and tables stay resident until it finishes;
//   3. after the launch, finished slots are recorded with their completion
//      time and freed.
// Requests that arrive while others run join at the next step, so work of
// different requests shares every launch.  The round budget is kServeRounds
// while requests wait for admission, kServeRoundsIdle when none does (fewer
// launches for long requests).  A request may carry its own k_max (the band
// |x - y| <= k_max of section 3.1): it then ends after round k_max with
// k_max + 1 when its distance is larger.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/ed.h"
#include "host.h"
#include "internal.h"

using namespace ed;

namespace {

constexpr int32_t kServeRounds = 256;       // rounds per slot per launch while requests wait
constexpr int32_t kServeRoundsIdle = 2048;  // ... while none does
constexpr size_t kServeQueueMax = 1u << 20;

uint64_t now_ns() {
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now().time_since_epoch())
                                     .count());
}

struct Request {
    uint64_t tag;
    std::vector<uint8_t> A, B;
    uint64_t t_arrive;
    int64_t k_max;  // -1: none
};

struct Slot {
    ed_pair* pair = nullptr;
    uint64_t tag = 0;
    uint64_t t_arrive = 0;
    int64_t k_max = -1;
    TaskPair st{};
    void* rows = nullptr;
    int64_t K = 0;
    uint64_t bytes = 0;
};

}  // namespace

struct ed_server {
    ed_ctx* ctx = nullptr;
    uint64_t budget = 0;
    uint32_t max_slots = 0;
    std::mutex mu;
    std::condition_variable cv_work;  // new request or stop
    std::condition_variable cv_done;  // a request finished
    std::deque<Request> pending;
    std::vector<ed_result> done;
    uint64_t submitted = 0, completed = 0;
    bool stop = false;
    int error = ED_OK;
    std::thread worker;
    hipStream_t stream = nullptr;       // task launches
    hipStream_t prep_stream = nullptr;  // admission: copies and packing, beside the running launch
    uint64_t used = 0;
    std::vector<Slot> slots;
};

namespace {

uint64_t pool_bytes(uint64_t b) { return b + (b >> 3) + 4096; }  // size-class slack

// Device bytes a request holds while resident.
uint64_t request_bytes(const ed_ctx* c, uint64_t n, uint64_t m, int64_t K) {
    uint64_t total = 0;
    const uint32_t b = c->opt.block ? c->opt.block : 32;
    for (uint64_t len : {n, m}) {
        const uint64_t tiles = std::max<uint64_t>(1, (len + kTileChars - 1) / kTileChars);
        total += pool_bytes((tiles * kTileWords2 + kPadWords) * 8);
        total += pool_bytes((tiles * kTileWords8 + kPadWords) * 8);
        total += pool_bytes(len + 16);  // staging copy of the host input
        if (c->opt.engine == ED_ENGINE_HASH) total += pool_bytes((len / b + 1) * 8);
    }
    total += pool_bytes(static_cast<uint64_t>(2 * (2 * K + 5)) * 4);
    return total;
}

int64_t serve_rows(const ed_ctx* c, int64_t maxnm, int64_t k_max) {
    const int64_t solo = task_solo_rounds(c);
    // every slot can save its frontier at any round up to the whole-pair limit
    int64_t K = std::max<int64_t>(std::min<int64_t>(maxnm, 2 * solo), maxnm / 16);
    if (k_max >= 0) K = std::min<int64_t>(K, std::max<int64_t>(k_max, 1));
    return std::max<int64_t>(1, std::min<int64_t>(K, maxnm));
}

void slot_free(ed_server* S, Slot& sl) {
    ed_ctx* c = S->ctx;
    if (sl.pair) {
        pair_free(sl.pair);
        delete sl.pair;
    }
    c->pool.put(sl.rows);
    S->used -= sl.bytes;
    sl = Slot();
}

// Grows the rows of a slot whose frontier reached their capacity.
int slot_grow(ed_server* S, Slot& sl) {
    ed_ctx* c = S->ctx;
    const int64_t maxnm = std::max<int64_t>(sl.st.p.a.len, sl.st.p.b.len);
    const int64_t t = sl.st.t;
    int64_t K2 = std::min<int64_t>(maxnm, std::max<int64_t>(2 * sl.K, t + kServeRoundsIdle + 1));
    if (sl.k_max >= 0) K2 = std::min<int64_t>(K2, std::max<int64_t>(sl.k_max, 1));
    if (K2 <= sl.K) return ED_EINTERNAL;
    void* nr = c->pool.get(static_cast<size_t>(2 * (2 * K2 + 5)) * 4);
    if (!nr) return ED_ENOMEM;
    int32_t* old = sl.st.cur ? sl.st.f1 : sl.st.f0;
    int32_t* nf0 = static_cast<int32_t*>(nr);
    hipError_t e = hipMemcpyAsync(nf0 + (K2 + 2) - (t + 2), old + (sl.K + 2) - (t + 2),
                                  static_cast<size_t>(2 * t + 5) * 4, hipMemcpyDeviceToDevice, S->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) {
        c->pool.put(nr);
        return ED_EDEVICE;
    }
    c->pool.put(sl.rows);
    S->used += static_cast<uint64_t>(4 * 2 * (2 * (K2 - sl.K)));
    sl.bytes += static_cast<uint64_t>(4 * 2 * (2 * (K2 - sl.K)));
    sl.rows = nr;
    sl.K = K2;
    sl.st.K = static_cast<int32_t>(K2);
    sl.st.f0 = nf0;
    sl.st.f1 = nf0 + (2 * K2 + 5);
    sl.st.cur = 0;
    return ED_OK;
}

void finish_slot(ed_server* S, Slot& sl, uint64_t k, int32_t status) {
    ed_result r;
    std::memset(&r, 0, sizeof r);
    r.tag = sl.tag;
    r.k = k;
    r.status = status;
    r.t_arrive_ns = sl.t_arrive;
    r.t_done_ns = now_ns();
    slot_free(S, sl);
    std::lock_guard<std::mutex> lk(S->mu);
    S->done.push_back(r);
    S->completed++;
    S->cv_done.notify_all();
}

// One launch + admission + collection step.  Called with ctx->mu held.
int serve_step(ed_server* S, std::vector<Request>& admitted_now, int32_t budget) {
    ed_ctx* c = S->ctx;
    // 1. one launch over every active slot (admitted in earlier steps)
    const int32_t solo = static_cast<int32_t>(task_solo_rounds(c));
    const int32_t br = block_rounds_of(c);
    std::vector<TaskPair> st;
    std::vector<long long> tasks;
    std::vector<size_t> idx;
    for (size_t j = 0; j < S->slots.size(); ++j) {
        Slot& sl = S->slots[j];
        if (sl.st.t >= sl.st.K && sl.st.t > solo && (sl.k_max < 0 || sl.st.t < sl.k_max)) {
            int rc = slot_grow(S, sl);
            if (rc != ED_OK) {
                sl.st.status = 4;
                continue;
            }
        }
        TaskPair tp = sl.st;
        tp.status = 0;
        tp.t_limit = tp.t + budget;
        const int32_t pi = static_cast<int32_t>(st.size());
        if (tp.t <= solo && tp.t <= kLdsRoundsMax) {
            tasks.push_back(task_solo(pi));
        } else if (!schedule_on_host(tp, pi, br, chunk_diags_of(c), tp.kmax, tasks)) {
            if (tp.kmax >= 0 && tp.t >= tp.kmax) {
                sl.st.status = 2;
                sl.st.result = tp.kmax + 1;
            } else {
                sl.st.status = 4;
            }
            continue;
        }
        st.push_back(tp);
        idx.push_back(j);
    }
    TaskRun run;
    bool launched = false;
    if (!st.empty()) {
        int rc = tasks_start(c, st, tasks, c->opt.engine, S->stream, run);
        if (rc != ED_OK) return rc;
        launched = true;
    }
    // 2. admission, beside the launch: copies and packing on the second stream
    std::vector<Slot> fresh;
    for (Request& rq : admitted_now) {
        Slot sl;
        const int64_t maxnm = static_cast<int64_t>(std::max(rq.A.size(), rq.B.size()));
        sl.K = serve_rows(c, maxnm, rq.k_max);
        sl.bytes = request_bytes(c, rq.A.size(), rq.B.size(), sl.K);
        sl.tag = rq.tag;
        sl.t_arrive = rq.t_arrive;
        sl.k_max = rq.k_max;
        int rc = prepare_locked(c, rq.A.data(), rq.A.size(), rq.B.data(), rq.B.size(), 0, S->prep_stream, &sl.pair);
        if (rc == ED_OK) {
            sl.rows = c->pool.get(static_cast<size_t>(2 * (2 * sl.K + 5)) * 4);
            if (!sl.rows) rc = ED_ENOMEM;
        }
        S->used += sl.bytes;
        if (rc != ED_OK) {
            finish_slot(S, sl, 0, rc);
            continue;
        }
        std::memset(&sl.st, 0, sizeof sl.st);
        sl.st.p = pair_dev(sl.pair);
        sl.st.K = static_cast<int32_t>(sl.K);
        sl.st.f0 = static_cast<int32_t*>(sl.rows);
        sl.st.f1 = sl.st.f0 + (2 * sl.K + 5);
        sl.st.found_t = INT32_MAX;
        sl.st.kmax = rq.k_max >= 0 ? static_cast<int32_t>(std::min<int64_t>(rq.k_max, INT32_MAX - 1)) : -1;
        fresh.push_back(sl);
    }
    // 3. the launch's results; the prepared strings are in place before the
    // next launch reads them
    if (launched) {
        int rc = tasks_wait(c, st, S->stream, run);
        if (rc != ED_OK) return rc;
        for (size_t q = 0; q < st.size(); ++q) S->slots[idx[q]].st = st[q];
    }
    if (!admitted_now.empty() && hipStreamSynchronize(S->prep_stream) != hipSuccess) {
        set_error("serve: admission stream failed");
        return ED_EDEVICE;
    }
    // collection
    std::vector<Slot> keep;
    keep.reserve(S->slots.size() + fresh.size());
    for (Slot& sl : S->slots) {
        const int32_t status = sl.st.status;
        if (status == 1 || status == 2) {
            // (2: the request's k_max was reached; the result is k_max + 1)
            sl.pair->rounds = static_cast<uint64_t>(sl.st.result);
            finish_slot(S, sl, static_cast<uint64_t>(sl.st.result), ED_OK);
        } else if (status == 4) {
            finish_slot(S, sl, 0, ED_EINTERNAL);
        } else {
            // round budget used (5) or rows full (3): continue next step
            sl.st.status = 0;
            keep.push_back(sl);
        }
    }
    for (Slot& sl : fresh) keep.push_back(sl);
    S->slots.swap(keep);
    return ED_OK;
}

void serve_worker(ed_server* S) {
    ed_ctx* c = S->ctx;
    (void)hipSetDevice(c->device);
    for (;;) {
        std::vector<Request> adm;
        int32_t budget = kServeRounds;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || !S->slots.empty(); });
            if (S->stop && S->slots.empty() && S->pending.empty()) return;
            budget = S->pending.empty() ? kServeRoundsIdle : kServeRounds;
            // admit by free slots and the HBM budget, in arrival order
            uint64_t used = S->used;
            size_t active = S->slots.size();
            while (!S->pending.empty() && active < S->max_slots) {
                Request& rq = S->pending.front();
                const int64_t maxnm = static_cast<int64_t>(std::max(rq.A.size(), rq.B.size()));
                const uint64_t need = request_bytes(c, rq.A.size(), rq.B.size(), serve_rows(c, maxnm, rq.k_max));
                if (used + need > S->budget) break;
                used += need;
                adm.push_back(std::move(rq));
                S->pending.pop_front();
                ++active;
            }
        }
        int rc;
        {
            std::lock_guard<std::mutex> lk(c->mu);
            rc = serve_step(S, adm, budget);
        }
        if (rc != ED_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            S->error = rc;
            S->stop = true;
            // fail everything left
            for (Request& rq : S->pending) {
                ed_result r;
                std::memset(&r, 0, sizeof r);
                r.tag = rq.tag;
                r.status = rc;
                r.t_arrive_ns = rq.t_arrive;
                r.t_done_ns = now_ns();
                S->done.push_back(r);
                S->completed++;
            }
            S->pending.clear();
            S->cv_done.notify_all();
            return;
        }
    }
}

}  // namespace

int ed_serve_open(ed_ctx* c, uint64_t hbm_budget_bytes, uint32_t max_slots, ed_server** out) {
    if (!c || !out || max_slots == 0 || hbm_budget_bytes == 0) return ED_EINVAL;
    *out = nullptr;
    ed_server* S = new (std::nothrow) ed_server();
    if (!S) return ED_ENOMEM;
    S->ctx = c;
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    {
        std::lock_guard<std::mutex> lk(c->mu);
        if (hipSetDevice(c->device) != hipSuccess || hipStreamCreate(&S->stream) != hipSuccess ||
            hipStreamCreate(&S->prep_stream) != hipSuccess) {
            if (S->stream) (void)hipStreamDestroy(S->stream);
            delete S;
            set_error("ed_serve_open: hipStreamCreate failed");
            return ED_EDEVICE;
        }
    }
    S->worker = std::thread(serve_worker, S);
    *out = S;
    return ED_OK;
}

int ed_serve_submit_band(ed_server* S, const uint8_t* A, uint64_t n, const uint8_t* B, uint64_t m, uint64_t tag,
                         int64_t k_max) {
    if (!S || (n && !A) || (m && !B) || n >= ED_MAX_LEN || m >= ED_MAX_LEN || k_max < -1) return ED_EINVAL;
    const int64_t maxnm = static_cast<int64_t>(std::max(n, m));
    if (request_bytes(S->ctx, n, m, serve_rows(S->ctx, maxnm, k_max)) > S->budget) {
        set_error("ed_serve_submit: request needs more than the HBM budget");
        return ED_ENOMEM;
    }
    Request rq;
    rq.tag = tag;
    rq.A.assign(A, A + n);
    rq.B.assign(B, B + m);
    rq.t_arrive = now_ns();
    rq.k_max = k_max;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return S->error != ED_OK ? S->error : ED_EINVAL;
    if (S->pending.size() >= kServeQueueMax) return ED_EBUSY;
    S->pending.push_back(std::move(rq));
    S->submitted++;
    S->cv_work.notify_one();
    return ED_OK;
}

int ed_serve_submit(ed_server* S, const uint8_t* A, uint64_t n, const uint8_t* B, uint64_t m, uint64_t tag) {
    return ed_serve_submit_band(S, A, n, B, m, tag, -1);
}

int ed_serve_poll(ed_server* S, ed_result* out, uint32_t max, uint32_t* got) {
    if (!S || !got || (max && !out)) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(S->mu);
    const uint32_t k = static_cast<uint32_t>(std::min<size_t>(max, S->done.size()));
    for (uint32_t i = 0; i < k; ++i) out[i] = S->done[i];
    S->done.erase(S->done.begin(), S->done.begin() + k);
    *got = k;
    return ED_OK;
}

int ed_serve_drain(ed_server* S) {
    if (!S) return ED_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    S->cv_done.wait(lk, [&] { return S->completed >= S->submitted || S->stop; });
    return S->error;
}

int ed_serve_close(ed_server* S) {
    if (!S) return ED_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->pending.clear();
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    {
        std::lock_guard<std::mutex> lk(S->ctx->mu);
        for (Slot& sl : S->slots) slot_free(S, sl);
        S->slots.clear();
        if (S->stream) (void)hipStreamDestroy(S->stream);
        if (S->prep_stream) (void)hipStreamDestroy(S->prep_stream);
    }
    const int err = S->error;
    delete S;
    return err;
}
