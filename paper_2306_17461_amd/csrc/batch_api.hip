// ed_batch: many prepared pairs in one persistent launch.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/ed.h"
#include "host.h"
#include "internal.h"

using namespace ed;

namespace {

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

namespace ed {

// Rows capacity guess for a pair inside a batch: pairs that outgrow it are
// finished by the single-pair path (which grows its rows).
int64_t batch_row_capacity(int64_t maxnm, int64_t k_max, uint32_t lds_rounds) {
    if (maxnm <= static_cast<int64_t>(lds_rounds)) return 0;
    int64_t K = std::max<int64_t>(2 * static_cast<int64_t>(lds_rounds), maxnm / 16);
    K = std::min<int64_t>(K, maxnm);
    if (k_max >= 0) K = std::min<int64_t>(K, std::max<int64_t>(k_max, 1));
    return K;
}

// Device buffers of one task launch (pair states, queue, rows).
struct TaskLaunch {
    void* blk = nullptr;
    TaskPair* d_pairs = nullptr;
    unsigned long long* d_seq = nullptr;
    long long* d_task = nullptr;
    unsigned long long* d_ctr = nullptr;  // head, tail
    int32_t* d_remaining = nullptr;
    uint32_t qcap = 0;
};

long long task_solo(int32_t pi) { return static_cast<long long>(static_cast<uint32_t>(pi)); }
long long task_chunk(int32_t pi, int32_t c) {
    return static_cast<long long>(static_cast<uint32_t>(pi)) | (static_cast<long long>(c + 1) << 32);
}

// Knobs of the many-pair kernel: their own option, else the single-pair one,
// else the default.
int32_t block_rounds_of(const ed_ctx* c) {
    const uint32_t v = c->opt.task_block_rounds ? c->opt.task_block_rounds
                       : c->opt.block_rounds    ? c->opt.block_rounds
                                                : kTaskDefaultBlockRounds;
    return static_cast<int32_t>(v);
}

uint32_t task_solo_rounds(const ed_ctx* c) {
    return c->opt.task_lds_rounds ? c->opt.task_lds_rounds
           : c->opt.lds_rounds    ? c->opt.lds_rounds
                                  : kTaskDefaultLdsRounds;
}

int32_t chunk_diags_of(const ed_ctx* c) {
    return static_cast<int32_t>(c->opt.chunk_diags ? c->opt.chunk_diags : kChunkDiags);
}

// Host-side twin of the device scheduler: the next super-step of a pair whose
// frontier f_t is in its rows.  Appends the chunk tasks; returns false when no
// round can be taken (rows full, k_max or the round budget reached).
bool schedule_on_host(TaskPair& tp, int32_t pi, int32_t block_rounds, int32_t chunk, int64_t k_max,
                      std::vector<long long>& tasks) {
    const int32_t t = tp.t;
    int64_t H = std::min<int64_t>(block_rounds, static_cast<int64_t>(tp.K) - t);
    H = std::min<int64_t>(H, (kLdsRowLen - chunk) / 2);
    if (k_max >= 0) H = std::min<int64_t>(H, k_max - t);
    H = std::min<int64_t>(H, static_cast<int64_t>(tp.t_limit) - t);
    if (H <= 0) return false;
    const int32_t T = t + static_cast<int32_t>(H);
    const int32_t total = 2 * T + 5;
    const int32_t nch = (total + chunk - 1) / chunk;
    tp.H = static_cast<int32_t>(H);
    tp.T = T;
    tp.chunk = chunk;
    tp.nchunks = nch;
    tp.chunks_left = nch;
    tp.found_t = INT32_MAX;
    for (int32_t c = 0; c < nch; ++c) tasks.push_back(task_chunk(pi, c));
    return true;
}

int tasks_start(ed_ctx* c, const std::vector<TaskPair>& st, const std::vector<long long>& first, uint32_t engine,
                hipStream_t s, TaskRun& run) {
    const uint64_t count = st.size();
    const uint32_t solo = task_solo_rounds(c);
    const int32_t C = chunk_diags_of(c);
    // every task that can be in flight at once: one per pair, plus one
    // super-step of chunks per pair with rows, plus slack for the workgroups
    uint64_t qcap = count + first.size() + 256;
    for (const TaskPair& tp : st)
        if (tp.K > 0) qcap += (2ull * tp.K + 5 + C - 1) / C;
    const size_t pairs_bytes = count * sizeof(TaskPair);
    const size_t head = (pairs_bytes + 255) & ~size_t(255);
    const size_t qbytes = qcap * 16;
    run.blk = c->pool.get(head + qbytes + 256);
    if (!run.blk) {
        set_error("ed_batch: device allocation failed");
        return ED_ENOMEM;
    }
    char* base = static_cast<char*>(run.blk);
    TaskParams tp;
    std::memset(&tp, 0, sizeof tp);
    tp.pairs = reinterpret_cast<TaskPair*>(base);
    tp.qseq = reinterpret_cast<unsigned long long*>(base + head);
    tp.qtask = reinterpret_cast<long long*>(base + head + qcap * 8);
    tp.qhead = reinterpret_cast<unsigned long long*>(base + head + qbytes);
    tp.qtail = tp.qhead + 1;
    tp.remaining = reinterpret_cast<int32_t*>(tp.qhead + 2);
    tp.qcap = static_cast<uint32_t>(qcap);
    tp.count = static_cast<int32_t>(count);
    tp.kmax = -1;  // per pair (TaskPair::kmax)
    tp.engine = static_cast<int32_t>(engine);
    tp.lane_words = static_cast<int32_t>(c->opt.lane_words ? c->opt.lane_words : 2u);
    tp.solo_rounds = static_cast<int32_t>(solo);
    tp.block_rounds = block_rounds_of(c);
    tp.chunk_diags = C;
    tp.h = ctx_hash(c);
    tp.counters = c->d_cnt;
    run.d_pairs = tp.pairs;
    run.pairs_bytes = pairs_bytes;
    // queue image: the first tasks full, every other slot waiting for lap 0
    // (host images kept with the run until it is waited for)
    run.seq.assign(qcap, 0);
    run.task.assign(qcap, 0);
    for (uint64_t q = 0; q < qcap; ++q) run.seq[q] = q;
    for (size_t q = 0; q < first.size(); ++q) {
        run.seq[q] = q + 1;
        run.task[q] = first[q];
    }
    run.ctr[0] = 0ull;
    run.ctr[1] = static_cast<unsigned long long>(first.size());
    run.remaining = 0;
    for (const TaskPair& p : st) run.remaining += p.status == 0 ? 1 : 0;
    int grid = c->opt.grid_blocks ? static_cast<int>(c->opt.grid_blocks) : c->task_grid_max;
    grid = std::max(1, grid);
    hipError_t e = hipMemcpyAsync(tp.pairs, st.data(), pairs_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tp.qseq, run.seq.data(), qcap * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tp.qtask, run.task.data(), qcap * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tp.qhead, run.ctr, 16, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(tp.remaining, &run.remaining, 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_ctl_init(c->d_ctl, c->d_cnt, nullptr, s);
    if (e == hipSuccess && run.remaining > 0) e = launch_tasks(tp, grid, s);
    if (e != hipSuccess) {
        (void)hipStreamSynchronize(s);
        c->pool.put(run.blk);
        run.blk = nullptr;
        set_error("task launch: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    return ED_OK;
}

int tasks_wait(ed_ctx* c, std::vector<TaskPair>& st, hipStream_t s, TaskRun& run) {
    hipError_t e = hipMemcpyAsync(st.data(), run.d_pairs, run.pairs_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    c->pool.put(run.blk);
    run.blk = nullptr;
    if (e != hipSuccess) {
        set_error("task launch: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    return ED_OK;
}

int tasks_run(ed_ctx* c, std::vector<TaskPair>& st, const std::vector<long long>& first, uint32_t engine,
              hipStream_t s) {
    TaskRun run;
    int rc = tasks_start(c, st, first, engine, s, run);
    if (rc != ED_OK) return rc;
    return tasks_wait(c, st, s, run);
}

int batch_locked(ed_ctx* c, ed_pair* const* pairs, uint64_t count, int64_t k_max, uint64_t* k_out,
                 int32_t* status_out, hipStream_t s) {
    if (count == 0) return ED_OK;
    const uint32_t engine = pairs[0]->engine;
    for (uint64_t i = 0; i < count; ++i) {
        if (!pairs[i] || pairs[i]->ctx != c) {
            set_error("ed_batch: pair %llu is NULL or from another context", (unsigned long long)i);
            return ED_EINVAL;
        }
        if (pairs[i]->engine != engine || (engine == ED_ENGINE_HASH && pairs[i]->r != pairs[0]->r)) {
            set_error("ed_batch: all pairs must use the same engine (and hash base)");
            return ED_EINVAL;
        }
    }
    if (count > static_cast<uint64_t>(INT32_MAX)) return ED_EINVAL;
    if (engine == ED_ENGINE_HASH && pairs[0]->r != c->r) {
        int rc = ctx_set_hash(c, pairs[0]->r);
        if (rc != ED_OK) return rc;
    }
    const uint32_t solo = task_solo_rounds(c);

    // processing order: largest pairs first (longest-processing-time first), or
    // a seeded permutation when testing order independence
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto size_of = [&](int32_t i) { return std::max(pairs[i]->len[0], pairs[i]->len[1]); };
    if (c->opt.flags & ED_FLAG_SHUFFLE) {
        std::vector<uint64_t> key(count);
        for (uint64_t i = 0; i < count; ++i) key[i] = mix64(c->opt.hash_seed * 0x9E3779B97F4A7C15ull + i);
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    } else {
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return size_of(a) > size_of(b); });
    }

    // rows for the pairs that can outgrow a whole-pair task, from one block
    std::vector<TaskPair> st(count);
    std::vector<int64_t> K(count, 0);
    size_t row_ints = 0;
    for (uint64_t i = 0; i < count; ++i) {
        const int64_t maxnm = static_cast<int64_t>(std::max(pairs[i]->len[0], pairs[i]->len[1]));
        K[i] = batch_row_capacity(maxnm, k_max, solo);
        if (K[i] > 0) row_ints += 2 * static_cast<size_t>(2 * K[i] + 5);
    }
    void* rows_blk = row_ints ? c->pool.get(row_ints * 4) : nullptr;
    if (row_ints && !rows_blk) {
        set_error("ed_batch: device allocation failed");
        return ED_ENOMEM;
    }
    int32_t* rows = static_cast<int32_t*>(rows_blk);
    size_t off = 0;
    for (uint64_t i = 0; i < count; ++i) {
        TaskPair& tp = st[i];
        std::memset(&tp, 0, sizeof tp);
        tp.p = pair_dev(pairs[i]);
        tp.K = static_cast<int32_t>(K[i]);
        if (K[i] > 0) {
            tp.f0 = rows + off;
            off += 2 * K[i] + 5;
            tp.f1 = rows + off;
            off += 2 * K[i] + 5;
        }
        tp.t_limit = INT32_MAX;
        tp.found_t = INT32_MAX;
        tp.kmax = k_max >= 0 ? static_cast<int32_t>(std::min<int64_t>(k_max, INT32_MAX - 1)) : -1;
    }
    std::vector<long long> tasks0;
    tasks0.reserve(count);
    for (int32_t pi : order) tasks0.push_back(task_solo(pi));
    int rc = tasks_run(c, st, tasks0, engine, s);
    c->pool.put(rows_blk);
    if (rc != ED_OK) return rc;
    int first = ED_OK;
    for (uint64_t i = 0; i < count; ++i) {
        int status = ED_OK;
        uint64_t k = 0;
        if (st[i].status == 1 || st[i].status == 2) {
            k = static_cast<uint64_t>(st[i].result);
            pairs[i]->rounds = k;
        } else if (st[i].status == 3) {
            // rows too small for this pair: finish it on the single-pair path
            status = distance_locked(c, pairs[i], k_max, &k, nullptr, 0, s);
        } else {
            if (first == ED_OK)
                set_error("ed_batch: pair %llu ended with status %d", (unsigned long long)i, st[i].status);
            status = ED_EINTERNAL;
        }
        if (k_out) k_out[i] = k;
        if (status_out) status_out[i] = status;
        if (status != ED_OK && first == ED_OK) first = status;
    }
    return first;
}

}  // namespace ed

int ed_batch(ed_ctx* c, ed_pair* const* pairs, uint64_t count, int64_t k_max, uint64_t* k_out,
             int32_t* status_out, void* hip_stream) {
    if (!c || (count && !pairs)) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return ED_EDEVICE;
    return batch_locked(c, pairs, count, k_max, k_out, status_out, static_cast<hipStream_t>(hip_stream));
}

// ---------------------------------------------------------------------------
// Autotuner of the many-pair kernel: coordinate descent over its three knobs,
// timing whole batches; every configuration must give the same distances.
// ---------------------------------------------------------------------------
int ed_autotune_batch(ed_ctx* c, ed_pair* const* pairs, uint64_t count, int64_t k_max, uint32_t passes,
                      ed_tune_result* out, void* hip_stream) {
    if (!c || (count && !pairs) || !out) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return ED_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    if (passes == 0) passes = 2;
    std::memset(out, 0, sizeof *out);
    const ed_options start = c->opt;
    std::vector<uint64_t> want(count), got(count);
    std::vector<int32_t> st(count);
    uint32_t evaluated = 0;

    // one timed batch with the current options; compares with `want` once set
    auto run = [&](bool reference, double* ms) -> int {
        const auto t0 = std::chrono::steady_clock::now();
        int rc = batch_locked(c, pairs, count, k_max, reference ? want.data() : got.data(), st.data(), s);
        const auto t1 = std::chrono::steady_clock::now();
        if (rc != ED_OK) return rc;
        *ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        ++evaluated;
        if (!reference) {
            for (uint64_t i = 0; i < count; ++i)
                if (got[i] != want[i]) {
                    set_error("ed_autotune_batch: pair %llu gave %llu under chunk_diags=%u "
                              "task_lds_rounds=%u task_block_rounds=%u, %llu before",
                              (unsigned long long)i, (unsigned long long)got[i], c->opt.chunk_diags,
                              c->opt.task_lds_rounds, c->opt.task_block_rounds,
                              (unsigned long long)want[i]);
                    return ED_EINTERNAL;
                }
        }
        return ED_OK;
    };

    // the starting configuration, with its knobs made explicit
    ed_options start_x = start;
    start_x.chunk_diags = static_cast<uint32_t>(chunk_diags_of(c));
    start_x.task_lds_rounds = task_solo_rounds(c);
    start_x.task_block_rounds = static_cast<uint32_t>(block_rounds_of(c));
    ed_options best = start_x;
    double warm = 0, default_ms = 0;
    c->opt = best;
    int rc = run(true, &warm);  // warm-up and reference distances
    if (rc == ED_OK) rc = run(false, &default_ms);
    if (rc != ED_OK) {
        c->opt = start;
        return rc;
    }
    double best_ms = default_ms;
    static const uint32_t kLds[] = {64, 128, 256, 512, 1024, 2048, 4096};
    static const uint32_t kBlock[] = {8, 16, 32, 64, 128, 256};
    static const uint32_t kChunk[] = {512, 1024, 1536, 1792, 2048, 4096, 6144};
    for (uint32_t pass = 0; pass < passes; ++pass) {
        bool moved = false;
        for (int knob = 0; knob < 3; ++knob) {
            const uint32_t* vals = knob == 0 ? kLds : knob == 1 ? kBlock : kChunk;
            const int nv = knob == 0 ? 7 : knob == 1 ? 6 : 7;
            for (int v = 0; v < nv; ++v) {
                ed_options cand = best;
                uint32_t& field = knob == 0 ? cand.task_lds_rounds
                                  : knob == 1 ? cand.task_block_rounds
                                              : cand.chunk_diags;
                if (field == vals[v]) continue;
                field = vals[v];
                // a chunk and its halo must fit one LDS row
                if (cand.chunk_diags + 2 * std::min<uint32_t>(cand.task_block_rounds, 4096) >
                    static_cast<uint32_t>(kLdsRowLen))
                    continue;
                c->opt = cand;
                double ms = 0;
                rc = run(false, &ms);
                if (rc != ED_OK) {
                    c->opt = start;
                    return rc;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                    moved = true;
                }
            }
        }
        if (!moved) break;
    }
    // re-time the winner and the start: the winner is kept only if it is
    // still faster (a lucky single timing is not kept)
    if (best_ms < default_ms) {
        double again = 0, again0 = 0;
        c->opt = best;
        rc = run(false, &again);
        if (rc == ED_OK) {
            c->opt = start_x;
            rc = run(false, &again0);
        }
        if (rc != ED_OK) {
            c->opt = start;
            return rc;
        }
        const double tb = std::min(again, best_ms), t0 = std::min(again0, default_ms);
        if (tb >= t0) {
            best = start_x;
            best_ms = t0;
        } else {
            best_ms = tb;
        }
        default_ms = t0;
    }
    c->opt = best;
    out->best = best;
    out->default_ms = default_ms;
    out->best_ms = best_ms;
    out->evaluated = evaluated;
    return ED_OK;
}
