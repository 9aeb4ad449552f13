// ed_batch: many prepared pairs in one persistent launch.
#include <algorithm>
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

int batch_locked(ed_ctx* c, ed_pair* const* pairs, uint64_t count, int64_t k_max, uint64_t* k_out,
                 int32_t* status_out, hipStream_t s) {
    if (count == 0) return ED_OK;
    const uint32_t engine = pairs[0]->engine;
    for (uint64_t i = 0; i < count; ++i) {
        if (!pairs[i] || pairs[i]->ctx != c) {
            set_error("ed_batch: pair %llu is NULL or from another context", (unsigned long long)i);
            return ED_EINVAL;
        }
        if (pairs[i]->engine != engine) {
            set_error("ed_batch: all pairs must use the same engine");
            return ED_EINVAL;
        }
    }
    if (count > static_cast<uint64_t>(INT32_MAX)) return ED_EINVAL;
    if (engine == ED_ENGINE_HASH && pairs[0]->seed != c->opt.hash_seed) {
        int rc = ctx_set_hash(c, pairs[0]->seed);
        if (rc != ED_OK) return rc;
    }
    const uint32_t lds_rounds = c->opt.lds_rounds ? c->opt.lds_rounds : kDefaultLdsRounds;
    const uint32_t lane_words = c->opt.lane_words ? c->opt.lane_words : (engine == ED_ENGINE_HASH ? 1u : 2u);

    // order: largest pairs first (longest-processing-time first), or a
    // seeded permutation when testing order independence
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto size_of = [&](int32_t i) {
        return std::max(pairs[i]->len[0], pairs[i]->len[1]);
    };
    if (c->opt.flags & ED_FLAG_SHUFFLE) {
        std::vector<uint64_t> key(count);
        for (uint64_t i = 0; i < count; ++i) key[i] = mix64(c->opt.hash_seed * 0x9E3779B97F4A7C15ull + i);
        std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return key[a] < key[b]; });
    } else {
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return size_of(a) > size_of(b); });
    }

    // rows for pairs that outgrow the LDS rounds, carved out of one block
    std::vector<int64_t> K(count, 0);
    size_t row_ints = 0;
    for (uint64_t i = 0; i < count; ++i) {
        const int64_t maxnm = static_cast<int64_t>(std::max(pairs[i]->len[0], pairs[i]->len[1]));
        K[i] = batch_row_capacity(maxnm, k_max, lds_rounds);
        if (K[i] > 0) row_ints += 2 * static_cast<size_t>(2 * K[i] + 5);
    }
    const size_t items_bytes = count * sizeof(BatchItem);
    const size_t order_bytes = count * 4;
    const size_t kout_bytes = count * 4;
    const size_t head = (items_bytes + order_bytes + kout_bytes + 64 + 255) & ~size_t(255);
    void* blk = c->pool.get(head + row_ints * 4 + 4);
    if (!blk) {
        set_error("ed_batch: device allocation failed");
        return ED_ENOMEM;
    }
    char* base = static_cast<char*>(blk);
    BatchItem* d_items = reinterpret_cast<BatchItem*>(base);
    int32_t* d_order = reinterpret_cast<int32_t*>(base + items_bytes);
    int32_t* d_kout = reinterpret_cast<int32_t*>(base + items_bytes + order_bytes);
    unsigned int* d_ticket = reinterpret_cast<unsigned int*>(base + items_bytes + order_bytes + kout_bytes);
    int32_t* rows = reinterpret_cast<int32_t*>(base + head);

    std::vector<BatchItem> items(count);
    size_t off = 0;
    for (uint64_t i = 0; i < count; ++i) {
        std::memset(&items[i], 0, sizeof(BatchItem));
        items[i].p = pair_dev(pairs[i]);
        items[i].K = static_cast<int32_t>(K[i]);
        if (K[i] > 0) {
            items[i].f0 = rows + off;
            off += 2 * K[i] + 5;
            items[i].f1 = rows + off;
            off += 2 * K[i] + 5;
        }
    }
    BatchParams bp;
    std::memset(&bp, 0, sizeof bp);
    bp.items = d_items;
    bp.order = d_order;
    bp.count = static_cast<int32_t>(count);
    bp.kmax = k_max >= 0 ? static_cast<int32_t>(std::min<int64_t>(k_max, INT32_MAX - 1)) : -1;
    bp.engine = static_cast<int32_t>(engine);
    bp.lane_words = static_cast<int32_t>(lane_words);
    bp.lds_rounds = static_cast<int32_t>(lds_rounds);
    bp.h = ctx_hash(c);
    bp.ticket = d_ticket;
    bp.k_out = d_kout;
    bp.counters = c->d_cnt;
    std::vector<int32_t> kres(count, -1);
    int grid = c->opt.grid_blocks ? static_cast<int>(c->opt.grid_blocks) : c->frontier_grid_max;
    grid = std::max(1, std::min<int>(grid, static_cast<int>(std::min<uint64_t>(count, INT32_MAX))));
    hipError_t e = hipMemcpyAsync(d_items, items.data(), items_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), order_bytes, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_fill_u32(d_ticket, 1, 0u, s);
    if (e == hipSuccess) e = launch_ctl_init(c->d_ctl, c->d_cnt, nullptr, s);
    if (e == hipSuccess) e = launch_batch(bp, grid, s);
    if (e == hipSuccess) e = hipMemcpyAsync(kres.data(), d_kout, kout_bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    c->pool.put(blk);
    if (e != hipSuccess) {
        set_error("ed_batch: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    int first = ED_OK;
    for (uint64_t i = 0; i < count; ++i) {
        int st = ED_OK;
        uint64_t k = 0;
        if (kres[i] >= 0) {
            k = static_cast<uint64_t>(kres[i]);
            pairs[i]->rounds = k;
        } else {
            // rows too small for this pair: finish it on the single-pair path
            st = distance_locked(c, pairs[i], k_max, &k, nullptr, 0, s);
        }
        if (k_out) k_out[i] = k;
        if (status_out) status_out[i] = st;
        if (st != ED_OK && first == ED_OK) first = st;
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
