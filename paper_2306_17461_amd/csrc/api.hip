// Host side of libed.so: the C ABI declared in include/ed.h.
#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/ed.h"
#include "internal.h"
#include "host.h"

using namespace ed;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

void ed::set_error(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

#define HIP_TRY(expr)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ed::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                          __LINE__);                                                     \
            return ED_EDEVICE;                                                           \
        }                                                                                \
    } while (0)

// ---------------------------------------------------------------------------
// host-side arithmetic mod 2^61-1 (powers of the base for the kernels)
// ---------------------------------------------------------------------------
static uint64_t hmul(uint64_t a, uint64_t b) {
    unsigned __int128 p = static_cast<unsigned __int128>(a) * b;
    uint64_t lo = static_cast<uint64_t>(p) & kP;
    uint64_t hi = static_cast<uint64_t>(p >> 61);
    uint64_t s = lo + hi;
    s = (s & kP) + (s >> 61);
    return s >= kP ? s - kP : s;
}

static uint64_t hadd(uint64_t a, uint64_t b) {
    const uint64_t s = a + b;
    return s >= kP ? s - kP : s;
}

static uint64_t hsub(uint64_t a, uint64_t b) { return a >= b ? a - b : a + kP - b; }
static uint64_t hpow(uint64_t r, uint64_t e) {
    uint64_t acc = 1, b = r;
    while (e) {
        if (e & 1) acc = hmul(acc, b);
        b = hmul(b, b);
        e >>= 1;
    }
    return acc;
}

uint64_t ed_hash_base(uint64_t seed) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const uint64_t span = kP - (1ull << 21);
    return (1ull << 20) + z % span;
}

// ---------------------------------------------------------------------------
// device memory pool: freed blocks are kept per rounded size and reused
// ---------------------------------------------------------------------------
static size_t round_size(size_t n) {
    if (n < 4096) return 4096;
    // 1/8-octave classes above 4 KiB
    size_t p = 4096;
    while (p < n) p <<= 1;
    const size_t step = p >> 3;
    size_t r = (p >> 1);
    while (r < n) r += step;
    return r;
}

void* DevPool::get(size_t bytes) {
    const size_t sz = round_size(bytes);
    auto it = free_.find(sz);
    if (it != free_.end() && !it->second.empty()) {
        void* p = it->second.back();
        it->second.pop_back();
        cached_ -= sz;
        live_[p] = sz;
        return p;
    }
    void* p = nullptr;
    if (hipMalloc(&p, sz) != hipSuccess) {
        (void)hipGetLastError();
        trim();
        if (hipMalloc(&p, sz) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
    }
    live_[p] = sz;
    return p;
}

void DevPool::put(void* p) {
    if (!p) return;
    auto it = live_.find(p);
    if (it == live_.end()) return;
    free_[it->second].push_back(p);
    cached_ += it->second;
    live_.erase(it);
}

void DevPool::trim() {
    for (auto& kv : free_)
        for (void* p : kv.second) (void)hipFree(p);
    free_.clear();
    cached_ = 0;
}

DevPool::~DevPool() {
    trim();
    for (auto& kv : live_) (void)hipFree(kv.first);
}

// ---------------------------------------------------------------------------
// context
// ---------------------------------------------------------------------------
void ed_default_options(ed_options* o) {
    std::memset(o, 0, sizeof *o);
    o->engine = ED_ENGINE_DIRECT;
    o->pack_bits = 0;
    o->block = 32;
    o->flags = 0;
    o->hash_seed = 0x5EED;
}

static int check_options(const ed_options* o) {
    if (o->engine > 1) return ED_EINVAL;
    if (o->pack_bits != 0 && o->pack_bits != 2 && o->pack_bits != 8) return ED_EINVAL;
    const uint32_t b = o->block ? o->block : 32;
    if (b > 4096 || (b & (b - 1)) != 0) return ED_EINVAL;
    if (o->lds_rounds > static_cast<uint32_t>(kLdsRoundsMax)) return ED_EINVAL;
    if (o->lane_words > 64) return ED_EINVAL;
    if (o->grid_blocks > static_cast<uint32_t>(kMaxGrid)) return ED_EINVAL;
    if (o->block_rounds > 4096) return ED_EINVAL;
    if (o->chunk_diags != 0 && (o->chunk_diags < 64 || o->chunk_diags > 8000)) return ED_EINVAL;
    if (o->task_lds_rounds > static_cast<uint32_t>(kLdsRoundsMax)) return ED_EINVAL;
    if (o->task_block_rounds > 4096) return ED_EINVAL;
    return ED_OK;
}

uint64_t ed::opt_base(const ed_options& o) {
    return (o.flags & ED_FLAG_WEAK_HASH) ? 1 : ed_hash_base(o.hash_seed);
}

int ed::ctx_set_hash(ed_ctx* c, uint64_t r) {
    if (c->d_pow && r == c->r) return ED_OK;
    std::vector<uint64_t> h(kPowEntries);
    // pow0 | pow1 | rtab
    uint64_t* p0 = h.data();
    uint64_t* p1 = p0 + 65536;
    uint64_t* rt = p1 + 65536;
    p0[0] = 1;
    for (int i = 1; i < 65536; ++i) p0[i] = hmul(p0[i - 1], r);
    const uint64_t r16 = hmul(p0[65535], r);
    p1[0] = 1;
    for (int i = 1; i < 65536; ++i) p1[i] = hmul(p1[i - 1], r16);
    for (int i = 0; i < 65; ++i) rt[i] = p0[i];
    for (int k = 0; k < 257; ++k) rt[kRtabRseg + k] = hpow(r, 64ull * k);
    const uint64_t R = hpow(r, kTileChars);
    uint64_t a = 1;
    for (int d = 0; d < 65; ++d) {
        rt[kRtabR + d] = a;
        a = hmul(a, R);
    }
    for (int k = 0; k < 8; ++k)
        for (int v = 0; v < 256; ++v) {
            uint64_t h = 0;
            for (int j = 0; j < 4; ++j) h = hadd(h, hmul(static_cast<uint64_t>((v >> (2 * j)) & 3), p0[31 - 4 * k - j]));
            rt[kRtabLut32 + 256 * k + v] = h;
            rt[kRtabLut8 + 256 * k + v] = hmul(static_cast<uint64_t>(v), p0[7 - k]);
        }
    // inverse powers: r^(P-2) = r^-1 (P prime, r not 0)
    const uint64_t rinv256 = hpow(hpow(r, kP - 2), 256);
    a = 1;
    for (int d = 0; d < 65; ++d) {
        rt[kRtabRinv256 + d] = a;
        a = hmul(a, rinv256);
    }
    a = hpow(R, 8);
    for (int j = 0; j < 10; ++j) {
        rt[kRtabR8pow2 + j] = a;
        a = hmul(a, a);
    }
    for (int l = 0; l < 64; ++l) rt[kRtabR8lane + l] = hpow(R, 8ull * (l + 1));
    for (int d = 0; d < 64; ++d) rt[kRtabRChunk + d] = hpow(R, 2048ull * d);
    a = 1;
    for (int j = 0; j < kScanChunkTiles; ++j) {
        rt[kRtabRTile + j] = a;
        a = hmul(a, R);
    }
    const uint64_t rinv = hpow(r, kP - 2);
    a = 1;
    for (int d = 0; d < 33; ++d) {
        rt[kRtabRinv32 + d] = a;
        a = hmul(a, rinv);
    }
    // Block hashes of 8-bit strings as int8 matrix products (prepare.hip):
    // each weight r^(31 - j) written exactly as 8 signed base-256 digits in
    // [-128, 127]; lane l = 16 g + i holds in byte e of its A operand digit
    // t = i mod 8 of the weight of character 16 (g mod 2) + e of a block when
    // g / 2 = i / 8 (the half of the 64 characters that row i sums), else
    // zero.  The characters enter as c - 128 and each product row with 2^19
    // added; the constant undoes both: 128 sum_j r^(31 - j) minus
    // 2^19 sum_t 256^t.
    auto digits = [](uint64_t w, int t) {
        int64_t v = static_cast<int64_t>(w);
        for (int u = 0;; ++u) {
            int64_t dg = v & 0xFF;
            if (dg >= 128) dg -= 256;
            if (u == t) return static_cast<int8_t>(dg);
            v = (v - dg) >> 8;
        }
    };
    int8_t* mA = reinterpret_cast<int8_t*>(rt + kRtabMmaA);
    for (int l = 0; l < 64; ++l) {
        const int i = l % 16, g = l / 16;
        for (int e = 0; e < 16; ++e) mA[16 * l + e] = (g / 2 == i / 8) ? digits(p0[31 - 16 * (g % 2) - e], i % 8) : 0;
    }
    uint64_t wblk = 0, geo = 0;
    for (int j = 0; j < 32; ++j) wblk = hadd(wblk, p0[j]);
    for (int t = 0; t < 8; ++t) geo = hadd(geo, 1ull << (8 * t));
    rt[kRtabMmaK] = hsub(hmul(128, wblk), hmul(1ull << 19, geo));
    if (!c->d_pow) {
        HIP_TRY(hipMalloc(&c->d_pow, kPowEntries * sizeof(uint64_t)));
    } else {
        // pack and table kernels of an earlier ed_prepare may still read the
        // old tables on a caller's stream (one that does not wait for the
        // null stream); the copy below must not overtake them
        HIP_TRY(hipDeviceSynchronize());
    }
    HIP_TRY(hipMemcpy(c->d_pow, h.data(), kPowEntries * sizeof(uint64_t), hipMemcpyHostToDevice));
    c->r = r;
    return ED_OK;
}

int ed_init(ed_ctx** out, int device, const ed_options* opt) {
    if (!out) return ED_EINVAL;
    *out = nullptr;
    ed_options o;
    if (opt)
        o = *opt;
    else
        ed_default_options(&o);
    if (check_options(&o) != ED_OK) {
        set_error("ed_init: invalid options");
        return ED_EINVAL;
    }
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) {
        set_error("ed_init: device %d out of range (%d devices)", device, ndev);
        return ED_EINVAL;
    }
    HIP_TRY(hipSetDevice(device));
    ed_ctx* c = new (std::nothrow) ed_ctx();
    if (!c) return ED_ENOMEM;
    c->device = device;
    c->opt = o;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        set_error("hipGetDeviceProperties failed");
        return ED_EDEVICE;
    }
    c->num_cu = prop.multiProcessorCount;
    int fg = 0;
    if (frontier_max_grid(device, &fg) != hipSuccess || fg < 1) fg = c->num_cu;
    c->frontier_grid_max = fg;
    int tg = 0;
    if (task_max_grid(device, &tg) != hipSuccess || tg < 1) tg = c->num_cu;
    c->task_grid_max = tg;
    if (hipMalloc(&c->d_ctl, sizeof(FrontierCtl)) != hipSuccess ||
        hipMalloc(&c->d_cnt, sizeof(CountersDev) * (kMaxGrid + 1)) != hipSuccess ||
        hipHostMalloc(&c->h_ctl, sizeof(FrontierCtl)) != hipSuccess ||
        hipHostMalloc(&c->h_cnt, sizeof(CountersDev)) != hipSuccess ||
        hipMalloc(&c->d_bar, static_cast<size_t>(kMaxGrid) * kBarStride * 4) != hipSuccess ||
        hipMalloc(&c->d_gpart, static_cast<size_t>(2) * kGridJobs * kMaxGrid * 4) != hipSuccess) {
        set_error("ed_init: allocation failed");
        ed_shutdown(c);
        return ED_ENOMEM;
    }
    if (hipEventCreate(&c->ev[0]) != hipSuccess || hipEventCreate(&c->ev[1]) != hipSuccess) {
        set_error("ed_init: hipEventCreate failed");
        ed_shutdown(c);
        return ED_EDEVICE;
    }
    int rc = ctx_set_hash(c, opt_base(o));
    if (rc == ED_OK) rc = scratch_setup(c);
    if (rc != ED_OK) {
        ed_shutdown(c);
        return rc;
    }
    *out = c;
    return ED_OK;
}

int ed_set_options(ed_ctx* c, const ed_options* opt) {
    if (!c || !opt) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    if (check_options(opt) != ED_OK) {
        set_error("ed_set_options: invalid options");
        return ED_EINVAL;
    }
    HIP_TRY(hipSetDevice(c->device));
    int rc = ctx_set_hash(c, opt_base(*opt));
    if (rc != ED_OK) return rc;
    c->opt = *opt;
    return ED_OK;
}

int ed_get_options(ed_ctx* c, ed_options* opt) {
    if (!c || !opt) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    *opt = c->opt;
    return ED_OK;
}

int ed_shutdown(ed_ctx* c) {
    if (!c) return ED_EINVAL;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->d_pow) (void)hipFree(c->d_pow);
    if (c->d_ctl) (void)hipFree(c->d_ctl);
    if (c->d_cnt) (void)hipFree(c->d_cnt);
    if (c->d_bar) (void)hipFree(c->d_bar);
    if (c->d_gpart) (void)hipFree(c->d_gpart);
    if (c->h_ctl) (void)hipHostFree(c->h_ctl);
    if (c->h_cnt) (void)hipHostFree(c->h_cnt);
    for (hipEvent_t& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return ED_OK;
}

// ---------------------------------------------------------------------------
// pairs
// ---------------------------------------------------------------------------
static int log2u(uint32_t b) {
    int l = 0;
    while ((1u << l) < b) ++l;
    return l;
}

void ed::pair_free(ed_pair* p) {
    DevPool& pool = p->ctx->pool;
    for (hipEvent_t& e : p->ev_prep)
        if (e) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    if (p->ev_done) {
        (void)hipEventDestroy(p->ev_done);
        p->ev_done = nullptr;
    }
    for (void** q : {&p->w2[0], &p->w2[1], &p->w4[0], &p->w4[1], &p->w8[0], &p->w8[1], &p->tab_blk[0], &p->tab_blk[1], &p->misc,
                     &p->stage[0], &p->stage[1], &p->f0, &p->f1}) {
        pool.put(*q);
        *q = nullptr;
    }
    p->tab[0] = p->tab[1] = nullptr;
}

PairDev ed::pair_dev(const ed_pair* p) {
    PairDev d;
    std::memset(&d, 0, sizeof d);
    d.a.w2 = static_cast<const uint64_t*>(p->w2[0]);
    d.b.w2 = static_cast<const uint64_t*>(p->w2[1]);
    d.a.w4 = static_cast<const uint64_t*>(p->w4[0]);
    d.b.w4 = static_cast<const uint64_t*>(p->w4[1]);
    d.a.w8 = static_cast<const uint64_t*>(p->w8[0]);
    d.b.w8 = static_cast<const uint64_t*>(p->w8[1]);
    d.a.tab = static_cast<const uint64_t*>(p->tab[0]);
    d.b.tab = static_cast<const uint64_t*>(p->tab[1]);
    d.a.len = static_cast<int32_t>(p->len[0]);
    d.b.len = static_cast<int32_t>(p->len[1]);
    d.alpha = reinterpret_cast<const uint32_t*>(static_cast<char*>(p->misc) + kMiscAlpha);
    d.log2b = p->log2b;
    d.force8 = p->force8;
    return d;
}

HashDev ed::ctx_hash(const ed_ctx* c) {
    HashDev h;
    h.r = c->r;
    h.pow0 = c->d_pow;
    h.pow1 = c->d_pow + 65536;
    h.rtab = c->d_pow + 2 * 65536;
    return h;
}

int ed::prepare_locked(ed_ctx* c, const uint8_t* A, uint64_t n, const uint8_t* B, uint64_t m,
                       int on_device, hipStream_t s, ed_pair** out) {
    *out = nullptr;
    if ((n && !A) || (m && !B) || n >= ED_MAX_LEN || m >= ED_MAX_LEN) {
        set_error("ed_prepare: invalid string arguments (n=%llu m=%llu)",
                  static_cast<unsigned long long>(n), static_cast<unsigned long long>(m));
        return ED_EINVAL;
    }
    ed_pair* p = new (std::nothrow) ed_pair();
    if (!p) return ED_ENOMEM;
    p->ctx = c;
    p->len[0] = n;
    p->len[1] = m;
    p->engine = c->opt.engine;
    const uint32_t b = c->opt.block ? c->opt.block : 32;
    p->log2b = log2u(b);
    p->force8 = c->opt.pack_bits == 8 ? 1 : 0;
    if (c->opt.engine == ED_ENGINE_HASH) {
        // tables with the base of the current options (a query on an older
        // pair may have left the context on that pair's base)
        const int rc = ctx_set_hash(c, opt_base(c->opt));
        if (rc != ED_OK) {
            delete p;
            return rc;
        }
    }
    p->r = c->r;
    const bool table = p->engine == ED_ENGINE_HASH;
    // 4-bit words for alphabets up to 16 symbols: the direct engine reads any
    // power-of-two width; the hash engine's partial-block hashes take 2 or 8
    const bool nib = !table && c->opt.pack_bits == 0;
    const uint8_t* src[2] = {A, B};
    int32_t tiles[2];
    for (int s2 = 0; s2 < 2; ++s2) {
        const uint64_t len = p->len[s2];
        tiles[s2] = static_cast<int32_t>(std::max<uint64_t>(1, (len + kTileChars - 1) / kTileChars));
        p->w2[s2] = c->pool.get((static_cast<size_t>(tiles[s2]) * kTileWords2 + kPadWords) * 8);
        p->w8[s2] = c->pool.get((static_cast<size_t>(tiles[s2]) * kTileWords8 + kPadWords) * 8);
        if (nib) p->w4[s2] = c->pool.get((static_cast<size_t>(tiles[s2]) * kTileWords4 + kPadWords) * 8);
        if (table) {
            p->tab_blk[s2] = c->pool.get(((len >> p->log2b) + 1) * 8 + kTabShift);
            if (p->tab_blk[s2]) p->tab[s2] = static_cast<char*>(p->tab_blk[s2]) + kTabShift;
        }
        if (!p->w2[s2] || !p->w8[s2] || (nib && !p->w4[s2]) || (table && !p->tab[s2])) {
            pair_free(p);
            delete p;
            set_error("ed_prepare: device allocation failed");
            return ED_ENOMEM;
        }
    }
    const int32_t total = tiles[0] + tiles[1];
    // pack: two workgroups per CU, each taking many chunks (more workgroups
    // measured slower)
    const int stream_grid = std::max(1, std::min(total, c->num_cu * 2));
    // alphabet word | tile hashes | chunk flags | tile prefixes | pack workgroup slots |
    // [lane prefixes | scan chunk hashes]
    const size_t agg_off = kMiscAlpha + 64;
    const size_t big_off = agg_off + static_cast<size_t>(total) * 8;
    const size_t pre_off = big_off + ((static_cast<size_t>(total) * kTileChunks + 7) & ~size_t(7));
    const size_t wor_off = pre_off + static_cast<size_t>(total) * 8;
    const size_t lane_off = wor_off + ((static_cast<size_t>(stream_grid) * 4 + 7) & ~size_t(7));
    const size_t tot_off = lane_off + (table ? static_cast<size_t>(total) * 64 * 8 : 0);
    p->misc = c->pool.get(tot_off + (table ? 2 * 64 * 8 : 0));
    if (!p->misc) {
        pair_free(p);
        delete p;
        return ED_ENOMEM;
    }
    char* misc = static_cast<char*>(p->misc);
    // staging: host inputs, or device inputs not 16-byte aligned
    const uint8_t* raw[2];
    for (int s2 = 0; s2 < 2; ++s2) {
        const uint64_t len = p->len[s2];
        const bool aligned = (reinterpret_cast<uintptr_t>(src[s2]) & 15u) == 0;
        if (len && (!on_device || !aligned)) {
            p->stage[s2] = c->pool.get(len + 16);
            if (!p->stage[s2]) {
                pair_free(p);
                delete p;
                return ED_ENOMEM;
            }
            hipError_t e = hipMemcpyAsync(p->stage[s2], src[s2], len,
                                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s);
            if (e != hipSuccess) {
                set_error("ed_prepare: input copy failed: %s", hipGetErrorString(e));
                pair_free(p);
                delete p;
                return ED_EDEVICE;
            }
            raw[s2] = static_cast<const uint8_t*>(p->stage[s2]);
        } else {
            raw[s2] = src[s2];
        }
    }
    PrepParams pp;
    std::memset(&pp, 0, sizeof pp);
    for (int s2 = 0; s2 < 2; ++s2) {
        pp.s[s2].raw = raw[s2];
        pp.s[s2].w2 = static_cast<uint64_t*>(p->w2[s2]);
        pp.s[s2].w4 = static_cast<uint64_t*>(p->w4[s2]);
        pp.s[s2].w8 = static_cast<uint64_t*>(p->w8[s2]);
        pp.s[s2].tab = static_cast<uint64_t*>(p->tab[s2]);
        pp.s[s2].len = static_cast<int32_t>(p->len[s2]);
        pp.s[s2].tiles = tiles[s2];
    }
    pp.s[0].tile0 = 0;
    pp.s[1].tile0 = tiles[0];
    pp.total_tiles = total;
    pp.log2b = p->log2b;
    pp.force8 = p->force8;
    pp.nt_copy = p->len[0] + p->len[1] > kNtCopyBytes ? 1 : 0;
    pp.build_table = table ? 1 : 0;
    pp.fuse_table = table && p->log2b == 5 ? 1 : 0;
    pp.r = c->r;
    pp.tile_agg = reinterpret_cast<uint64_t*>(misc + agg_off);
    pp.tile_prefix = reinterpret_cast<uint64_t*>(misc + pre_off);
    pp.lane_excl = table ? reinterpret_cast<uint64_t*>(misc + lane_off) : nullptr;
    pp.chunk_tot = table ? reinterpret_cast<uint64_t*>(misc + tot_off) : nullptr;
    pp.alpha = reinterpret_cast<uint32_t*>(misc + kMiscAlpha);
    pp.packed_any = reinterpret_cast<uint32_t*>(misc + kMiscAlpha + 4);
    pp.chunk_big = reinterpret_cast<uint8_t*>(misc + big_off);
    pp.wg_or = reinterpret_cast<uint32_t*>(misc + wor_off);
    pp.pack_grid = stream_grid;
    pp.scan_chunks = (tiles[0] + kScanChunkTiles - 1) / kScanChunkTiles + (tiles[1] + kScanChunkTiles - 1) / kScanChunkTiles;
    pp.rtab = c->d_pow + 2 * 65536;
    // table passes: as many workgroups as fit by LDS (at most one tile per wavefront)
    const int table_grid = c->num_cu * 4;
    if (c->opt.flags & ED_FLAG_TIMING) {
        HIP_TRY(hipEventCreate(&p->ev_prep[0]));
        HIP_TRY(hipEventCreate(&p->ev_prep[1]));
        if (table) HIP_TRY(hipEventCreate(&p->ev_prep[2]));
        HIP_TRY(hipEventRecord(p->ev_prep[0], s));
        p->prep_timed = true;
    }
    HIP_TRY(launch_pack(pp, stream_grid, s));
    if (table && p->prep_timed) HIP_TRY(hipEventRecord(p->ev_prep[2], s));
    // the rest pass usually has nothing to do (a packable pair): a small grid
    // keeps that cheap
    HIP_TRY(launch_after_pack(pp, std::max(1, std::min(total, c->num_cu)), s));
    if (table) HIP_TRY(launch_table(pp, table_grid, s));
    if (p->prep_timed) HIP_TRY(hipEventRecord(p->ev_prep[1], s));
    p->launches_prepare = 2 + (table ? (pp.fuse_table ? 2 : 4) : 0);
    if (c->opt.pack_bits == 2) {
        uint32_t alpha = 0;
        HIP_TRY(hipMemcpyAsync(&alpha, pp.alpha, 4, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (alpha > 3u) {
            pair_free(p);
            delete p;
            set_error("ed_prepare: pack_bits=2 but a character is above 3 (OR of characters = %u)", alpha);
            return ED_EINVAL;
        }
    }
    // (without the event, ed_release waits for the whole device instead)
    if (hipEventCreateWithFlags(&p->ev_done, hipEventDisableTiming) != hipSuccess) p->ev_done = nullptr;
    if (p->ev_done && hipEventRecord(p->ev_done, s) != hipSuccess) {
        (void)hipEventDestroy(p->ev_done);
        p->ev_done = nullptr;
    }
    *out = p;
    return ED_OK;
}

int ed_prepare(ed_ctx* c, const uint8_t* A, uint64_t n, const uint8_t* B, uint64_t m,
               int inputs_on_device, void* hip_stream, ed_pair** out) {
    if (!c || !out) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    int rc = prepare_locked(c, A, n, B, m, inputs_on_device, static_cast<hipStream_t>(hip_stream), out);
    if (rc == ED_OK)
        (*out)->ns_prepare =
            std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int ed_release(ed_pair* p) {
    if (!p) return ED_EINVAL;
    ed_ctx* c = p->ctx;
    std::lock_guard<std::mutex> lk(c->mu);
    (void)hipSetDevice(c->device);
    // the prepare's kernels may still be queued on the caller's stream; every
    // other call on a pair returns after its work
    if (p->ev_done)
        (void)hipEventSynchronize(p->ev_done);
    else
        (void)hipDeviceSynchronize();
    pair_free(p);
    delete p;
    return ED_OK;
}

// ---------------------------------------------------------------------------
// distance
// ---------------------------------------------------------------------------
static int frontier_grid(const ed_ctx* c) {
    int g = c->opt.grid_blocks ? static_cast<int>(c->opt.grid_blocks) : c->num_cu;
    return std::max(1, std::min(g, c->frontier_grid_max));
}

int ed::frontier_setup(ed_ctx* c, ed_pair* p, FrontierParams& fp) {
    if (p->engine == ED_ENGINE_HASH && (!p->tab[0] || !p->tab[1])) {
        set_error("ed_distance: pair has no prefix tables");
        return ED_EINVAL;
    }
    if (p->engine == ED_ENGINE_HASH && p->r != c->r) {
        int rc = ctx_set_hash(c, p->r);
        if (rc != ED_OK) return rc;
    }
    const uint32_t lds_rounds = c->opt.lds_rounds ? c->opt.lds_rounds : kDefaultLdsRounds;
    const uint32_t lane_words = c->opt.lane_words ? c->opt.lane_words
                                                  : (p->engine == ED_ENGINE_HASH ? 1u : 2u);
    std::memset(&fp, 0, sizeof fp);
    fp.p = pair_dev(p);
    fp.h = ctx_hash(c);
    fp.kmax = -1;
    fp.lds_rounds = (c->opt.flags & ED_FLAG_NO_PHASE_A) ? 0 : static_cast<int32_t>(lds_rounds);
    fp.engine = static_cast<int32_t>(p->engine);
    fp.lane_words = static_cast<int32_t>(lane_words);
    fp.block_rounds = static_cast<int32_t>(c->opt.block_rounds ? c->opt.block_rounds : kDefaultBlockRounds);
    fp.wait_ticks = kWaitTicks;
    fp.grid_rounds = (p->engine == ED_ENGINE_DIRECT && !(c->opt.flags & ED_FLAG_NO_GRID_ROUNDS)) ? 1 : 0;
    fp.gpart = c->d_gpart;
    fp.hash_first = (p->engine == ED_ENGINE_HASH && (c->opt.flags & ED_FLAG_HASH_FIRST)) ? 1 : 0;
    fp.ctl = c->d_ctl;
    fp.bar = c->d_bar;
    fp.counters = c->d_cnt;
    return ED_OK;
}

void ed::counters_add(CountersDev& a, const CountersDev& b) {
    a.updates += b.updates;
    a.lcp_chars += b.lcp_chars;
    a.wave_lcps += b.wave_lcps;
    a.grid_lcps += b.grid_lcps;
    a.wg_lcps += b.wg_lcps;
    a.hash_queries += b.hash_queries;
    a.hash_probes += b.hash_probes;
    a.hash_ne_len += b.hash_ne_len;
    a.collisions += b.collisions;
}

int ed::frontier_once(ed_ctx* c, const FrontierParams& fp, hipStream_t s, double* gpu_ns) {
    const bool timed = (c->opt.flags & ED_FLAG_TIMING) != 0;
    hipError_t e = launch_ctl_init(c->d_ctl, c->d_cnt, c->d_bar, s);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[0], s);
    if (e == hipSuccess) e = launch_frontier(fp, frontier_grid(c), s);
    if (e == hipSuccess && timed) e = hipEventRecord(c->ev[1], s);
    if (e == hipSuccess) e = launch_counters_sum(c->d_cnt, s);
    if (e == hipSuccess) e = hipMemcpyAsync(c->h_ctl, c->d_ctl, sizeof(FrontierCtl), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->h_cnt, c->d_cnt + kMaxGrid, sizeof(CountersDev), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        set_error("ed_distance: frontier launch failed: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    if (timed && gpu_ns) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, c->ev[0], c->ev[1]) == hipSuccess) *gpu_ns += 1e6 * ms;
    }
    return ED_OK;
}

int ed::distance_locked(ed_ctx* c, ed_pair* p, int64_t k_max, uint64_t* k_out, int32_t* rows,
                        uint64_t rows_cap, hipStream_t s, int32_t* fixed_rows, int64_t fixed_K) {
    if (fixed_rows && (k_max < 0 || k_max > fixed_K || rows)) {
        set_error("distance_locked: fixed rows need 0 <= k_max <= %lld", (long long)fixed_K);
        return ED_EINVAL;
    }
    FrontierParams fp;
    int rc = frontier_setup(c, p, fp);
    if (rc != ED_OK) return rc;
    const int64_t n = static_cast<int64_t>(p->len[0]), m = static_cast<int64_t>(p->len[1]);
    const int64_t maxnm = std::max(n, m);
    int64_t K = std::min<int64_t>(maxnm, c->opt.init_rows ? int64_t(c->opt.init_rows) : int64_t(1) << 17);
    if (k_max >= 0) K = std::min<int64_t>(K, std::max<int64_t>(k_max, 1));
    K = std::max<int64_t>(K, 1);
    // caller-owned rows: sized for every round up to k_max, never grown
    if (fixed_rows) K = std::max<int64_t>(k_max, 1);
    int32_t* d_dump = nullptr;
    void* dump_buf = nullptr;
    if (rows) {
        dump_buf = c->pool.get(std::max<uint64_t>(rows_cap, 1) * 4);
        if (!dump_buf) return ED_ENOMEM;
        d_dump = static_cast<int32_t*>(dump_buf);
    }
    auto alloc_rows = [&](int64_t Kn, void** a, void** b) -> bool {
        if (fixed_rows) {
            *a = fixed_rows;
            *b = fixed_rows + (2 * Kn + 5);
            return Kn <= fixed_K;
        }
        *a = c->pool.get(static_cast<size_t>(2 * Kn + 5) * 4);
        *b = c->pool.get(static_cast<size_t>(2 * Kn + 5) * 4);
        return *a && *b;
    };
    auto free_rows = [&](void* a, void* b) {
        if (fixed_rows) return;
        c->pool.put(a);
        c->pool.put(b);
    };
    void *f0 = nullptr, *f1 = nullptr;
    if (!alloc_rows(K, &f0, &f1)) {
        free_rows(f0, f1);
        c->pool.put(dump_buf);
        return ED_ENOMEM;
    }
    fp.kmax = k_max >= 0 ? static_cast<int32_t>(std::min<int64_t>(k_max, INT32_MAX - 1)) : -1;
    fp.dump = d_dump;
    fp.dump_cap = static_cast<int64_t>(rows_cap);
    int32_t t0 = 0;
    int launches = 0;
    double gpu_ns = 0;
    uint64_t rounds_a = 0;
    double us_a = 0, us_b = 0;
    CountersDev total;
    std::memset(&total, 0, sizeof total);
    uint64_t result = 0;
    for (;;) {
        fp.f0 = static_cast<int32_t*>(f0);
        fp.f1 = static_cast<int32_t*>(f1);
        fp.K = static_cast<int32_t>(K);
        fp.t0 = t0;
        rc = frontier_once(c, fp, s, &gpu_ns);
        if (rc != ED_OK) break;
        ++launches;
        counters_add(total, *c->h_cnt);
        const FrontierCtl& st = *c->h_ctl;
        if (launches == 1) {
            rounds_a = static_cast<uint64_t>(st.phase_t);
            us_a = (st.clk_switch - st.clk_begin) / 100.0;  // s_memrealtime: 100 MHz
        }
        if (st.clk_end >= st.clk_switch) us_b += (st.clk_end - st.clk_switch) / 100.0;
        if (st.status == 1 || st.status == 2) {
            result = static_cast<uint64_t>(st.result_t);
            break;
        }
        if (st.status == 3) {
            // grow the rows and resume from the saved frontier f_t
            const int64_t t = st.result_t;
            const int64_t K2 = std::min<int64_t>(maxnm, std::max<int64_t>(2 * K, t + 1));
            if (K2 <= K || fixed_rows) {
                set_error("ed_distance: capacity exhausted at t=%lld (K=%lld)", (long long)t, (long long)K);
                rc = ED_EINTERNAL;
                break;
            }
            void *g0 = nullptr, *g1 = nullptr;
            if (!alloc_rows(K2, &g0, &g1)) {
                free_rows(g0, g1);
                rc = ED_ENOMEM;
                break;
            }
            void* srcrow = st.wbuf == 0 ? f0 : f1;
            // entries [-(t+2), t+2] of the old row -> same diagonals of the new row
            hipError_t e = hipMemcpyAsync(static_cast<int32_t*>(g0) + (K2 + 2) - (t + 2),
                               static_cast<int32_t*>(srcrow) + (K + 2) - (t + 2),
                               static_cast<size_t>(2 * t + 5) * 4, hipMemcpyDeviceToDevice, s);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            free_rows(f0, f1);
            f0 = g0;
            f1 = g1;
            if (e != hipSuccess) {
                set_error("ed_distance: row copy failed: %s", hipGetErrorString(e));
                rc = ED_EDEVICE;
                break;
            }
            K = K2;
            t0 = static_cast<int32_t>(t);
            continue;
        }
        set_error("ed_distance: frontier kernel ended with status %d at t=%d", st.status, st.result_t);
        rc = ED_EINTERNAL;
        break;
    }
    free_rows(f0, f1);
    if (rc == ED_OK) {
        *k_out = result;
        p->rounds = result;
        if (k_max < 0 && !rows) {
            p->known_k = static_cast<int64_t>(result);
            p->known_engine = p->engine;
        }
        p->counters = total;
        p->launches_distance = launches;
        p->gpu_ns_frontier = gpu_ns;
        p->rounds_phase_a = rounds_a;
        p->us_phase_a = us_a;
        p->us_phase_b = us_b;
        if (rows) {
            const uint64_t need = (result + 1) * (result + 1);
            if (need > rows_cap) {
                set_error("ed_distance_dump: %llu rows need %llu entries, capacity %llu",
                          (unsigned long long)(result + 1), (unsigned long long)need,
                          (unsigned long long)rows_cap);
                rc = ED_EINVAL;
            } else {
                hipError_t e = hipMemcpy(rows, d_dump, need * 4, hipMemcpyDeviceToHost);
                if (e != hipSuccess) {
                    set_error("ed_distance_dump: copy failed: %s", hipGetErrorString(e));
                    rc = ED_EDEVICE;
                }
            }
        }
    }
    c->pool.put(dump_buf);
    return rc;
}

int ed_distance(ed_ctx* c, ed_pair* p, int64_t k_max, uint64_t* k_out, void* hip_stream) {
    if (!c || !p || !k_out || p->ctx != c) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    const hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int rc;
    if ((c->opt.flags & ED_FLAG_CERTIFY) && p->engine == ED_ENGINE_HASH && k_max < 0) {
        // the hash result with its traced path checked directly; a failed check
        // (a collision) is answered by the direct engine on the same pair
        std::vector<PathStep> path;
        rc = align_locked(c, p, k_out, path, s);
        if (rc == ED_ECOLLISION) {
            ++p->certify_retries;
            p->engine = ED_ENGINE_DIRECT;
            rc = distance_locked(c, p, -1, k_out, nullptr, 0, s);
            p->engine = ED_ENGINE_HASH;
        }
    } else {
        rc = distance_locked(c, p, k_max, k_out, nullptr, 0, s);
    }
    p->ns_distance = std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    return rc;
}

int ed_distance_dump(ed_ctx* c, ed_pair* p, int64_t k_max, uint64_t* k_out, int32_t* rows,
                     uint64_t rows_cap, void* hip_stream) {
    if (!c || !p || !k_out || !rows || p->ctx != c) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    return distance_locked(c, p, k_max, k_out, rows, rows_cap, static_cast<hipStream_t>(hip_stream));
}

// ---------------------------------------------------------------------------
// stats, buffers, debug queries
// ---------------------------------------------------------------------------
int ed_pair_stats(const ed_pair* p, ed_stats* o) {
    if (!p || !o) return ED_EINVAL;
    std::memset(o, 0, sizeof *o);
    o->n = p->len[0];
    o->m = p->len[1];
    uint32_t alpha = 0;
    const char* misc = static_cast<const char*>(p->misc);
    if (hipMemcpy(&alpha, misc + kMiscAlpha, 4, hipMemcpyDeviceToHost) != hipSuccess) {
        set_error("ed_pair_stats: copy failed");
        return ED_EDEVICE;
    }
    o->bits_per_char = (alpha <= 3u && !p->force8) ? 2 : ((alpha <= 15u && p->w4[0] && !p->force8) ? 4 : 8);
    o->engine = p->engine;
    o->rounds = p->rounds;
    o->updates = p->counters.updates;
    o->lcp_chars = p->counters.lcp_chars;
    o->wave_lcps = p->counters.wave_lcps;
    o->grid_lcps = p->counters.grid_lcps;
    o->wg_lcps = p->counters.wg_lcps;
    o->hash_queries = p->counters.hash_queries;
    o->hash_probes = p->counters.hash_probes;
    o->collisions = p->counters.collisions;
    // Schwartz-Zippel: for distinct strings of length L, h(A) - h(B) is a
    // nonzero polynomial of degree <= L - 1 in the base, so a base drawn
    // uniformly from the kP - 2^21 admissible values makes them hash alike
    // with probability <= (L - 1) / (kP - 2^21).  A run can go wrong only
    // where a verdict that decides a search step is a false "equal"; in the
    // run without collisions those verdicts on distinct strings are the first
    // "unequal" probe of each step, whose L - 1 the kernels add up.
    o->collision_bound = static_cast<double>(p->counters.hash_ne_len) / static_cast<double>(kP - (1ull << 21));
    o->launches = static_cast<uint64_t>(p->launches_distance);
    o->certify_retries = p->certify_retries;
    o->align_device_bytes = p->align_bytes;
    o->align_segment_rounds = p->align_seg;
    o->ns_prepare = p->ns_prepare;
    o->ns_distance = p->ns_distance;
    o->gpu_ns_frontier_kernel = p->gpu_ns_frontier;
    o->gpu_ns_lcp_kernel = p->gpu_ns_lcp;
    o->rounds_phase_a = p->rounds_phase_a;
    o->us_phase_a = p->us_phase_a;
    o->us_phase_b = p->us_phase_b;
    if (p->prep_timed) {
        float ms = 0.f;
        if (hipEventSynchronize(p->ev_prep[1]) == hipSuccess &&
            hipEventElapsedTime(&ms, p->ev_prep[0], p->ev_prep[1]) == hipSuccess)
            o->gpu_ns_prepare_kernel = 1e6 * ms;
        if (p->ev_prep[2] && hipEventElapsedTime(&ms, p->ev_prep[2], p->ev_prep[1]) == hipSuccess)
            o->gpu_ns_table_kernel = 1e6 * ms;
    }
    return ED_OK;
}

int ed_pair_buffer(ed_ctx* c, const ed_pair* p, int which, int kind, void* out, uint64_t cap,
                   uint64_t* len_out) {
    if (!c || !p || which < 0 || which > 1 || !len_out) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    const uint64_t len = p->len[which];
    const void* src = nullptr;
    uint64_t bytes = 0;
    if (kind == ED_BUF_PACKED2) {
        src = p->w2[which];
        bytes = (len + 31) / 32 * 8;
    } else if (kind == ED_BUF_BYTES) {
        src = p->w8[which];
        bytes = len;
    } else if (kind == ED_BUF_PACKED4) {
        src = p->w4[which];
        bytes = (len + 15) / 16 * 8;
        if (!src) {
            set_error("ed_pair_buffer: no 4-bit layout (hash engine or fixed pack_bits)");
            return ED_EINVAL;
        }
    } else if (kind == ED_BUF_TABLE) {
        src = p->tab[which];
        bytes = ((len >> p->log2b) + 1) * 8;
        if (!src) {
            set_error("ed_pair_buffer: no table (direct engine)");
            return ED_EINVAL;
        }
    } else {
        return ED_EINVAL;
    }
    *len_out = bytes;
    if (!out) return ED_OK;
    if (cap < bytes) {
        set_error("ed_pair_buffer: capacity %llu < %llu", (unsigned long long)cap, (unsigned long long)bytes);
        return ED_EINVAL;
    }
    HIP_TRY(hipDeviceSynchronize());
    if (bytes) HIP_TRY(hipMemcpy(out, src, bytes, hipMemcpyDeviceToHost));
    return ED_OK;
}

int ed_debug_lcp(ed_ctx* c, ed_pair* p, int engine, const int64_t* x, const int64_t* y,
                 uint64_t count, int64_t* out, void* hip_stream) {
    if (!c || !p || (count && (!x || !y || !out))) return ED_EINVAL;
    if (engine < -1 || engine > 3) return ED_EINVAL;
    std::lock_guard<std::mutex> lk(c->mu);
    HIP_TRY(hipSetDevice(c->device));
    const int eng = engine < 0 ? static_cast<int>(p->engine) : engine;
    if (eng == 1 && (!p->tab[0] || !p->tab[1])) {
        set_error("ed_debug_lcp: hash engine needs a pair prepared with tables");
        return ED_EINVAL;
    }
    for (uint64_t i = 0; i < count; ++i) {
        if (x[i] < 0 || y[i] < 0 || static_cast<uint64_t>(x[i]) > p->len[0] ||
            static_cast<uint64_t>(y[i]) > p->len[1]) {
            set_error("ed_debug_lcp: query %llu out of range", (unsigned long long)i);
            return ED_EINVAL;
        }
    }
    if (count == 0) return ED_OK;
    if (eng == 1 && p->r != c->r) {
        int rc = ctx_set_hash(c, p->r);
        if (rc != ED_OK) return rc;
    }
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void* buf = c->pool.get(count * 28);
    if (!buf) return ED_ENOMEM;
    int64_t* dx = static_cast<int64_t*>(buf);
    int64_t* dy = dx + count;
    int64_t* dout = dy + count;
    int32_t* dresult = reinterpret_cast<int32_t*>(dout + count);
    LcpQueryParams q;
    std::memset(&q, 0, sizeof q);
    q.p = pair_dev(p);
    q.h = ctx_hash(c);
    q.x = dx;
    q.y = dy;
    q.out = dout;
    q.count = static_cast<int64_t>(count);
    q.engine = eng;
    q.lane_words = c->opt.lane_words ? static_cast<int32_t>(c->opt.lane_words) : (eng == 1 ? 1 : 2);
    q.counters = c->d_cnt;
    q.result = dresult;
    hipError_t e = hipMemcpyAsync(dx, x, count * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dy, y, count * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_ctl_init(c->d_ctl, c->d_cnt, nullptr, s);
    hipEvent_t ev[2] = {nullptr, nullptr};
    const bool timed = (c->opt.flags & ED_FLAG_TIMING) != 0;
    if (eng == 3) {
        // grid tier: one launch per query over the whole grid
        if (e == hipSuccess) e = launch_fill_i32(dresult, static_cast<int64_t>(count), INT32_MAX, s);
        if (e == hipSuccess && timed) e = hipEventCreate(&ev[0]);
        if (e == hipSuccess && timed) e = hipEventCreate(&ev[1]);
        if (e == hipSuccess && timed) e = hipEventRecord(ev[0], s);
        for (uint64_t i = 0; i < count && e == hipSuccess; ++i) {
            q.query = static_cast<int64_t>(i);
            e = launch_lcp_grid(q, c->num_cu, s);
        }
        if (e == hipSuccess && timed) e = hipEventRecord(ev[1], s);
        if (e == hipSuccess) e = launch_lcp_grid_finish(q, s);
    } else if (e == hipSuccess) {
        e = launch_lcp_queries(q, s);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = launch_counters_sum(c->d_cnt, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->h_cnt, c->d_cnt + kMaxGrid, sizeof(CountersDev), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    c->pool.put(buf);
    if (e == hipSuccess && timed && ev[1]) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[0], ev[1]) == hipSuccess) p->gpu_ns_lcp = 1e6 * ms;
    }
    for (hipEvent_t v : ev)
        if (v) (void)hipEventDestroy(v);
    if (e != hipSuccess) {
        set_error("ed_debug_lcp: %s", hipGetErrorString(e));
        return ED_EDEVICE;
    }
    p->counters = *c->h_cnt;
    return ED_OK;
}

const char* ed_strerror(int status) {
    switch (status) {
        case ED_OK: return "ok";
        case ED_EINVAL: return "invalid argument";
        case ED_ENOMEM: return "out of memory";
        case ED_EDEVICE: return "device error";
        case ED_ECOLLISION: return "hash collision not resolved";
        case ED_EBUSY: return "busy";
        case ED_EINTERNAL: return "internal error";
        default: return "unknown status";
    }
}

const char* ed_last_error(void) { return g_last_error.c_str(); }
