// Device building blocks: arithmetic mod 2^61-1, packed-string word fetch,
// and the two LCP engines (direct word compare; prefix-hash search).
#pragma once
#include "internal.h"

namespace ed {

// ---------------------------------------------------------------------------
// Arithmetic modulo P = 2^61 - 1 (the hash of section 2 with a word-size
// modulus).  Operands are always reduced (< P).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t mp_fold(uint64_t s) {  // any s < 2^64
    s = (s & kP) + (s >> 61);
    return s >= kP ? s - kP : s;
}
__device__ __forceinline__ uint64_t mp_add(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s >= kP ? s - kP : s;
}
__device__ __forceinline__ uint64_t mp_sub(uint64_t a, uint64_t b) {
    return a >= b ? a - b : a + kP - b;
}
__device__ __forceinline__ uint64_t mp_mul(uint64_t a, uint64_t b) {
    // a*b = hi*2^64 + lo and 2^64 = 8 (mod P); hi < 2^58 since a, b < 2^61.
    uint64_t lo = a * b;
    uint64_t hi = __umul64hi(a, b);
    return mp_fold((hi << 3) + (lo & kP) + (lo >> 61));
}

// ---------------------------------------------------------------------------
// Wavefront helpers (wave64).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int lane_id() { return __lane_id(); }
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }
__device__ __forceinline__ int ctz64(uint64_t v) { return __builtin_ctzll(v); }
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    return __shfl(static_cast<unsigned long long>(v), src);
}
__device__ __forceinline__ int shfl_i32(int v, int src) { return __shfl(v, src); }

// ---------------------------------------------------------------------------
// A packed string: chars-per-word 2^lcpw, bits-per-char bpc.  fetch(pos)
// returns the 64 bits holding characters pos, pos+1, ... (little-endian:
// character pos in the lowest bits).  Words past the string are zero padding.
// ---------------------------------------------------------------------------
// Device-global words: loads through this type are global (not flat)
// instructions, which LDS operations do not have to wait for.
typedef const uint64_t __attribute__((address_space(1))) gword;

struct SView {
    gword* w;
    int32_t len;
    int32_t lcpw;  // 5 (2-bit), 4 (4-bit) or 3 (8-bit)
    int32_t bpc;   // 2, 4 or 8
    int32_t lbpc;  // log2(bpc): shifts instead of divisions
};

__device__ __forceinline__ uint64_t fetch(const SView& s, int32_t pos) {
    const int32_t q = pos >> s.lcpw;
    const uint32_t sh = static_cast<uint32_t>((pos & ((1 << s.lcpw) - 1)) << s.lbpc);
    const uint64_t lo = s.w[q];
    const uint64_t hi = s.w[q + 1];
    // (hi << 1) << (63 - sh) equals hi << (64 - sh) and is 0 for sh = 0
    return (lo >> sh) | ((hi << 1) << (63 - sh));
}

__device__ __forceinline__ void pair_views(const PairDev& p, uint32_t alpha, SView& A, SView& B) {
    const bool two = (alpha <= 3u) && !p.force8;
    const bool four = !two && alpha <= 15u && !p.force8 && p.a.w4 && p.b.w4;
    A.w = (gword*)(two ? p.a.w2 : (four ? p.a.w4 : p.a.w8));
    B.w = (gword*)(two ? p.b.w2 : (four ? p.b.w4 : p.b.w8));
    A.len = p.a.len;
    B.len = p.b.len;
    A.lcpw = B.lcpw = two ? 5 : (four ? 4 : 3);
    A.bpc = B.bpc = two ? 2 : (four ? 4 : 8);
    A.lbpc = B.lbpc = two ? 1 : (four ? 2 : 3);
}

// ---------------------------------------------------------------------------
// Engine (a), lane tier: one lane compares up to `maxw` words of A from x and
// B from y (at most lim characters).  Returns the matched length; sets *more
// when maxw full words matched and lim is not reached (the LCP continues).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t lcp_lane(const SView& A, const SView& B, int32_t x, int32_t y,
                                            int32_t lim, int maxw, bool* more) {
    const int32_t cpw = 1 << A.lcpw;
    int32_t l = 0;
    for (int k = 0; k < maxw; ++k) {
        if (l >= lim) return lim;
        const uint64_t d = fetch(A, x + l) ^ fetch(B, y + l);
        if (d) {
            const int32_t c = l + (ctz64(d) >> A.lbpc);
            return c < lim ? c : lim;
        }
        l += cpw;
    }
    if (l >= lim) return lim;
    *more = true;
    return l;
}

// ---------------------------------------------------------------------------
// Engine (a), wave tier: all 64 lanes extend one LCP (uniform x, y, lim)
// from offset l, two words per lane per step (1024 chars at 8-bit, 4096 at
// 2-bit), with coalesced loads.  Returns the LCP (uniform).
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t lcp_wave_direct(const SView& A, const SView& B, int32_t x,
                                                   int32_t y, int32_t lim, int32_t l) {
    const int lane = lane_id();
    while (l < lim) {
        const int32_t p0 = l + (lane << A.lcpw);
        const int32_t p1 = p0 + (64 << A.lcpw);
        uint64_t d0 = 0, d1 = 0;
        if (p0 < lim) d0 = fetch(A, x + p0) ^ fetch(B, y + p0);
        if (p1 < lim) d1 = fetch(A, x + p1) ^ fetch(B, y + p1);
        const uint64_t b0 = ballot(d0 != 0);
        if (b0) {
            const int s = ctz64(b0);
            const uint64_t dd = shfl_u64(d0, s);
            const int32_t c = l + (s << A.lcpw) + (ctz64(dd) >> A.lbpc);
            return c < lim ? c : lim;
        }
        const uint64_t b1 = ballot(d1 != 0);
        if (b1) {
            const int s = ctz64(b1);
            const uint64_t dd = shfl_u64(d1, s);
            const int32_t c = l + ((64 + s) << A.lcpw) + (ctz64(dd) >> A.lbpc);
            return c < lim ? c : lim;
        }
        l += 128 << A.lcpw;
    }
    return lim;
}

// Minimum over the 64 lanes of a wavefront.
__device__ __forceinline__ int32_t wave_min(int32_t v) {
    for (int o = 32; o > 0; o >>= 1) {
        const int32_t u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

// Engine (a), wave tier with a step budget: at most `steps` steps of 4 words
// per lane (8192 characters at 2-bit, 2048 at 8-bit per step).  Returns the
// matched length; `done` tells whether the LCP is complete.
__device__ __forceinline__ int32_t lcp_wave_steps(const SView& A, const SView& B, int32_t x, int32_t y,
                                                  int32_t lim, int32_t l, int steps, bool& done) {
    constexpr int W = 4;
    const int lane = lane_id();
    for (int s = 0; s < steps && l < lim; ++s) {
        uint64_t d[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int32_t p = l + ((w * 64 + lane) << A.lcpw);
            const bool ok = p < lim;
            const int32_t q = ok ? p : 0;
            const uint64_t v = fetch(A, x + q) ^ fetch(B, y + q);
            d[w] = ok ? v : 0;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint64_t b = ballot(d[w] != 0);
            if (b) {
                const int s0 = ctz64(b);
                const int32_t c = l + ((w * 64 + s0) << A.lcpw) + (ctz64(shfl_u64(d[w], s0)) >> A.lbpc);
                done = true;
                return c < lim ? c : lim;
            }
        }
        l += (W * 64) << A.lcpw;
    }
    done = l >= lim;
    return l < lim ? l : lim;
}

// ---------------------------------------------------------------------------
// Work counters of one thread.  The per-diagonal counts stay in registers;
// the counts of rarer events (LCPs beyond the lane tier, hash probes) go to
// `sh`, the workgroup's copy in LDS, through one lane per wavefront.
// ---------------------------------------------------------------------------
struct Cnt {
    unsigned long long updates;    // this lane's diagonal updates
    unsigned long long lcp_chars;  // characters matched by this lane's slides
    unsigned long long ne_len;     // sum of L - 1 over the deciding "unequal" verdicts of hash searches
    CountersDev* sh;               // workgroup counters (LDS)
};

__device__ __forceinline__ void cnt_bind(Cnt& c, CountersDev* sh) {
    c.updates = 0;
    c.lcp_chars = 0;
    c.ne_len = 0;
    c.sh = sh;
}

__device__ __forceinline__ void cnt_init_shared(CountersDev* sh) {
    if (threadIdx.x < sizeof(CountersDev) / 8) reinterpret_cast<unsigned long long*>(sh)[threadIdx.x] = 0;
}

// ---------------------------------------------------------------------------
// Engine (b): prefix hashes.  H(S, p) = h(S[0..p)) is rebuilt from the
// blocked table as T[p/b] * r^(p mod b) + h(S[(p/b)b .. p)) (Algorithm 2,
// GetHash, with the block index read as floor(p/b)).  Equality of
// A[x..x+L) and B[y..y+L) is tested as
//   H(A, x+L) - H(B, y+L) == (H(A, x) - H(B, y)) * r^L   (mod P),
// which is the comparison of h(A[x..x+L)) and h(B[y..y+L)) via the inverse
// concatenation of section 2.
// ---------------------------------------------------------------------------
struct HashQ {
    HashDev h;             // r (h.pow0 / h.pow1 as global pointers below)
    gword* pow0;           // r^a, a < 65536
    gword* pow1;           // r^(65536 a), a < 65536
    gword* rinv;           // r^(-d), d = 0..32
    uint64_t r4;           // r^4
    uint64_t r32;          // r^32
    const uint64_t (*lut32)[256];  // LDS: packed byte k of a 2-bit word, weights r^(31-4k-j)
    int32_t log2b;
};

__device__ __forceinline__ uint64_t pow_r(const HashQ& q, int32_t L) {
    return mp_mul(q.pow0[L & 0xFFFF], q.pow1[static_cast<uint32_t>(L) >> 16]);
}

// h(S[s .. s+e)), s a multiple of the block size.
__device__ __forceinline__ uint64_t partial_hash(const SView& S, const HashQ& q, int32_t s,
                                                 int32_t e) {
    uint64_t h = 0;
    int32_t i = 0;
    if (S.bpc == 2) {
        // whole packed bytes (4 characters) through the LDS table, when the
        // block start is byte aligned (b >= 4)
        if ((s & 3) == 0) {
            for (; i + 4 <= e; i += 4) {
                const int32_t pos = s + i;
                const uint64_t word = S.w[pos >> 5];
                const uint32_t byte = static_cast<uint32_t>(word >> (((pos >> 2) & 7) * 8)) & 0xFFu;
                h = mp_add(mp_mul(h, q.r4), q.lut32[7][byte]);  // weights r^(3-j)
            }
        }
        for (; i < e; ++i) {
            const int32_t pos = s + i;
            const uint64_t c = (S.w[pos >> 5] >> ((pos & 31) * 2)) & 3u;
            h = mp_add(mp_mul(h, q.h.r), c);
        }
    } else {
        for (; i < e; ++i) {
            const int32_t pos = s + i;
            const uint64_t c = (S.w[pos >> 3] >> ((pos & 7) * 8)) & 0xFFu;
            h = mp_add(mp_mul(h, q.h.r), c);
        }
    }
    return h;
}

// b = 32 on 2-bit strings: the block's characters past e are masked to zero
// and the whole block is hashed with the weights r^(31-k) (8 table lookups),
// giving M = h(S[32j .. 32j+e)) r^(32-e); then
// H = T[j] r^e + h(S[32j .. 32j+e)) = (T[j] r^32 + M) r^(e-32).
__device__ __forceinline__ uint64_t block32_masked_hash(const SView& S, const HashQ& q, int32_t j, int32_t e) {
    const uint64_t w = S.w[j] & ((1ull << (2 * e)) - 1);
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += q.lut32[k][(w >> (8 * k)) & 0xFFu];
    return mp_fold(s);
}

__device__ __forceinline__ uint64_t get_hash(const SView& S, gword* T, const HashQ& q,
                                             int32_t p) {
    const int32_t j = p >> q.log2b;
    const int32_t e = p & ((1 << q.log2b) - 1);
    uint64_t h = T[j];
    if (!e) return h;
    if (q.log2b == 5) {
        if (S.bpc == 2)
            return mp_mul(mp_add(mp_mul(h, q.r32), block32_masked_hash(S, q, j, e)), q.rinv[32 - e]);
        // 8-bit: the block's two words of the shorter side are loaded together
        // and at most 16 characters are folded from registers: the prefix when
        // e <= 16, else (when the next entry exists) the suffix, with
        // H = (T[j+1] - h(S[p .. 32(j+1)))) r^(e-32)
        if (e <= 16) {
            const uint64_t w0 = S.w[4 * j], w1 = S.w[4 * j + 1];
            uint64_t hp = 0;
            for (int c = 0; c < e; ++c)
                hp = mp_add(mp_mul(hp, q.h.r), ((c < 8 ? w0 >> (8 * c) : w1 >> (8 * (c - 8))) & 0xFFu));
            return mp_add(mp_mul(h, q.pow0[e]), hp);
        }
        if (32 * (j + 1) <= S.len) {
            const uint64_t w2 = S.w[4 * j + 2], w3 = S.w[4 * j + 3];
            uint64_t hs = 0;
            for (int c = e; c < 32; ++c)
                hs = mp_add(mp_mul(hs, q.h.r), ((c < 24 ? w2 >> (8 * (c - 16)) : w3 >> (8 * (c - 24))) & 0xFFu));
            return mp_mul(mp_sub(T[j + 1], hs), q.rinv[32 - e]);
        }
    }
    return mp_add(mp_mul(h, q.pow0[e]), partial_hash(S, q, j << q.log2b, e));
}

// Wave-parallel LCP by hashing (uniform x, y, lim; the first l0 characters
// are known to match and l0 < lim).  Galloping: lane k tests L = l0 * 2^(k+1)
// (the last probe clamped to lim); then 64-ary narrowing of the interval
// (lo equal, hi unequal) until it spans at most one direct wave step; the
// direct step finds the mismatch character, which confirms the answer.  When
// the direct step finds no mismatch below hi, a hash collision made some
// "equal" verdict wrong: the LCP is recomputed directly (counted).
__device__ __forceinline__ int32_t lcp_wave_hash(const SView& A, const SView& B, gword* TA,
                                 gword* TB, const HashQ& q, int32_t x, int32_t y,
                                 int32_t lim, int32_t l0, Cnt& cnt) {
    const int lane = lane_id();
    const int32_t cpw = 1 << A.lcpw;
    const int32_t span = 64 * cpw;  // one direct step
    const uint64_t hax = get_hash(A, TA, q, x);
    const uint64_t hby = get_hash(B, TB, q, y);
    const uint64_t d0 = mp_sub(hax, hby);
    if (lane == 0) atomicAdd(&cnt.sh->hash_queries, 1ull);

    auto eq = [&](int32_t L) -> bool {
        const uint64_t lhs = mp_sub(get_hash(A, TA, q, x + L), get_hash(B, TB, q, y + L));
        return lhs == mp_mul(d0, pow_r(q, L));
    };

    int32_t lo = l0, hi;
    {
        // galloping probes
        const int64_t Lr = static_cast<int64_t>(l0) << (lane < 40 ? lane + 1 : 40);
        const int64_t Lprev = static_cast<int64_t>(l0) << (lane < 40 ? lane : 40);
        const bool active = Lprev < lim;  // first probe that reaches lim is the last one
        const int32_t L = static_cast<int32_t>(Lr < lim ? Lr : lim);
        const bool e = active ? eq(L) : true;
        const uint64_t pa = ballot(active);
        if (lane == 0) atomicAdd(&cnt.sh->hash_probes, static_cast<unsigned long long>(__builtin_popcountll(pa)));
        const uint64_t ne = ballot(active && !e);
        if (ne == 0) return lim;  // every probe up to lim matched
        const int k = ctz64(ne);
        hi = shfl_i32(L, k);
        if (k > 0) lo = shfl_i32(L, k - 1);
        // the one verdict on distinct strings that decides this step
        if (lane == 0) cnt.ne_len += static_cast<unsigned long long>(hi - 1);
    }
    while (hi - lo > span) {
        const int32_t step = (hi - lo + 63) / 64;
        const int32_t M = lo + (lane + 1) * step;
        const bool active = M < hi;
        const bool e = active ? eq(M) : true;
        const uint64_t act = ballot(active);
        if (lane == 0) atomicAdd(&cnt.sh->hash_probes, static_cast<unsigned long long>(__builtin_popcountll(act)));
        const uint64_t ne = ballot(active && !e);
        if (ne) {
            const int k = ctz64(ne);
            const int32_t nhi = shfl_i32(M, k);
            if (k > 0) lo = shfl_i32(M, k - 1);
            hi = nhi;
            if (lane == 0) cnt.ne_len += static_cast<unsigned long long>(hi - 1);
        } else {
            lo = shfl_i32(M, 63 - __builtin_clzll(act));
        }
    }
    // direct step over [lo, hi): hi is certainly unequal (different hashes
    // mean different strings), so a mismatch lies in [0, hi)
    const int32_t p = lo + (lane << A.lcpw);
    uint64_t d = 0;
    if (p < hi) d = fetch(A, x + p) ^ fetch(B, y + p);
    const uint64_t bm = ballot(d != 0);
    if (bm) {
        const int s = ctz64(bm);
        const uint64_t dd = shfl_u64(d, s);
        const int32_t c = lo + (s << A.lcpw) + (ctz64(dd) >> A.lbpc);
        if (c < hi) return c;
    }
    // no mismatch in [lo, hi): a collision hid one below lo
    if (lane == 0) atomicAdd(&cnt.sh->collisions, 1ull);
    return lcp_wave_direct(A, B, x, y, lim, 0);
}

// LDS copy of the host-built tables of packed bytes: lut32[k][v] is the hash
// of the 4 characters of byte v as byte k of a 32-character word, weights
// r^(31-4k-j) (row 7 is the hash of the 4 characters alone).
__device__ __forceinline__ void load_lut32(uint64_t (*lut32)[256], const uint64_t* rtab, int tid, int nthreads) {
    for (int i = tid; i < 8 * 256; i += nthreads) lut32[i >> 8][i & 255] = rtab[kRtabLut32 + i];
}

// ---------------------------------------------------------------------------
// The slide of one diagonal: LCP(c, c - i) on the chosen engine.  Called by
// all 64 lanes of a wave together; lanes with valid=false take part in the
// wave-level work only.  Returns the LCP for valid lanes (0 otherwise).
// ---------------------------------------------------------------------------
struct Engine {
    SView A, B;
    gword* TA;
    gword* TB;
    HashQ q;
    int32_t kind;        // 0 direct, 1 hash
    int32_t lane_words;
    int32_t hash_first;  // hash engine: a slide past the lane stage goes to the hash search at once
};

__device__ __forceinline__ int32_t slide(const Engine& en, bool valid, int32_t x, int32_t y,
                                         Cnt& cnt) {
    int32_t lim = 0, l = 0;
    bool more = false;
    if (valid) {
        const int32_t la = en.A.len - x, lb = en.B.len - y;
        lim = la < lb ? la : lb;
        if (lim > 0) l = lcp_lane(en.A, en.B, x, y, lim, en.lane_words, &more);
    }
    uint64_t pend = ballot(more);
    while (pend) {
        const int src = ctz64(pend);
        pend &= pend - 1;
        const int32_t jx = shfl_i32(x, src), jy = shfl_i32(y, src);
        const int32_t jlim = shfl_i32(lim, src), jl = shfl_i32(l, src);
        int32_t r;
        if (en.kind == 1 && jl > 0)
            r = lcp_wave_hash(en.A, en.B, en.TA, en.TB, en.q, jx, jy, jlim, jl, cnt);
        else
            r = lcp_wave_direct(en.A, en.B, jx, jy, jlim, jl);
        if (lane_id() == 0) atomicAdd(&cnt.sh->wave_lcps, 1ull);
        if (lane_id() == src) l = r;
    }
    if (valid) cnt.lcp_chars += static_cast<unsigned long long>(l);
    return l;
}

// Every thread of the workgroup: wave sums of the register counters into the
// LDS copy, then one thread adds the LDS copy to the workgroup's own slot of
// the global counters (no address shared between workgroups: a shared
// counter would serialise one atomic per workgroup; the slots are summed by
// counters_sum_kernel).
__device__ __forceinline__ void flush_counters(Cnt& c, CountersDev* g) {
    auto red = [](unsigned long long v) {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        return v;
    };
    const unsigned long long u = red(c.updates), lc = red(c.lcp_chars), he = red(c.ne_len);
    if (lane_id() == 0) {
        if (u) atomicAdd(&c.sh->updates, u);
        if (lc) atomicAdd(&c.sh->lcp_chars, lc);
        if (he) atomicAdd(&c.sh->hash_ne_len, he);
    }
    __syncthreads();
    if (threadIdx.x == 0 && g) {
        g += blockIdx.x % kMaxGrid;
        const CountersDev& s = *c.sh;
        if (s.updates) atomicAdd(&g->updates, s.updates);
        if (s.lcp_chars) atomicAdd(&g->lcp_chars, s.lcp_chars);
        if (s.wave_lcps) atomicAdd(&g->wave_lcps, s.wave_lcps);
        if (s.grid_lcps) atomicAdd(&g->grid_lcps, s.grid_lcps);
        if (s.wg_lcps) atomicAdd(&g->wg_lcps, s.wg_lcps);
        if (s.hash_queries) atomicAdd(&g->hash_queries, s.hash_queries);
        if (s.hash_probes) atomicAdd(&g->hash_probes, s.hash_probes);
        if (s.hash_ne_len) atomicAdd(&g->hash_ne_len, s.hash_ne_len);
        if (s.collisions) atomicAdd(&g->collisions, s.collisions);
    }
}

}  // namespace ed
