// Prepare a pair: the input bytes of both strings are read once.
//   pack_kernel   streaming, one wavefront per 4096-character chunk:
//                 alphabet detection (bitwise OR of every character; 2-bit
//                 packing is possible when the OR is <= 3), each chunk in the
//                 narrowest layout its characters allow (2-bit words, 4-bit
//                 words, or the 8-bit copy); with prefix tables of block size
//                 32 it also takes the block hashes of the input bytes on the
//                 matrix cores and the first table pass;
//   after_pack_kernel  the pair's alphabet from the pack workgroups' slots,
//                 the chunks the pair's layout still lacks (rest pass), and
//                 at b = 32 the chunk totals of the tile-hash scan;
//   table_*       (hash engine) prefix table T[j] = h(S[0..jb)) mod 2^61-1
//                 (sections 3.2 and 3.3, Algorithm 2 "Build"): block hashes
//                 (matrix products at b = 32, else LDS lookup tables over the
//                 packed words or the 8-bit copy; h is linear in the
//                 characters), combined under the concatenation
//                 h(S1 S2) = h(S1) r^|S2| + h(S2) within each tile, across
//                 tiles by a separate scan of the tile hashes.
#include "device.h"

namespace ed {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef int i32x4 __attribute__((ext_vector_type(4)));

// LDS of the table passes (one of the two lookup tables, by the pair's packing)
struct TableShared {
    union {
        uint64_t lut32[8][256];  // packed byte k of a 2-bit word: sum_j c_j r^(31-4k-j)
        uint64_t lut8[8][256];   // byte k of an 8-char word: v r^(7-k)
    };
    uint64_t rp[65];       // r^p
    uint64_t rseg[257];    // r^(64 k)
    uint64_t rinv256[65];  // r^(-256 d)
    uint64_t stage[kPrepThreads / 64][64 * 9];  // per wavefront: T entries of a tile, 9 slots per lane
};

// The fields of one of the two strings, chosen by a uniform flag: a select
// between two kernel arguments (scalar registers), not an indexed load.
struct StrSel {
    const uint8_t* raw;
    uint64_t* w2;
    uint64_t* w4;
    uint64_t* w8;
    uint64_t* tab;
    int32_t len;
    int32_t tile0;
    __device__ __forceinline__ StrSel(const PrepParams& P, bool second)
        : raw(second ? P.s[1].raw : P.s[0].raw),
          w2(second ? P.s[1].w2 : P.s[0].w2),
          w4(second ? P.s[1].w4 : P.s[0].w4),
          w8(second ? P.s[1].w8 : P.s[0].w8),
          tab(second ? P.s[1].tab : P.s[0].tab),
          len(second ? P.s[1].len : P.s[0].len),
          tile0(second ? P.s[1].tile0 : P.s[0].tile0) {}
};

__device__ __forceinline__ int32_t imin32(int32_t a, int32_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint32_t pack_dword(uint32_t d) {
    // four 8-bit characters -> four 2-bit codes (low bits of each byte)
    return (d & 3u) | ((d >> 6) & 0xCu) | ((d >> 12) & 0x30u) | ((d >> 18) & 0xC0u);
}

__device__ __forceinline__ uint64_t pack_nibbles(uint32_t d) {
    // four 8-bit characters -> four 4-bit codes (low bits of each byte)
    return (d & 0xFu) | ((d >> 4) & 0xF0u) | ((d >> 8) & 0xF00u) | ((d >> 12) & 0xF000u);
}

// Hash of a unit of U characters of a packed word (U = 4, 8, 16, 32; unit u
// of the word): sum over its bytes of lut32[8 - U/4 + k], the entries whose
// weights r^(U-1-4k-j) match the unit's length.  At most 8 terms below 2^61
// are added before the fold, so the sum stays below 2^64.
template <int U>
__device__ __forceinline__ uint64_t unit_hash2(const TableShared& S, uint64_t w, int u) {
    constexpr int nb = U / 4;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < nb; ++k) s += S.lut32[8 - nb + k][(w >> (8 * (u * nb + k))) & 0xFFu];
    return mp_fold(s);
}

// Hash of one 8-bit word (8 characters).
__device__ __forceinline__ uint64_t word_hash8(const TableShared& S, uint64_t w) {
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += S.lut8[k][(w >> (8 * k)) & 0xFFu];
    return mp_fold(s);
}

}  // namespace


// Block hashes of 32 characters on the matrix cores.  h of a block is linear
// in its characters, h = sum_j c_j r^(31 - j), and with each weight written
// as 8 signed base-256 digits d[j][t] it is sum_t 256^t X_t with
// X_t = sum_j c_j d[j][t]: an int8 matrix product of the characters with a
// digit matrix.  One v_mfma_i32_16x16x64_i8 takes 16 columns of 64
// characters (two blocks, one per half) against 16 rows (two halves x 8
// digits; each row's weights are zero outside its half).  Characters enter
// as c - 128 (signed bytes) and the host constant restores the offsets.
// Lane l (i = l mod 16, g = l / 16) holds rows 4g .. 4g + 3 of column i:
// digits 4 (g mod 2) .. + 3 of the block in half g / 2.  The hash does not
// depend on the packing (a 2-bit code is the character's value), so it is
// taken from the input bytes.
//
// Product p of a tile takes its characters 1024 p .. + 1023 (one load
// instruction reads them all): column i, half h is block 32 p + 16 h + i,
// lane l's operand is its characters 16 (g mod 2) .. + 15 (kMmaOff).  The
// A operand holds at the same byte positions the digits of those
// characters' weights, so each character meets its own weights whichever
// way the instruction orders its 64 products.  Products come in pairs: the
// even-g lanes keep the first product's block, the odd-g lanes the
// second's, and one exchange between lanes l and l ^ 16 completes every
// lane's digits.
__device__ __forceinline__ int32_t mma_off(int lane) {
    return 32 * (lane & 15) + 512 * (lane >> 5) + 16 * ((lane >> 4) & 1);
}

// This lane's digits of one product (4 (g mod 2) .. + 3) as a value mod P
// times 256^(4 (g mod 2)); the offset makes the digit sums non-negative.
__device__ __forceinline__ uint64_t mma_part(i32x4 x, int32_t rot) {
    uint64_t z = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) z += static_cast<uint64_t>(static_cast<uint32_t>(x[i] + (1 << 19))) << (8 * i);
    return ((z << rot) & kP) + (z >> (61 - rot));  // z 2^rot mod P, z < 2^61
}

// The even-g lane keeps product 0's value, the odd-g lane product 1's; each
// takes the other half of its digits from lane l ^ 16.
__device__ __forceinline__ uint64_t mma_pair(uint64_t z0, uint64_t z1, bool even, uint64_t kfix) {
    const uint64_t own = even ? z0 : z1;
    const uint64_t send = even ? z1 : z0;
    return mp_fold(own + __shfl_xor(static_cast<unsigned long long>(send), 16) + kfix);
}

__device__ __forceinline__ i32x4 as_i32x4(u32x4 v, uint32_t x) {
    return i32x4{static_cast<int>(v.x ^ x), static_cast<int>(v.y ^ x), static_cast<int>(v.z ^ x),
                 static_cast<int>(v.w ^ x)};
}

// Streaming pass: wavefront w takes chunks of 4096 characters w, w + W, ...
// (W wavefronts in the grid), or, when it takes the block hashes too, tiles
// w, w + W, ... chunk by chunk; a chunk is 4 loads of 1024 characters, lane
// l holding the 16 characters at 16 l of each, or at mma_off(l) when the
// block hashes are taken (every load and store instruction covers a
// contiguous range).  It packs
// each piece into 32 bits (a quarter of a packed word) or copies it to the
// 8-bit words, both stored at the piece's own position.  Chunk slots past
// the end of a string are written as zeros (padding the last tile).
//
// With prefix tables of block size 32 (fuse_table) the pass also takes the
// block hashes of its tile from the same registers (see above), stores each
// at T[j + 1] (block j), the slot whose prefix value the emission pass
// writes over it, and, as the first table pass does for other block sizes,
// folds the 8 blocks of each lane's 256 characters and stores the in-tile
// prefix of each lane (lane_excl) and the tile's hash (tile_agg).
// A store of the packed words or the 8-bit copy: non-temporal for a pair
// larger than the memory-side cache (nothing reads it again before the
// frontier, and it would only evict other lines), else an ordinary store
// (the lines stay for the frontier's first reads).
template <bool NT, typename T>
__device__ __forceinline__ void pack_store(T* p, T v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <bool NT>
__global__ __launch_bounds__(kPrepThreads) void pack_kernel(PrepParams P) {
    __shared__ uint64_t stage[kPrepThreads / 64][64 * 9];
    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t nwaves = static_cast<int32_t>((gridDim.x * blockDim.x) >> 6);
    const int32_t total = P.total_tiles;
    const bool fuse = P.fuse_table != 0;
    // the operands' order only when the block hashes are taken
    const int32_t off = fuse ? mma_off(lane) : 16 * lane;
    const int g4 = lane >> 4;
    const bool even = (g4 & 1) == 0;
    uint64_t* st = &stage[threadIdx.x >> 6][0];
    i32x4 ablk{0, 0, 0, 0};
    uint64_t kblk = 0, r32 = 0, rseg = 0, rinv = 0;
    if (fuse) {
        const u32x4 av = reinterpret_cast<const u32x4*>(P.rtab + kRtabMmaA)[lane];
        ablk = as_i32x4(av, 0u);
        kblk = P.rtab[kRtabMmaK];
        r32 = P.rtab[32];
        rseg = P.rtab[kRtabRseg + 4 * (63 - lane)];  // r^(256 (63 - lane))
        rinv = P.rtab[kRtabRinv256 + 64 - lane];     // r^(-256 (64 - lane))
    }
    const int32_t rot = even ? 0 : 32;
    // the block this lane ends up with in pair q: 64 q + lam
    const int32_t lam = (lane & 15) + 16 * (g4 >> 1) + 32 * (g4 & 1);
    uint32_t orr = 0;
    uint32_t packed_any = 0;  // bit c: this wavefront wrote a chunk of class c < 2
    // chunk c (of its string) in v
    auto load = [&](const StrSel& str, int32_t c, u32x4 (&v)[4]) {
        const int32_t cbase = c * kChunkChars;
        const int32_t len = str.len;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t pos = cbase + k * 1024 + off;
            if (pos + 16 <= len) {
                v[k] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(str.raw + pos));
            } else {
                uint32_t d[4] = {0, 0, 0, 0};
                for (int j = 0; j < 16; ++j)
                    if (pos + j < len) d[j >> 2] |= static_cast<uint32_t>(str.raw[pos + j]) << (8 * (j & 3));
                v[k].x = d[0];
                v[k].y = d[1];
                v[k].z = d[2];
                v[k].w = d[3];
            }
        }
    };
    // alphabet OR, 2-bit words, 4-bit words or 8-bit copy, chunk class
    auto pack = [&](const StrSel& str, int32_t c, const u32x4 (&v)[4]) {
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) o |= v[k].x | v[k].y | v[k].z | v[k].w;
        orr |= o;
        const bool big = ballot((o & 0xFCFCFCFCu) != 0u) != 0;
        const bool nib = big && str.w4 && ballot((o & 0xF0F0F0F0u) != 0u) == 0;
        if (!big) {
            uint32_t* dst = reinterpret_cast<uint32_t*>(str.w2 + static_cast<int64_t>(c) * kChunkWords2);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                pack_store<NT>(dst + k * 64 + (off >> 4), pack_dword(v[k].x) | (pack_dword(v[k].y) << 8) |
                                                              (pack_dword(v[k].z) << 16) | (pack_dword(v[k].w) << 24));
        } else if (nib) {
            uint64_t* dst = str.w4 + static_cast<int64_t>(c) * kChunkWords4;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                dst[k * 64 + (off >> 4)] = pack_nibbles(v[k].x) | (pack_nibbles(v[k].y) << 16) |
                                           (pack_nibbles(v[k].z) << 32) | (pack_nibbles(v[k].w) << 48);
        }
        if ((big && !nib) || P.force8) {
            u32x4* dst = reinterpret_cast<u32x4*>(str.w8 + static_cast<int64_t>(c) * kChunkWords8);
#pragma unroll
            for (int k = 0; k < 4; ++k) pack_store<NT>(dst + k * 64 + (off >> 4), v[k]);
        }
        const uint32_t cls = !big ? 0u : (nib ? 1u : 2u);
        if (lane == 0) P.chunk_big[str.tile0 * kTileChunks + c] = static_cast<uint8_t>(cls);
        packed_any |= cls < 2u ? (1u << cls) : 0u;
    };
    u32x4 v[4];
    if (!fuse) {
        // chunks w, w + W, ... (no state across chunks)
        const int32_t chunks = total * kTileChunks;
        for (int32_t gc = wave; gc < chunks; gc += nwaves) {
            const StrSel str(P, gc >= P.s[1].tile0 * kTileChunks);
            const int32_t c = gc - str.tile0 * kTileChunks;
            load(str, c, v);
            pack(str, c, v);
        }
    } else {
        // tiles w, w + W, ..., chunk by chunk; the next chunk's loads are
        // issued before this chunk's work
        u32x4 nv[4];
        int32_t g = wave;
        int cc = 0;
        if (g < total) {
            const StrSel str(P, g >= P.s[1].tile0);
            load(str, (g - str.tile0) * kTileChunks, v);
        }
        while (g < total) {
            int32_t ng = g;
            int ncc = cc + 1;
            if (ncc == kTileChunks) {
                ncc = 0;
                ng += nwaves;
            }
            if (ng < total) {
                const StrSel nstr(P, ng >= P.s[1].tile0);
                load(nstr, (ng - nstr.tile0) * kTileChunks + ncc, nv);
            }
            const StrSel str(P, g >= P.s[1].tile0);
            const int32_t t = g - str.tile0;
            pack(str, t * kTileChunks + cc, v);
#pragma unroll
            for (int k = 0; k < 4; k += 2) {
                const i32x4 x0 = __builtin_amdgcn_mfma_i32_16x16x64_i8(ablk, as_i32x4(v[k], 0x80808080u),
                                                                       i32x4{0, 0, 0, 0}, 0, 0, 0);
                const i32x4 x1 = __builtin_amdgcn_mfma_i32_16x16x64_i8(ablk, as_i32x4(v[k + 1], 0x80808080u),
                                                                       i32x4{0, 0, 0, 0}, 0, 0, 0);
                const int32_t blk = 64 * (2 * cc + k / 2) + lam;
                st[(blk >> 3) * 9 + (blk & 7)] = mma_pair(mma_part(x0, rot), mma_part(x1, rot), even, kblk);
            }
            if (cc == kTileChunks - 1) {
                const int32_t base = t * (kTileChars / 32) + 1;  // T index of the tile's first block end
                const int32_t last = str.len >> 5;
                __builtin_amdgcn_wave_barrier();
                // block hashes to T (64 consecutive entries per store); this
                // lane's 8 blocks folded by Horner's rule
                uint64_t h = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const int32_t i = k * 64 + lane;
                    if (base + i <= last) str.tab[base + i] = st[(i >> 3) * 9 + (i & 7)];
                    h = mp_add(mp_mul(h, r32), st[lane * 9 + k]);
                }
                __builtin_amdgcn_wave_barrier();
                // I(l) = sum over lanes l' <= l of h(l') r^(256 (63 - l')): the
                // tile's hash is I(63), the hash of its characters before lane
                // l is I(l - 1) r^(-256 (64 - l))
                uint64_t x = mp_mul(h, rseg);
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint64_t y = __shfl_up(static_cast<unsigned long long>(x), d);
                    if (lane >= d) x = mp_add(x, y);
                }
                const uint64_t ip = __shfl_up(static_cast<unsigned long long>(x), 1);
                P.lane_excl[static_cast<int64_t>(g) * 64 + lane] = lane == 0 ? 0 : mp_mul(ip, rinv);
                if (lane == 63) P.tile_agg[g] = x;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) v[k] = nv[k];
            g = ng;
            cc = ncc;
        }
    }
    // this workgroup's alphabet OR and chunk classes in a slot of its own
    // (no atomics, nothing to clear first); after_pack_kernel reduces them
    __shared__ uint32_t wor[kPrepThreads / 64];
    orr |= orr >> 16;
    orr |= orr >> 8;
    orr &= 0xFFu;
    for (int s = 32; s > 0; s >>= 1) orr |= __shfl_xor(orr, s);
    if (lane == 0) wor[threadIdx.x >> 6] = orr | (packed_any << 8);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t o = 0;
        for (int w = 0; w < kPrepThreads / 64; ++w) o |= wor[w];
        P.wg_or[blockIdx.x] = o;
    }
}

// Prefix tables of both strings (hash engine), after pack_kernel (and
// after_pack_kernel), in three passes with no shared counter.  A tile of
// 16384 characters is one wavefront's work, 256 consecutive characters per
// lane; tiles are assigned statically to wavefronts.
//   table_tiles_kernel<false>  per tile: the hash of each lane's characters
//                              (Horner over words), an inclusive scan over the
//                              lanes under h(S1 S2) = h(S1) r^|S2| + h(S2);
//                              stores each lane's exclusive prefix within the
//                              tile (lane_excl) and the tile's hash (tile_agg)
//   table_total_kernel,        per string: prefix hash before every tile
//   table_scan_kernel          (tile_prefix), Horner over tiles with R = r^16384
//   table_tiles_kernel<true>   per lane: the prefix hash at its first
//                              character from the two, then Horner over its
//                              units with T[j] written at every block end
// The characters come from the 2-bit words when the pair is packable, from the
// 8-bit copy otherwise.  Past the end of a string the words are zero; values
// there are never written to T.
constexpr int kLaneChars = kTileChars / 64;    // 256
constexpr int kLaneWords2 = kLaneChars / 32;   // 8 packed words
constexpr int kLaneWords8 = kLaneChars / 8;    // 32 byte-words

// The lane's packed words of tile g (four 16-byte loads).
__device__ __forceinline__ void load_lane2(const PrepParams& P, int32_t g, int lane, uint64_t (&v)[kLaneWords2]) {
    const StrSel str(P, g >= P.s[1].tile0);
    const int32_t t = g - str.tile0;
    const u32x4* src = reinterpret_cast<const u32x4*>(str.w2 + static_cast<int64_t>(t) * kTileWords2 + lane * kLaneWords2);
#pragma unroll
    for (int k = 0; k < kLaneWords2 / 2; ++k) {
        const u32x4 q = src[k];
        v[2 * k] = static_cast<uint64_t>(q.x) | (static_cast<uint64_t>(q.y) << 32);
        v[2 * k + 1] = static_cast<uint64_t>(q.z) | (static_cast<uint64_t>(q.w) << 32);
    }
}

__device__ __forceinline__ void load_lane8(const PrepParams& P, int32_t g, int lane, uint64_t (&v)[kLaneWords8]) {
    const StrSel str(P, g >= P.s[1].tile0);
    const int32_t t = g - str.tile0;
    const u32x4* src = reinterpret_cast<const u32x4*>(str.w8 + static_cast<int64_t>(t) * kTileWords8 + lane * kLaneWords8);
#pragma unroll
    for (int k = 0; k < kLaneWords8 / 2; ++k) {
        const u32x4 q = src[k];
        v[2 * k] = static_cast<uint64_t>(q.x) | (static_cast<uint64_t>(q.y) << 32);
        v[2 * k + 1] = static_cast<uint64_t>(q.z) | (static_cast<uint64_t>(q.w) << 32);
    }
}

// Writes T at block end e (e - seg in (0, 256]) with value h: into the
// wavefront's staging slots when `st` is set (b = 32 .. 128), else directly.
struct TabPut {
    uint64_t* tab;
    uint64_t* st;  // this lane's 9 staging slots, or nullptr
    int32_t seg, len, log2b, bmask;
    __device__ __forceinline__ void operator()(int32_t e, uint64_t h) const {
        if ((e & bmask) == 0 && e <= len) {
            if (st)
                st[((e - seg) >> log2b) - 1] = h;
            else
                tab[e >> log2b] = h;
        }
    }
};

// Emission of T over the lane's characters in units of U characters of
// packed words (U = 4, 8, 16 or 32, U <= b): h enters as the prefix hash at
// the lane's first character.
template <int U>
__device__ __forceinline__ void emit_units2(const TableShared& S, const uint64_t (&v)[kLaneWords2], uint64_t h,
                                            const TabPut& put) {
    const uint64_t ru = S.rp[U];
#pragma unroll
    for (int q = 0; q < kLaneWords2; ++q) {
#pragma unroll
        for (int u = 0; u < 32 / U; ++u) {
            h = mp_add(mp_mul(h, ru), unit_hash2<U>(S, v[q], u));
            put(put.seg + q * 32 + (u + 1) * U, h);
        }
    }
}

// SMALLB: instantiation for blocks of at most 4 characters (units of 4
// characters or single characters); the others use units of 8 to 32.
template <bool EMIT, bool TWO, bool SMALLB>
__device__ __forceinline__ void table_tiles(const PrepParams& P, TableShared& S, int32_t gw, int32_t W, int lane,
                                            int wave) {
    const int32_t total = P.total_tiles;
    const int32_t log2b = P.log2b;
    const int32_t bmask = (1 << log2b) - 1;
    // b = 32 .. 128: a tile's 16384 / b entries go through LDS, so that every
    // store instruction writes 64 consecutive entries
    const bool staged = log2b >= 5 && log2b <= 7;
    const int32_t lepl = 8 - log2b;  // log2 of the entries per lane when staged
    constexpr int NW = TWO ? kLaneWords2 : kLaneWords8;
    uint64_t cur[NW];
    uint64_t nxt[kLaneWords2];
    if constexpr (TWO) {
        if (gw < total) load_lane2(P, gw, lane, cur);
    }
    for (int32_t g = gw; g < total; g += W) {
        if constexpr (TWO) {
            // the next tile's words are requested before this tile's arithmetic
            if (g + W < total) load_lane2(P, g + W, lane, nxt);
        } else {
            load_lane8(P, g, lane, cur);
        }
        const StrSel str(P, g >= P.s[1].tile0);
        const int32_t t = g - str.tile0;
        const int32_t seg = t * kTileChars + lane * kLaneChars;
        const int32_t len = str.len;
        if constexpr (!EMIT) {
            uint64_t h = 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                if constexpr (TWO)
                    h = mp_add(mp_mul(h, S.rp[32]), unit_hash2<32>(S, cur[q], 0));
                else
                    h = mp_add(mp_mul(h, S.rp[8]), word_hash8(S, cur[q]));
            }
            // I(l) = sum over lanes l' <= l of h(l') r^(256 (63 - l')): a plain
            // prefix sum; the tile's hash is I(63) and the hash of its
            // characters before lane l is I(l - 1) r^(-256 (64 - l))
            uint64_t x = mp_mul(h, S.rseg[4 * (63 - lane)]);
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint64_t y = __shfl_up(static_cast<unsigned long long>(x), d);
                if (lane >= d) x = mp_add(x, y);
            }
            const uint64_t ip = __shfl_up(static_cast<unsigned long long>(x), 1);
            P.lane_excl[static_cast<int64_t>(g) * 64 + lane] = lane == 0 ? 0 : mp_mul(ip, S.rinv256[64 - lane]);
            if (lane == 63) P.tile_agg[g] = x;
        } else {
            const TabPut put{str.tab, staged ? &S.stage[wave][lane * 9] : nullptr, seg, len, log2b, bmask};
            if (seg < len || (t == 0 && lane == 0)) {
                // prefix hash at the lane's first character
                uint64_t h = mp_add(mp_mul(P.tile_prefix[g], S.rseg[4 * lane]),
                                    P.lane_excl[static_cast<int64_t>(g) * 64 + lane]);
                if (t == 0 && lane == 0) str.tab[0] = 0;
                if constexpr (TWO && !SMALLB) {
                    if (log2b >= 5)
                        emit_units2<32>(S, cur, h, put);
                    else if (log2b == 4)
                        emit_units2<16>(S, cur, h, put);
                    else
                        emit_units2<8>(S, cur, h, put);
                } else if constexpr (TWO) {
                    if (log2b == 2) {
                        emit_units2<4>(S, cur, h, put);
                    } else {  // b = 1 or 2: single characters
#pragma unroll
                        for (int q = 0; q < NW; ++q)
                            for (int c = 0; c < 32; ++c) {
                                h = mp_add(mp_mul(h, S.rp[1]), (cur[q] >> (2 * c)) & 3u);
                                put(seg + 32 * q + c + 1, h);
                            }
                    }
                } else if constexpr (!SMALLB) {  // b >= 8: 8-bit words
#pragma unroll
                    for (int q = 0; q < NW; ++q) {
                        h = mp_add(mp_mul(h, S.rp[8]), word_hash8(S, cur[q]));
                        put(seg + 8 * (q + 1), h);
                    }
                } else {  // b = 1, 2 or 4: single characters
#pragma unroll
                    for (int q = 0; q < NW; ++q)
                        for (int c = 0; c < 8; ++c) {
                            h = mp_add(mp_mul(h, S.rp[1]), (cur[q] >> (8 * c)) & 0xFFu);
                            put(seg + 8 * q + c + 1, h);
                        }
                }
            }
            if (staged) {
                // entry i (of 64 << lepl) of the tile comes from lane i >> lepl;
                // T index t * (16384 >> log2b) + 1 + i
                __builtin_amdgcn_wave_barrier();
                const int32_t base = t * (kTileChars >> log2b) + 1;
                const int32_t last = len >> log2b;
                for (int32_t k = 0; k < (1 << lepl); ++k) {
                    const int32_t i = k * 64 + lane;
                    const int32_t j = base + i;
                    if (j <= last) str.tab[j] = S.stage[wave][(i >> lepl) * 9 + (i & ((1 << lepl) - 1))];
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if constexpr (TWO) {
#pragma unroll
            for (int k = 0; k < kLaneWords2; ++k) cur[k] = nxt[k];
        }
    }
}

// Block size 32: the emission pass from the block hashes pack_kernel stored
// in T (the characters are not read again).  The hash of the string before a
// tile is that of the string before its chunk (c chunks of 2048 tiles before
// it: sum over them of tot(q) R^(2048 (c - 1 - q)), one term per lane) times
// R^j (j = the tile's place in its chunk) plus the in-chunk prefix that
// after_pack_kernel stored.  Per tile the 512 entries come through the
// wavefront's staging slots, each lane turns the 8 of its 256 characters
// into prefix values, starting from the prefix hash at its first character,
// and they go back to T, 64 consecutive entries per store.  The next tile's
// entries are requested before this tile's arithmetic.  A kernel of its own:
// few registers and little LDS, so that many wavefronts keep loads in flight.
__global__ __launch_bounds__(kPrepThreads) void table_emit_kernel(PrepParams P, const uint64_t* rtab) {
    __shared__ uint64_t stage[kPrepThreads / 64][64 * 9];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int32_t gw = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(blockIdx.x * (kPrepThreads / 64) + (tid >> 6)));
    const int32_t W = static_cast<int32_t>(gridDim.x * (kPrepThreads / 64));
    const int32_t total = P.total_tiles;
    uint64_t* st = &stage[tid >> 6][0];
    const uint64_t r32 = rtab[32];
    const uint64_t rlane = rtab[kRtabRseg + 4 * lane];  // r^(256 lane)
    const int32_t first1 = (P.s[1].tile0 + kScanChunkTiles - 1) / kScanChunkTiles;  // string 1's chunk 0
    uint64_t cur[8], nxt[8];
    // per tile: in-chunk prefix, this lane's term of the string before the
    // chunk and its power, R^j, this lane's in-tile prefix
    uint64_t loc = 0, ct = 0, cw = 0, rj = 0, ex = 0;
    uint64_t nloc = 0, nct = 0, ncw = 0, nrj = 0, nex = 0;
    auto fetch = [&](int32_t g, uint64_t (&e)[8], uint64_t& lo, uint64_t& t, uint64_t& w, uint64_t& r,
                     uint64_t& le) {
        const bool second = g >= P.s[1].tile0;
        const StrSel str(P, second);
        const int32_t tt = g - str.tile0;
        const int32_t base = tt * (kTileChars / 32) + 1;
        const int32_t last = str.len >> 5;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t i = k * 64 + lane;
            e[k] = base + i <= last ? str.tab[base + i] : 0;
        }
        const int32_t c = tt / kScanChunkTiles;
        lo = P.tile_prefix[g];
        t = lane < c ? P.chunk_tot[(second ? first1 : 0) + lane] : 0;
        w = lane < c ? rtab[kRtabRChunk + (c - 1 - lane)] : 0;
        r = rtab[kRtabRTile + (tt - c * kScanChunkTiles)];
        le = P.lane_excl[static_cast<int64_t>(g) * 64 + lane];
    };
    if (gw < total) fetch(gw, cur, loc, ct, cw, rj, ex);
    for (int32_t g = gw; g < total; g += W) {
        if (g + W < total) fetch(g + W, nxt, nloc, nct, ncw, nrj, nex);
        uint64_t cy = mp_mul(ct, cw);
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) cy = mp_add(cy, __shfl_xor(static_cast<unsigned long long>(cy), d));
        const uint64_t pre = mp_add(mp_mul(cy, rj), loc);
        const StrSel str(P, g >= P.s[1].tile0);
        const int32_t t = g - str.tile0;
        const int32_t base = t * (kTileChars / 32) + 1;
        const int32_t last = str.len >> 5;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t i = k * 64 + lane;
            st[(i >> 3) * 9 + (i & 7)] = cur[k];
        }
        if (t == 0 && lane == 0) str.tab[0] = 0;
        __builtin_amdgcn_wave_barrier();
        uint64_t h = mp_add(mp_mul(pre, rlane), ex);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            h = mp_add(mp_mul(h, r32), st[lane * 9 + q]);
            st[lane * 9 + q] = h;
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int32_t i = k * 64 + lane;
            if (base + i <= last) str.tab[base + i] = st[(i >> 3) * 9 + (i & 7)];
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < 8; ++k) cur[k] = nxt[k];
        loc = nloc;
        ct = nct;
        cw = ncw;
        rj = nrj;
        ex = nex;
    }
}

template <bool EMIT, bool SMALLB>
__global__ __launch_bounds__(kPrepThreads) void table_tiles_kernel(PrepParams P, const uint64_t* rtab) {
    __shared__ TableShared S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const bool two = *P.alpha <= 3u;
    const int32_t gw = __builtin_amdgcn_readfirstlane(static_cast<int32_t>(blockIdx.x * (kPrepThreads / 64) + (tid >> 6)));
    const int32_t W = static_cast<int32_t>(gridDim.x * (kPrepThreads / 64));

    // lookup tables and powers, built on the host (kRtab* layout)
    if (two) {
        for (int i = tid; i < 8 * 256; i += kPrepThreads) S.lut32[i >> 8][i & 255] = rtab[kRtabLut32 + i];
    } else {
        for (int i = tid; i < 8 * 256; i += kPrepThreads) S.lut8[i >> 8][i & 255] = rtab[kRtabLut8 + i];
    }
    for (int i = tid; i < 65; i += kPrepThreads) S.rp[i] = rtab[i];
    for (int i = tid; i < 257; i += kPrepThreads) S.rseg[i] = rtab[kRtabRseg + i];
    for (int i = tid; i < 65; i += kPrepThreads) S.rinv256[i] = rtab[kRtabRinv256 + i];
    __syncthreads();
    if (two)
        table_tiles<EMIT, true, SMALLB>(P, S, gw, W, lane, tid >> 6);
    else
        table_tiles<EMIT, false, SMALLB>(P, S, gw, W, lane, tid >> 6);
}

// Pass 2: prefix[u] = h(S[0 .. 16384 u)) from the tile hashes, with
// R = r^16384, in chunks of kScanChunk tiles, one workgroup per chunk of each
// string (the chunks of string 0 first).  Other block sizes, two launches:
// table_total_kernel folds each chunk to its hash (Horner's rule),
// table_scan_kernel takes the hash of the string before its chunk from those
// of the earlier chunks (one term per lane, times R^(kScanChunk d), summed
// over the wavefront) and scans its chunk with it.  At b = 32
// after_pack_kernel scans each chunk from zero and stores its hash, and the
// emission pass adds the string before the chunk.  Within a chunk each thread folds 8 consecutive tiles,
// the threads' values are combined by inclusive scans under
// x(l) = x(l - d) R^(8 d) + x(l) within each wavefront and then over the
// wavefronts.  The last chunk is zero-padded: its hash is never used and
// the padding only follows the last real tile.  Powers of R come from the
// host.
constexpr int kScanThreads = 256, kScanPer = 8, kScanChunk = kScanThreads * kScanPer;  // 2048 tiles
static_assert(kScanChunk == kScanChunkTiles, "scan chunk size");
static_assert(kScanThreads == kPrepThreads, "after_pack_kernel folds chunks with the pack block size");
constexpr int kScanWaves = kScanThreads / 64;

struct ScanChunk {
    int32_t tile0;  // first tile of the string
    int32_t c;      // chunk within the string
    int32_t cn;     // real tiles in the chunk
    int32_t first;  // workgroup of the string's chunk 0
};

__device__ __forceinline__ ScanChunk scan_chunk(const PrepParams& P) {
    const int32_t t1 = P.s[1].tile0;
    const int32_t c0 = (t1 + kScanChunk - 1) / kScanChunk;
    const bool second = static_cast<int32_t>(blockIdx.x) >= c0;
    ScanChunk k;
    k.tile0 = second ? t1 : 0;
    k.first = second ? c0 : 0;
    k.c = static_cast<int32_t>(blockIdx.x) - k.first;
    const int32_t tiles = second ? P.total_tiles - t1 : t1;
    k.cn = imin32(kScanChunk, tiles - k.c * kScanChunk);
    return k;
}

// Horner over the thread's tiles and the inclusive scan over the wavefront.
__device__ __forceinline__ uint64_t scan_fold(const uint64_t* agg, int32_t cn, const uint64_t* rtab, int tid,
                                              uint64_t (&a)[kScanPer]) {
    const uint64_t R = rtab[kRtabR + 1];
    const uint64_t* R8p = rtab + kRtabR8pow2;  // R^(8 * 2^j)
    const int lane = tid & 63;
    uint64_t h = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        const int32_t i = kScanPer * tid + j;
        a[j] = i < cn ? agg[i] : 0;
        h = mp_add(mp_mul(h, R), a[j]);
    }
#pragma unroll
    for (int d = 1, j = 0; d < 64; d <<= 1, ++j) {
        const uint64_t y = __shfl_up(static_cast<unsigned long long>(h), d);
        if (lane >= d) h = mp_add(mp_mul(y, R8p[j]), h);
    }
    return h;
}

__device__ __forceinline__ void chunk_total(const PrepParams& P, const uint64_t* rtab) {
    __shared__ uint64_t wtot[kScanWaves];
    const int tid = threadIdx.x;
    const ScanChunk k = scan_chunk(P);
    uint64_t a[kScanPer];
    const uint64_t h = scan_fold(P.tile_agg + k.tile0 + k.c * kScanChunk, k.cn, rtab, tid, a);
    if ((tid & 63) == 63) wtot[tid >> 6] = h;
    __syncthreads();
    if (tid == 0) {
        const uint64_t Rw = rtab[kRtabR8pow2 + 6];  // R^512: tiles per wavefront
        uint64_t x = 0;
        for (int w = 0; w < kScanWaves; ++w) x = mp_add(mp_mul(x, Rw), wtot[w]);
        P.chunk_tot[blockIdx.x] = x;
    }
}

__global__ __launch_bounds__(kScanThreads) void table_total_kernel(PrepParams P, const uint64_t* rtab) {
    chunk_total(P, rtab);
}

// The scan of one chunk (the workgroup's) to the prefix hash before each of
// its tiles (tile_prefix).  CARRY: the prefix includes the string before the
// chunk, taken from the totals of the earlier chunks (complete before this
// launch).  Otherwise the values start from zero at the chunk (the emission
// pass adds the string before the chunk) and the chunk's total is stored too.
template <bool CARRY>
__device__ __forceinline__ void scan_chunk_tiles(const PrepParams& P, const uint64_t* rtab) {
    __shared__ uint64_t buf[kScanChunk];
    __shared__ uint64_t wtot[kScanWaves];
    __shared__ uint64_t wpre[kScanWaves];  // prefix before each wavefront's tiles
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const ScanChunk k = scan_chunk(P);
    const uint64_t R = rtab[kRtabR + 1];
    const uint64_t* R8p = rtab + kRtabR8pow2;
    const uint64_t Rlane = rtab[kRtabR8lane + lane];  // R^(8 (lane + 1))
    uint64_t a[kScanPer];
    const uint64_t h = scan_fold(P.tile_agg + k.tile0 + k.c * kScanChunk, k.cn, rtab, tid, a);
    if (lane == 63) wtot[wave] = h;
    __syncthreads();
    if (wave == 0) {
        // the string before the chunk: sum over earlier chunks i of
        // tot(i) R^(kScanChunk (c - 1 - i)) (at most 64 chunks per string)
        uint64_t cy = 0;
        if constexpr (CARRY) {
            cy = lane < k.c ? mp_mul(P.chunk_tot[k.first + lane], rtab[kRtabRChunk + (k.c - 1 - lane)]) : 0;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) cy = mp_add(cy, __shfl_xor(static_cast<unsigned long long>(cy), d));
        }
        // over the wavefronts (512 tiles each), the carry ahead of the first
        uint64_t x = lane < kScanWaves ? wtot[lane] : 0;
        if (lane == 0) x = mp_add(mp_mul(cy, R8p[6]), x);
#pragma unroll
        for (int d = 1, j = 6; d < kScanWaves; d <<= 1, ++j) {
            const uint64_t y = __shfl_up(static_cast<unsigned long long>(x), d);
            if (lane >= d) x = mp_add(mp_mul(y, R8p[j]), x);
        }
        const uint64_t xp = __shfl_up(static_cast<unsigned long long>(x), 1);
        if (lane < kScanWaves) wpre[lane] = lane == 0 ? cy : xp;
        // without the carry the last wavefront's inclusive value is the
        // chunk's hash (the padding of a last chunk is never used)
        if constexpr (!CARRY) {
            if (lane == kScanWaves - 1) P.chunk_tot[blockIdx.x] = x;
        }
    }
    __syncthreads();
    const uint64_t pw = wpre[wave];
    const uint64_t incl = mp_add(mp_mul(pw, Rlane), h);
    const uint64_t ex = __shfl_up(static_cast<unsigned long long>(incl), 1);
    uint64_t p = lane == 0 ? pw : ex;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
        buf[kScanPer * tid + j] = p;
        p = mp_add(mp_mul(p, R), a[j]);
    }
    __syncthreads();
    uint64_t* pre = P.tile_prefix + k.tile0 + k.c * kScanChunk;
    for (int i = tid; i < k.cn; i += kScanThreads) pre[i] = buf[i];
}

__global__ __launch_bounds__(kScanThreads) void table_scan_kernel(PrepParams P, const uint64_t* rtab) {
    scan_chunk_tiles<true>(P, rtab);
}

// Second pass, once the pair's alphabet is known: the layout it is read in
// (2-bit when no character is above 3; else 4-bit when none is above 15 and
// the pair has a 4-bit layout; else 8-bit) for the chunks the first pass
// wrote in a narrower one (chunk classes below the layout's).  Nothing to do
// when the 2-bit words are complete or no chunk needs it.  Each wavefront
// reads the classes of 64 chunks at a time.
__device__ __forceinline__ void rest_pass(const PrepParams& P, uint32_t alpha, uint32_t classes) {
    if (alpha <= 3u || P.force8) return;
    const bool four = alpha <= 15u && P.s[0].w4 && P.s[1].w4;
    const uint32_t below = four ? 1u : 2u;  // classes to rewrite: those below this
    if ((classes & ((1u << below) - 1u)) == 0u) return;
    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t nwaves = static_cast<int32_t>((gridDim.x * blockDim.x) >> 6);
    const int32_t total = P.total_tiles * kTileChunks;
    const int32_t split = P.s[1].tile0 * kTileChunks;
    for (int32_t g0 = wave * 64; g0 < total; g0 += nwaves * 64) {
        uint64_t todo = ballot(g0 + lane < total && P.chunk_big[g0 + lane] < below);
        while (todo) {
            const int32_t g = g0 + ctz64(todo);
            todo &= todo - 1;
            const StrSel str(P, g >= split);
            const int32_t c = g - str.tile0 * kTileChunks;
            const int32_t seg_start = c * kChunkChars + lane * kSegChars;
            if (four) {
                uint64_t* dst = str.w4 + static_cast<int64_t>(c) * kChunkWords4 + lane * 4;
                for (int k = 0; k < 4; ++k) {
                    uint64_t v = 0;
                    for (int j = 0; j < 16; ++j) {
                        const int32_t p = seg_start + 16 * k + j;
                        if (p < str.len) v |= static_cast<uint64_t>(str.raw[p] & 0xFu) << (4 * j);
                    }
                    dst[k] = v;
                }
            } else {
                uint64_t* dst = str.w8 + static_cast<int64_t>(c) * kChunkWords8 + lane * 8;
                for (int k = 0; k < 8; ++k) {
                    uint64_t v = 0;
                    for (int j = 0; j < 8; ++j) {
                        const int32_t p = seg_start + 8 * k + j;
                        if (p < str.len) v |= static_cast<uint64_t>(str.raw[p]) << (8 * j);
                    }
                    dst[k] = v;
                }
            }
        }
    }
}

// The kernel after pack_kernel: every workgroup reduces the pack kernel's
// per-workgroup slots to the pair's alphabet OR and chunk classes (workgroup
// 0 stores them for the later kernels and the host), runs the rest pass, and
// with block hashes taken by the pack kernel the first scan_chunks workgroups
// also scan their chunk of tile hashes from zero and store its total; the
// emission pass adds the part of the string before the chunk.
__global__ __launch_bounds__(kPrepThreads) void after_pack_kernel(PrepParams P, const uint64_t* rtab) {
    __shared__ uint32_t red[kPrepThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63;
    uint32_t v = 0;
    for (int i = tid; i < P.pack_grid; i += kPrepThreads) v |= P.wg_or[i];
    for (int s = 32; s > 0; s >>= 1) v |= __shfl_xor(v, s);
    if (lane == 0) red[tid >> 6] = v;
    __syncthreads();
    uint32_t o = 0;
    for (int w = 0; w < kPrepThreads / 64; ++w) o |= red[w];
    const uint32_t alpha = o & 0xFFu, classes = o >> 8;
    if (blockIdx.x == 0 && tid == 0) {
        *P.alpha = alpha;
        *P.packed_any = classes;
    }
    rest_pass(P, alpha, classes);
    if (P.fuse_table && static_cast<int32_t>(blockIdx.x) < P.scan_chunks) scan_chunk_tiles<false>(P, rtab);
}

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

hipError_t launch_pack(const PrepParams& pp, int grid, hipStream_t s) {
    if (pp.nt_copy)
        hipLaunchKernelGGL(pack_kernel<true>, dim3(grid), dim3(kPrepThreads), 0, s, pp);
    else
        hipLaunchKernelGGL(pack_kernel<false>, dim3(grid), dim3(kPrepThreads), 0, s, pp);
    return hipGetLastError();
}

hipError_t launch_table(const PrepParams& pp, int grid, hipStream_t s) {
    // one tile per wavefront at a time
    const int need = (pp.total_tiles + kPrepThreads / 64 - 1) / (kPrepThreads / 64);
    if (grid > need) grid = need;
    if (grid < 1) grid = 1;
    hipError_t e;
    if (!pp.fuse_table) {  // else pack_kernel did the first pass
        hipLaunchKernelGGL((table_tiles_kernel<false, false>), dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int chunks = pp.scan_chunks;
    if (!pp.fuse_table) {  // else after_pack_kernel folded the chunks
        hipLaunchKernelGGL(table_total_kernel, dim3(chunks), dim3(kScanThreads), 0, s, pp, pp.rtab);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!pp.fuse_table) {  // else after_pack_kernel scanned each chunk from zero
        hipLaunchKernelGGL(table_scan_kernel, dim3(chunks), dim3(kScanThreads), 0, s, pp, pp.rtab);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (pp.fuse_table)
        hipLaunchKernelGGL(table_emit_kernel, dim3(2 * grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    else if (pp.log2b <= 2)
        hipLaunchKernelGGL((table_tiles_kernel<true, true>), dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    else
        hipLaunchKernelGGL((table_tiles_kernel<true, false>), dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    return hipGetLastError();
}

hipError_t launch_after_pack(const PrepParams& pp, int grid, hipStream_t s) {
    if (pp.fuse_table && grid < pp.scan_chunks) grid = pp.scan_chunks;
    hipLaunchKernelGGL(after_pack_kernel, dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ed
