// Prepare a pair: the input bytes of both strings are read once.
//   pack_kernel   streaming, one wavefront per 4096-character chunk, no LDS:
//                 alphabet detection (bitwise OR of every character; 2-bit
//                 packing is possible when the OR is <= 3), 2-bit packing of
//                 every chunk without a character > 3, and an 8-bit copy of
//                 every chunk with one (the rest of the copy, when the pair
//                 cannot be packed, is written by copy8_rest_kernel);
//   table_*       (hash engine) prefix table T[j] = h(S[0..jb)) mod 2^61-1
//                 (sections 3.2 and 3.3, Algorithm 2 "Build") from the packed
//                 words (or the 8-bit copy): block hashes from LDS lookup
//                 tables (h is linear in the characters), combined under the
//                 concatenation h(S1 S2) = h(S1) r^|S2| + h(S2) within each
//                 tile, across tiles by a separate scan of the tile hashes.
#include "device.h"

namespace ed {

namespace {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

struct PrepShared {
    // one of the two, by the pair's packing (halves the LDS per workgroup)
    union {
        uint64_t lut32[8][256];  // packed byte k of a 2-bit word: sum_j c_j r^(31-4k-j)
        uint64_t lut8[8][256];   // byte k of an 8-char word: v r^(7-k)
    };
    uint64_t lut4[256];      // packed byte (4 chars): c0 r^3 + c1 r^2 + c2 r + c3
    uint64_t rp[65];         // r^p
    uint64_t rseg[257];      // r^(64 k)
    uint64_t wsum[kPrepThreads / 64];
};

// The fields of one of the two strings, chosen by a uniform flag: a select
// between two kernel arguments (scalar registers), not an indexed load.
struct StrSel {
    const uint8_t* raw;
    uint64_t* w2;
    uint64_t* w8;
    uint64_t* tab;
    int32_t len;
    int32_t tile0;
    __device__ __forceinline__ StrSel(const PrepParams& P, bool second)
        : raw(second ? P.s[1].raw : P.s[0].raw),
          w2(second ? P.s[1].w2 : P.s[0].w2),
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

// Hash of the 64 characters of one segment, processed in units of U chars
// (U divides b); when EMIT, writes T at every block end inside the segment.
// `h` enters as the prefix hash at the segment start.
template <bool EMIT>
__device__ __forceinline__ uint64_t seg_pass(const PrepShared& S, const uint32_t (&dw)[16],
                                             const uint64_t (&pk)[2], bool big, int32_t log2b,
                                             uint64_t h, int32_t seg_start, int32_t len,
                                             uint64_t* tab) {
    const int32_t bmask = (1 << log2b) - 1;
    auto emit = [&](int32_t pos) {
        if (EMIT) {
            const int32_t e = seg_start + pos;
            if ((e & bmask) == 0 && e <= len) tab[e >> log2b] = h;
        }
    };
    if (!big) {
        if (log2b >= 5) {  // units of 32 characters: one packed word
            for (int w = 0; w < 2; ++w) {
                uint64_t s = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) s += S.lut32[k][(pk[w] >> (8 * k)) & 0xFF];
                h = mp_add(mp_mul(h, S.rp[32]), mp_fold(s));
                emit(32 * (w + 1));
            }
        } else if (log2b >= 2) {  // units of 4 characters: one packed byte
            for (int u = 0; u < 16; ++u) {
                const uint32_t byte = static_cast<uint32_t>(pk[u >> 3] >> (8 * (u & 7))) & 0xFFu;
                h = mp_add(mp_mul(h, S.rp[4]), S.lut4[byte]);
                emit(4 * (u + 1));
            }
        } else {  // single characters
            for (int c = 0; c < 64; ++c) {
                const uint64_t ch = (pk[c >> 5] >> (2 * (c & 31))) & 3u;
                h = mp_add(mp_mul(h, S.rp[1]), ch);
                emit(c + 1);
            }
        }
    } else {
        if (log2b >= 3) {  // units of 8 characters: one 8-bit word
            for (int w = 0; w < 8; ++w) {
                uint64_t s = 0;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t v = (dw[2 * w + (k >> 2)] >> (8 * (k & 3))) & 0xFFu;
                    s += S.lut8[k][v];
                }
                h = mp_add(mp_mul(h, S.rp[8]), mp_fold(s));
                emit(8 * (w + 1));
            }
        } else {
            for (int c = 0; c < 64; ++c) {
                const uint64_t ch = (dw[c >> 2] >> (8 * (c & 3))) & 0xFFu;
                h = mp_add(mp_mul(h, S.rp[1]), ch);
                emit(c + 1);
            }
        }
    }
    return h;
}

__device__ __forceinline__ uint64_t wave_sum_mod(uint64_t v) {
    for (int o = 32; o > 0; o >>= 1) v = mp_add(v, __shfl_xor(static_cast<unsigned long long>(v), o));
    return v;
}

}  // namespace

__global__ void prep_clear_kernel(PrepParams P) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i == 0) *P.alpha = 0u;
}

// Streaming pass: wavefront w takes chunks w, w + W, ... (W wavefronts in the
// grid).  Every load and store instruction covers a contiguous range: lane l
// holds the 16-character pieces at chunk offsets 1024 k + 16 l (k = 0..3),
// packs each into 32 bits (the low or high half of a packed word) and writes
// them at 32-bit index 64 k + l of the chunk.  Chunk slots past the end of a
// string are written as zeros (padding the last tile).
__global__ __launch_bounds__(kPrepThreads) void pack_kernel(PrepParams P) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t nwaves = static_cast<int32_t>((gridDim.x * blockDim.x) >> 6);
    const int32_t total = P.total_tiles * kTileChunks;
    const int32_t split = P.s[1].tile0 * kTileChunks;
    uint32_t orr = 0;
    for (int32_t g = wave; g < total; g += nwaves) {
        const StrSel str(P, g >= split);
        const int32_t c = g - str.tile0 * kTileChunks;
        const int32_t cbase = c * kChunkChars;
        const int32_t len = str.len;
        u32x4 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int32_t pos = cbase + k * 1024 + lane * 16;
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
        uint32_t o = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) o |= v[k].x | v[k].y | v[k].z | v[k].w;
        orr |= o;
        const bool big = ballot((o & 0xFCFCFCFCu) != 0u) != 0;
        if (!big) {
            uint32_t* dst = reinterpret_cast<uint32_t*>(str.w2 + static_cast<int64_t>(c) * kChunkWords2);
#pragma unroll
            for (int k = 0; k < 4; ++k)
                dst[k * 64 + lane] = pack_dword(v[k].x) | (pack_dword(v[k].y) << 8) | (pack_dword(v[k].z) << 16) |
                                     (pack_dword(v[k].w) << 24);
        }
        if (big || P.force8) {
            u32x4* dst = reinterpret_cast<u32x4*>(str.w8 + static_cast<int64_t>(c) * kChunkWords8);
#pragma unroll
            for (int k = 0; k < 4; ++k) dst[k * 64 + lane] = v[k];
        }
        if (lane == 0) P.chunk_big[g] = big ? 1 : 0;
    }
    // one atomic per workgroup at most, and none when the bits are already
    // there: atomics on one address from every wavefront serialise
    __shared__ uint32_t wor[kPrepThreads / 64];
    orr |= orr >> 16;
    orr |= orr >> 8;
    orr &= 0xFFu;
    for (int s = 32; s > 0; s >>= 1) orr |= __shfl_xor(orr, s);
    if (lane == 0) wor[threadIdx.x >> 6] = orr;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t o = 0;
        for (int w = 0; w < kPrepThreads / 64; ++w) o |= wor[w];
        const uint32_t cur = __hip_atomic_load(P.alpha, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if ((cur | o) != cur) atomicOr(P.alpha, o);
    }
}

// Prefix tables of both strings (hash engine), after pack_kernel (and
// copy8_rest_kernel), in three passes with no shared counter: tiles of 16384
// characters are assigned statically to workgroups.
//   table_tiles_kernel<false>  hash of every tile -> tile_agg[g]
//   table_scan_kernel          per string, prefix hash before every tile ->
//                              tile_prefix[g] (Horner over tiles, R = r^16384)
//   table_tiles_kernel<true>   block-scan of each tile from its prefix and
//                              T[j] at every block end inside it
// The characters come from the 2-bit words when the pair is packable, from the
// 8-bit copy otherwise.
template <bool EMIT>
__global__ __launch_bounds__(kPrepThreads) void table_tiles_kernel(PrepParams P, const uint64_t* rtab) {
    __shared__ PrepShared S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const bool two = *P.alpha <= 3u;

    // rtab: r^0..r^64 | r^(64k), k = 0..256 | R^d, d = 0..64
    for (int i = tid; i < 65; i += kPrepThreads) S.rp[i] = rtab[i];
    for (int i = tid; i < 257; i += kPrepThreads) S.rseg[i] = rtab[65 + i];
    __syncthreads();
    for (int e = tid; e < 8 * 256; e += kPrepThreads) {
        const int k = e >> 8, v = e & 255;
        if (two) {
            uint64_t h = 0;
            for (int j = 0; j < 4; ++j)
                h = mp_add(h, mp_mul(static_cast<uint64_t>((v >> (2 * j)) & 3), S.rp[31 - 4 * k - j]));
            S.lut32[k][v] = h;
        } else {
            S.lut8[k][v] = mp_mul(static_cast<uint64_t>(v), S.rp[7 - k]);
        }
    }
    for (int v = tid; v < 256; v += kPrepThreads) {
        uint64_t h = 0;
        for (int j = 0; j < 4; ++j)
            h = mp_add(h, mp_mul(static_cast<uint64_t>((v >> (2 * j)) & 3), S.rp[3 - j]));
        S.lut4[v] = h;
    }

    for (int32_t g = blockIdx.x; g < P.total_tiles; g += gridDim.x) {
        __syncthreads();  // tables ready; wsum of the previous tile consumed
        const StrSel str(P, g >= P.s[1].tile0);
        const int32_t t = g - str.tile0;
        const int32_t seg_start = t * kTileChars + tid * kSegChars;
        const int32_t len = str.len;
        const bool big = !two;

        // the 64 characters of this thread (zero past the string)
        uint32_t dw[16];
        uint64_t pk[2];
        if (two) {
            const u32x4 v = *reinterpret_cast<const u32x4*>(str.w2 + static_cast<int64_t>(t) * kTileWords2 + tid * 2);
            pk[0] = static_cast<uint64_t>(v.x) | (static_cast<uint64_t>(v.y) << 32);
            pk[1] = static_cast<uint64_t>(v.z) | (static_cast<uint64_t>(v.w) << 32);
#pragma unroll
            for (int k = 0; k < 16; ++k) dw[k] = 0;
        } else {
            const u32x4* src = reinterpret_cast<const u32x4*>(str.w8 + static_cast<int64_t>(t) * kTileWords8 + tid * 8);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const u32x4 v = src[k];
                dw[4 * k + 0] = v.x;
                dw[4 * k + 1] = v.y;
                dw[4 * k + 2] = v.z;
                dw[4 * k + 3] = v.w;
            }
            pk[0] = pk[1] = 0;
        }

        // ---- segment hash, block-scan within the tile ----
        const uint64_t hseg = seg_pass<false>(S, dw, pk, big, P.log2b, 0, seg_start, len, nullptr);
        uint64_t x = hseg;  // inclusive over the wave, Hillis-Steele
        for (int d = 1; d < 64; d <<= 1) {
            const uint64_t y = __shfl_up(static_cast<unsigned long long>(x), d);
            if (lane >= d) x = mp_add(mp_mul(y, S.rseg[d]), x);
        }
        if (lane == 63) S.wsum[wave] = x;
        __syncthreads();
        if (!EMIT) {
            if (tid == 0) {
                uint64_t agg = 0;
                for (int v = 0; v < kPrepThreads / 64; ++v) agg = mp_add(mp_mul(agg, S.rseg[64]), S.wsum[v]);
                P.tile_agg[g] = agg;
            }
        } else {
            uint64_t pre = 0;  // hash of the waves before this one
            for (int v = 0; v < wave; ++v) pre = mp_add(mp_mul(pre, S.rseg[64]), S.wsum[v]);
            const uint64_t xprev = __shfl_up(static_cast<unsigned long long>(x), 1);
            const uint64_t excl_thread = lane == 0 ? pre : mp_add(mp_mul(pre, S.rseg[lane]), xprev);
            // emit T at block ends: prefix at segment start, then the units
            const uint64_t tp = P.tile_prefix[g];
            const uint64_t hstart = mp_add(mp_mul(tp, S.rseg[tid]), excl_thread);
            if (seg_start < len) seg_pass<true>(S, dw, pk, big, P.log2b, hstart, seg_start, len, str.tab);
            if (t == 0 && tid == 0) str.tab[0] = 0;
        }
    }
}

// Pass 2: one workgroup per string.  prefix[t] = h(S[0 .. 16384 t)) from the
// tile hashes by Horner's rule with R = r^16384: each thread folds a run of
// consecutive tiles, the runs are combined by a scan under
// (a, na) . (b, nb) = (a R^nb + b, na + nb), and each thread writes the
// prefixes of its run.
__global__ __launch_bounds__(1024) void table_scan_kernel(PrepParams P, const uint64_t* rtab) {
    __shared__ uint64_t Rp[32];  // R^(2^k)
    __shared__ uint64_t hs[1024];
    __shared__ int32_t ns[1024];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const StrSel str(P, blockIdx.x == 1);
    const int32_t tiles = (blockIdx.x == 1 ? P.total_tiles : P.s[1].tile0) - str.tile0;
    if (tid == 0) {
        Rp[0] = rtab[65 + 257 + 1];
        for (int k = 1; k < 32; ++k) Rp[k] = mp_mul(Rp[k - 1], Rp[k - 1]);
    }
    __syncthreads();
    auto powR = [&](int32_t e) {
        uint64_t r = 1;
        for (int k = 0; e; ++k, e >>= 1)
            if (e & 1) r = mp_mul(r, Rp[k]);
        return r;
    };
    const int32_t blk = (tiles + nthr - 1) / nthr;
    const int32_t lo = imin32(tiles, tid * blk), hi = imin32(tiles, lo + blk);
    const uint64_t R = Rp[0];
    const uint64_t* agg = P.tile_agg + str.tile0;
    uint64_t h = 0;
    for (int32_t u = lo; u < hi; ++u) h = mp_add(mp_mul(h, R), agg[u]);
    int32_t n = hi - lo;
    // inclusive scan over threads (Hillis-Steele through LDS)
    for (int d = 1; d < nthr; d <<= 1) {
        hs[tid] = h;
        ns[tid] = n;
        __syncthreads();
        if (tid >= d) {
            const uint64_t a = hs[tid - d];
            const int32_t na = ns[tid - d];
            h = mp_add(mp_mul(a, powR(n)), h);
            n += na;
        }
        __syncthreads();
    }
    hs[tid] = h;
    __syncthreads();
    uint64_t p = tid == 0 ? 0 : hs[tid - 1];
    uint64_t* pre = P.tile_prefix + str.tile0;
    for (int32_t u = lo; u < hi; ++u) {
        pre[u] = p;
        p = mp_add(mp_mul(p, R), agg[u]);
    }
}

// Second pass for pairs that cannot be packed: 8-bit copy of the chunks the
// first pass packed instead.  Exits at once when the pair is packable.
__global__ __launch_bounds__(kPrepThreads) void copy8_rest_kernel(PrepParams P) {
    const uint32_t alpha = *P.alpha;
    if (alpha <= 3u || P.force8) return;
    const int lane = threadIdx.x & 63;
    const int32_t wave = __builtin_amdgcn_readfirstlane(static_cast<int32_t>((blockIdx.x * blockDim.x + threadIdx.x) >> 6));
    const int32_t nwaves = static_cast<int32_t>((gridDim.x * blockDim.x) >> 6);
    const int32_t total = P.total_tiles * kTileChunks;
    const int32_t split = P.s[1].tile0 * kTileChunks;
    for (int32_t g = wave; g < total; g += nwaves) {
        if (P.chunk_big[g]) continue;
        const StrSel str(P, g >= split);
        const int32_t c = g - str.tile0 * kTileChunks;
        const int32_t seg_start = c * kChunkChars + lane * kSegChars;
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

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

__global__ void fill_u32_kernel(unsigned int* p, int64_t n, unsigned int v) {
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
         i += static_cast<int64_t>(gridDim.x) * blockDim.x)
        p[i] = v;
}

hipError_t launch_prep_clear(const PrepParams& pp, hipStream_t s) {
    const int blocks = (pp.total_tiles + 255) / 256 + 1;
    hipLaunchKernelGGL(prep_clear_kernel, dim3(blocks), dim3(256), 0, s, pp);
    return hipGetLastError();
}

hipError_t launch_pack(const PrepParams& pp, int grid, hipStream_t s) {
    hipLaunchKernelGGL(pack_kernel, dim3(grid), dim3(kPrepThreads), 0, s, pp);
    return hipGetLastError();
}

hipError_t launch_table(const PrepParams& pp, int grid, hipStream_t s) {
    hipLaunchKernelGGL(table_tiles_kernel<false>, dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(table_scan_kernel, dim3(2), dim3(1024), 0, s, pp, pp.rtab);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(table_tiles_kernel<true>, dim3(grid), dim3(kPrepThreads), 0, s, pp, pp.rtab);
    return hipGetLastError();
}

hipError_t launch_copy8_rest(const PrepParams& pp, int grid, hipStream_t s) {
    hipLaunchKernelGGL(copy8_rest_kernel, dim3(grid), dim3(kPrepThreads), 0, s, pp);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_i32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned int* p, int64_t n, unsigned int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

}  // namespace ed
