// Structures shared by the host library and the kernels of libed.so.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ed {

constexpr int32_t kNone = -(1 << 30);  // "no cell on this diagonal"
constexpr uint64_t kP = 0x1FFFFFFFFFFFFFFFull;  // 2^61 - 1

// Frontier kernels: threads per workgroup.
constexpr int kFrontierThreads = 1024;
// Largest number of rounds one workgroup keeps in LDS (two int32 rows of
// 2*kLdsRoundsMax + 5 entries each).
constexpr int kLdsRoundsMax = 4096;
constexpr int kLdsRowLen = 2 * kLdsRoundsMax + 5;

// Prepare kernel: 256 threads x 64 characters per tile.
constexpr int kPrepThreads = 256;
constexpr int kSegChars = 64;
constexpr int kTileChars = kPrepThreads * kSegChars;  // 16384
constexpr int kTileWords2 = kTileChars / 32;          // 512 packed words per tile
constexpr int kTileWords4 = kTileChars / 16;          // 1024 4-bit words per tile
constexpr int kTileWords8 = kTileChars / 8;           // 2048 byte-words per tile
// Streaming pass: one wavefront per chunk of 64 lanes x 64 characters.
constexpr int kChunkChars = 64 * kSegChars;           // 4096
constexpr int kTileChunks = kTileChars / kChunkChars;  // 4
constexpr int kChunkWords2 = kChunkChars / 32;        // 128
constexpr int kChunkWords4 = kChunkChars / 16;        // 256
constexpr int kChunkWords8 = kChunkChars / 8;         // 512
// Words of zero padding after the last tile of every packed buffer.
constexpr int kPadWords = 256;
// Tiles per chunk of the scan of the tile hashes (one workgroup per chunk).
constexpr int kScanChunkTiles = 2048;


// One string as the kernels see it.
struct StrDev {
    const uint64_t* w2;   // 2-bit packed words (complete when the pair is packable)
    const uint64_t* w4;   // 4-bit words (direct engine; complete when every character is below 16
                          // and above 3 somewhere), or nullptr
    const uint64_t* w8;   // 8-bit copy as words (written when not packable)
    const uint64_t* tab;  // prefix table (hash engine) or nullptr
    int32_t len;
    int32_t pad_;
};

// One pair.
struct PairDev {
    StrDev a, b;
    const uint32_t* alpha;  // device word: OR of all characters of A and B (+ force bits)
    int32_t log2b;          // hash block size b = 1 << log2b
    int32_t force8;         // 1 = use the 8-bit copies even if packable
};

// Hash parameters shared by build and query.
struct HashDev {
    uint64_t r;             // base
    const uint64_t* pow0;   // r^a, a < 65536
    const uint64_t* pow1;   // r^(65536 a), a < 65536
    const uint64_t* rtab;   // lookup tables and powers (kRtab* layout)
};

// Per-run counters (device), summed with atomics at kernel exit.
struct CountersDev {
    unsigned long long updates;
    unsigned long long lcp_chars;
    unsigned long long wave_lcps;
    unsigned long long grid_lcps;    // LCPs answered by the grid tier (ed_debug_lcp engine 3)
    unsigned long long wg_lcps;      // LCPs extended by a whole workgroup
    unsigned long long hash_queries;
    unsigned long long hash_probes;
    unsigned long long hash_ne_len;  // sum of L - 1 over the deciding "unequal" hash verdicts
    unsigned long long collisions;
};

// Control block of one single-pair launch (device memory).
struct FrontierCtl {
    unsigned int release;   // device-wide barrier: epoch released by workgroup 0
    int32_t phase;          // 0: one workgroup; 1: grid-wide
    int32_t phase_t;        // round reached when going grid-wide
    int32_t found_t;        // smallest round whose frontier reaches (n, m); INT32_MAX before
    int32_t status;         // 0 running, 1 done, 2 k_max reached, 3 out of capacity, 4 error
    int32_t result_t;       // reported rounds (k, k_max + 1, or last round at capacity)
    int32_t wbuf;           // which buffer (0/1) holds the last frontier
    int32_t pad_;
    uint64_t clk_begin;     // s_memrealtime (100 MHz) at kernel start
    uint64_t clk_switch;    // ... when the one-workgroup phase ended
    uint64_t clk_end;       // ... at kernel end
};

// Device-wide barrier flags: one 128-byte line per workgroup.
constexpr int kBarStride = 32;  // uint32 per line
constexpr int kMaxGrid = 1024;
// LCPs queued per round for the workgroup or grid tier
constexpr int kGridJobs = 128;

struct FrontierParams {
    PairDev p;
    HashDev h;
    int32_t* f0;       // global frontier rows, 2K+5 entries each, diagonal i at [i + K + 2]
    int32_t* f1;
    int32_t K;         // supports rounds t <= K
    int32_t t0;        // first round already computed (resume: f_t0 is in f0)
    int32_t kmax;      // -1 = none
    int32_t lds_rounds;  // rounds run by workgroup 0 alone, rows in LDS (<= kLdsRoundsMax)
    int32_t block_rounds;  // grid-wide phase: rounds between device-wide barriers
    int32_t engine;
    int32_t lane_words;
    int32_t grid_rounds;  // 1: the first rounds may run on every workgroup (direct engine)
    int32_t hash_first;   // 1: hash engine, slides past the lane stage go to the hash search at once
    int32_t pad2_;
    uint64_t wait_ticks;  // a wait on another workgroup or wavefront gives up after this many
                          // s_memrealtime ticks (100 MHz) and the launch ends with status 4
    FrontierCtl* ctl;
    unsigned int* bar;  // kMaxGrid lines of kBarStride uint32
    int32_t* gpart;     // grid rounds: 2 x kGridJobs x kMaxGrid per-workgroup first mismatches
    // optional per-round rows (device) from round dump_t0 on (a resumed launch
    // dumps from its start round): with dump_w = 0 and no dump_rows every
    // diagonal, row t at t*t - dump_t0*dump_t0 and diagonal i at + t + i;
    // otherwise the rows of the KeepLayout {dump_cone, dump_t0, dump_lo,
    // dump_w, dump_iend, dump_kend}.  Rows past dump_cap entries are dropped.
    int32_t* dump;
    int64_t dump_cap;
    int32_t dump_cone;
    int32_t dump_t0;
    int32_t dump_lo;
    int32_t dump_w;
    int32_t dump_iend;
    int32_t dump_kend;
    CountersDev* counters;
};

// Work-stealing launch over (pair, diagonal-chunk) tasks (batch and serving).
// State of one pair in device memory; it persists across launches.
struct TaskPair {
    PairDev p;
    int32_t* f0;          // global rows, 2K+5 entries each, diagonal i at [i + K + 2]
    int32_t* f1;
    int32_t K;            // rows support rounds t <= K (0: no rows)
    int32_t t;            // rounds completed
    int32_t cur;          // row holding f_t (0: f0, 1: f1)
    int32_t status;       // 0 active, 1 done, 2 k_max reached, 3 out of rows, 4 error, 5 round budget used
    int32_t result;       // k (status 1) or k_max + 1 (status 2)
    int32_t t_limit;      // stop with status 5 when t reaches it (INT32_MAX: none)
    int32_t H, T;         // current super-step: rounds t -> T = t + H
    int32_t chunk;        // diagonals per chunk task
    int32_t nchunks;
    int32_t chunks_left;  // chunk tasks of the super-step not finished yet
    int32_t found_t;      // smallest round reaching (n, m) in the super-step (INT32_MAX: none)
    int32_t kmax;         // stop after round kmax with result kmax + 1 (-1: none)
    int32_t pad_;
};

// Task encoding (always >= 0; -1 means "no task"): pair index in the low 32
// bits; the high 32 bits hold 0 for a whole-pair task, chunk index + 1 for a
// chunk task.
constexpr uint32_t kTaskSolo = 0u;

struct TaskParams {
    TaskPair* pairs;
    int32_t count;
    int32_t kmax;           // -1 = none
    int32_t engine;
    int32_t lane_words;
    int32_t solo_rounds;    // a whole-pair task runs rounds up to this t (LDS rows)
    int32_t block_rounds;   // rounds per chunk super-step (H)
    int32_t chunk_diags;    // diagonals per chunk task
    int32_t pad_;
    HashDev h;
    unsigned long long* qseq;   // per slot: sequence number (slot full when = position + 1)
    long long* qtask;           // per slot: task
    unsigned long long* qhead;  // next position to pop
    unsigned long long* qtail;  // next position to push
    int32_t* remaining;         // pairs still active in this launch
    uint32_t qcap;
    uint32_t pad2_;
    CountersDev* counters;
};

// Prepare launch: both strings of one pair in one kernel.
struct PrepString {
    const uint8_t* raw;    // input bytes (device), 16-byte aligned
    uint64_t* w2;          // packed output
    uint64_t* w4;          // 4-bit output (nullptr: no 4-bit layout for this pair)
    uint64_t* w8;          // 8-bit copy output
    uint64_t* tab;         // prefix table output (nullptr: no table)
    int32_t len;
    int32_t tiles;         // ceil(len / kTileChars), at least 1
    int32_t tile0;         // first global tile index of this string
    int32_t pad_;
};

struct PrepParams {
    PrepString s[2];
    int32_t total_tiles;
    int32_t log2b;
    int32_t force8;        // write 8-bit copies of every tile
    int32_t nt_copy;       // packed words and 8-bit copy with non-temporal stores (a pair larger than the MALL)
    int32_t build_table;
    int32_t fuse_table;    // block size 32: pack_kernel takes the block hashes (the first table pass)
    uint64_t r;            // hash base
    uint64_t* tile_agg;    // total_tiles entries: hash of each tile
    uint64_t* tile_prefix; // total_tiles entries: hash of its string before each tile (b = 32: of
                           // the tile's chunk of 2048 tiles before it)
    uint64_t* chunk_tot;   // per chunk of 2048 tiles of each string: its hash (prefix scan)
    uint64_t* lane_excl;   // 64 per tile: hash of the tile's characters before each lane's 256
    uint32_t* alpha;       // OR of all characters (written by after_pack_kernel)
    uint32_t* packed_any;  // bit c set when some chunk is of class c < 2 (after_pack_kernel)
    uint32_t* wg_or;       // pack_grid slots: each pack workgroup's OR | classes << 8
    int32_t pack_grid;     // workgroups of the pack launch
    int32_t scan_chunks;   // workgroups of the scan: chunks of kScanChunk tiles of both strings
    uint8_t* chunk_big;    // per chunk (kTileChunks per tile) its class: 0 no character > 3 (2-bit
                           // words written), 1 some above 3, none above 15 and a 4-bit layout (4-bit
                           // words written), 2 otherwise (8-bit copy written)
    const uint64_t* rtab;  // the kRtab* layout below
};

// Power and lookup tables of the table passes and of the hash queries, built
// on the host with the other power tables (R = r^kTileChars):
//   r^p, p = 0..64 | r^(64k), k = 0..256 | R^d, d = 0..64 |
//   lut32[k][v] = sum_j c_j r^(31-4k-j), c_j = 2-bit code j of byte v (k = 0..7) |
//   lut8[k][v] = v r^(7-k) (k = 0..7) | r^(-256 d), d = 0..64 |
//   R^(8 * 2^j), j = 0..9 | R^(8 (l + 1)), l = 0..63 | r^(-d), d = 0..32 |
//   per lane l = 0..63 the 16 int8 of its A operand of the block-hash matrix
//   product (two entries) | the constant term of that product |
//   R^(2048 d), d = 0..63 | R^j, j = 0..2047
constexpr int kRtabRseg = 65;
constexpr int kRtabR = kRtabRseg + 257;
constexpr int kRtabLut32 = kRtabR + 65;
constexpr int kRtabLut8 = kRtabLut32 + 8 * 256;
constexpr int kRtabRinv256 = kRtabLut8 + 8 * 256;
constexpr int kRtabR8pow2 = kRtabRinv256 + 65;
constexpr int kRtabR8lane = kRtabR8pow2 + 10;
constexpr int kRtabRinv32 = kRtabR8lane + 64;
constexpr int kRtabMmaA = kRtabRinv32 + 34;  // 16-byte aligned
constexpr int kRtabMmaK = kRtabMmaA + 128;
constexpr int kRtabRChunk = kRtabMmaK + 1;
constexpr int kRtabRTile = kRtabRChunk + 64;
constexpr int kRtabEntries = kRtabRTile + kScanChunkTiles;

struct LcpQueryParams {
    PairDev p;
    HashDev h;
    const int64_t* x;
    const int64_t* y;
    int64_t* out;
    int64_t count;
    int32_t engine;
    int32_t lane_words;
    CountersDev* counters;
    int32_t* result;  // grid tier: per-query first mismatch (INT32_MAX before launch)
    int64_t query;    // grid tier: the query this launch answers
};

// Kernel launchers (defined in the .hip files).
hipError_t launch_pack(const PrepParams& pp, int grid, hipStream_t s);
// after the pack kernel, always: the pair's alphabet and chunk classes, the
// rest pass, and (block hashes taken by the pack kernel) the chunk totals
hipError_t launch_after_pack(const PrepParams& pp, int grid, hipStream_t s);
hipError_t launch_table(const PrepParams& pp, int grid, hipStream_t s);
// cnt: kMaxGrid + 1 counter slots (one per workgroup, then their sum)
// One step of a traced path: at round t the path is on diagonal i, its run of
// matches is [c, f) (x = characters of A consumed), and (c, c - i) follows from
// the path's point at round t - 1 by `kind`.
enum StepKind : int32_t {
    kStepStart = 0,  // t = 0: (0, 0)
    kStepSub = 1,    // from (f', f' - i) on diagonal i: both advance
    kStepDel = 2,    // from diagonal i - 1: x advances (A character deleted)
    kStepIns = 3,    // from diagonal i + 1: y advances (B character inserted)
    kStepNone = 4,   // the same point (the diagonal's end was reached before)
    kStepFail = 5,   // no candidate produced the start (not expected)
};
struct PathStep {
    int32_t i, c, f, kind;
};
// A run of matches to re-check: A[x .. x + len) against B[y .. y + len).
struct VerifySeg {
    int32_t x, y, len, pad;
};

hipError_t launch_ctl_init(FrontierCtl* ctl, CountersDev* cnt, unsigned int* bar, hipStream_t s);
// Rows kept for a traceback, from round t0 on: row u holds the diagonals
// [lo(u), hi(u)] at dump[off(u) + j - lo(u)].
//   window (cone = 0): lo = wlo, hi = wlo + w - 1, off = (u - t0) w;
//   cone (cone = 1, t0 = 0): the diagonals that a path ending on diagonal
//   iend at round kend can visit, lo(u) = max(-u, iend - (kend - u)),
//   hi(u) = min(u, iend + (kend - u)); row u has room for min(2u + 1,
//   2(kend - u) + 1) entries, so with h = floor(kend / 2) off(u) = u^2 for
//   u <= h + 1, else (h + 1)^2 + (kend - h)^2 - (kend - u + 1)^2, and the
//   rows of rounds 0 .. kend take cone_total(kend) = off(kend + 1) entries.
struct KeepLayout {
    int32_t cone, t0, wlo, w, iend, kend;
};

__host__ __device__ inline int64_t cone_off(int64_t u, int64_t k) {
    const int64_t h = k / 2;
    return u <= h + 1 ? u * u : (h + 1) * (h + 1) + (k - h) * (k - h) - (k - u + 1) * (k - u + 1);
}

__host__ __device__ inline int64_t cone_total(int64_t k) { return cone_off(k + 1, k); }

__host__ __device__ inline void keep_bounds(const KeepLayout& L, int32_t u, int32_t& lo, int32_t& hi) {
    if (L.cone) {
        const int32_t a = L.iend - (L.kend - u), b = L.iend + (L.kend - u);
        lo = a > -u ? a : -u;
        hi = b < u ? b : u;
    } else {
        lo = L.wlo;
        hi = L.wlo + L.w - 1;
    }
}

__host__ __device__ inline void keep_row(const KeepLayout& L, int32_t u, int32_t& lo, int32_t& hi, int64_t& off) {
    keep_bounds(L, u, lo, hi);
    off = L.cone ? cone_off(u, L.kend) : static_cast<int64_t>(u - L.t0) * L.w;
}

// The steps of an optimal path for rounds te .. tb + 1 (and round 0 when tb
// = 0) from the frontier rows of rounds tb .. te kept in layout L (L.t0 =
// tb), starting on diagonal i_end of round te; state: [0] 0 ok, 1 bad start,
// 2 no candidate; [1], [2] the path's diagonal and row value at round tb.
hipError_t launch_traceback(const int32_t* dump, const KeepLayout& L, int32_t tb, int32_t te, int32_t i_end,
                            int32_t n, int32_t m, PathStep* out, int32_t* state, hipStream_t s);
// Sets *bad (nonzero) when some segment's characters differ.
hipError_t launch_verify(const PairDev& p, const VerifySeg* segs, int64_t count, uint32_t* bad, int grid,
                         hipStream_t s);
hipError_t launch_counters_sum(CountersDev* cnt, hipStream_t s);
hipError_t launch_frontier(const FrontierParams& fp, int grid, hipStream_t s);
hipError_t frontier_max_grid(int device, int* grid_out);
hipError_t launch_tasks(const TaskParams& tp, int grid, hipStream_t s);
hipError_t task_max_grid(int device, int* grid_out);
hipError_t launch_lcp_queries(const LcpQueryParams& qp, hipStream_t s);
hipError_t launch_lcp_grid(const LcpQueryParams& qp, int grid, hipStream_t s);
hipError_t launch_lcp_grid_finish(const LcpQueryParams& qp, hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);

}  // namespace ed
