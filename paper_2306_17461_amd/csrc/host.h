// Host-side state of libed.so (context, pair, device memory pool).
#pragma once
#include <map>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/ed.h"
#include "internal.h"

namespace ed {

// Device memory pool: released blocks are cached per size class and reused.
class DevPool {
  public:
    void* get(size_t bytes);
    void put(void* p);
    void trim();
    size_t cached() const { return cached_; }
    ~DevPool();

  private:
    std::map<size_t, std::vector<void*>> free_;
    std::unordered_map<void*, size_t> live_;
    size_t cached_ = 0;
};

// pow0 (65536) | pow1 (65536) | r^0..r^64 | r^(64k), k = 0..256 | R^d, d = 0..64
constexpr size_t kPowEntries = 2 * 65536 + kRtabEntries;
// a prefix table starts 248 bytes into its block, so that T[1] and with it the
// entries of every tile's blocks (T[512 t + 1 .. 512 t + 512] at b = 32) fill
// whole cache lines: the table passes read and write them 512 bytes at a time
constexpr size_t kTabShift = 248;
// the pack kernel writes the packed words and the 8-bit copy with
// non-temporal stores when the pair's input exceeds the 256 MiB memory-side
// cache (MALL; a variant of the kernel of its own): packed strings
// that fit stay there for the frontier's reads (with every packed word and
// copy stored non-temporally the frontier of the n = 1e8 pairs at k = 1e5 took
// 178-181 ms at 2 bits and 250 ms at 8 bits, against 168-171 and 236-239 ms,
// measured on one device), a copy that does not fit only evicts other lines
constexpr uint64_t kNtCopyBytes = 256ull << 20;

// layout of a pair's small device block
constexpr size_t kMiscAlpha = 64;

// single-pair kernel (measured best at n = 1e8 for k = 1e2 .. 1e5)
constexpr uint32_t kDefaultLdsRounds = 512;
constexpr uint32_t kDefaultBlockRounds = 64;
// many-pair kernel, when neither its own knob nor the single-pair one is set
// (a chunk task of 128 rounds: at 32 one n = 1e7, k = 1.8e5 pair took 864 ms
// in this kernel, at 128 500 ms; 4096 small pairs and the serving traces are
// faster too; 2048 rounds of a whole pair in one workgroup: 4096 small pairs
// 5% faster than at 1024, the serving traces the same, 4096 raises their p99)
constexpr uint32_t kTaskDefaultLdsRounds = 2048;
constexpr uint32_t kTaskDefaultBlockRounds = 128;
// diagonals per chunk task: with a halo of H = 128 per side a chunk's window
// stays within one pass of the 1024-thread workgroup (2 diagonals per thread)
constexpr int32_t kChunkDiags = 1536;
// a wait of the frontier kernel on another workgroup or wavefront gives up
// after 600 s of the 100 MHz real-time clock (the launch then reports an
// error): far beyond any wait of a working launch, so that only a launch that
// would never end is cut
constexpr uint64_t kWaitTicks = 60000000000ull;

}  // namespace ed

struct ed_ctx {
    int device = 0;
    ed_options opt;
    std::mutex mu;
    int num_cu = 0;
    int frontier_grid_max = 0;
    int task_grid_max = 0;
    uint64_t r = 0;              // hash base of opt.hash_seed
    uint64_t* d_pow = nullptr;   // power tables (see kPowEntries)
    ed::FrontierCtl* d_ctl = nullptr;
    ed::CountersDev* d_cnt = nullptr;
    ed::FrontierCtl* h_ctl = nullptr;  // pinned
    ed::CountersDev* h_cnt = nullptr;  // pinned
    hipEvent_t ev[2] = {nullptr, nullptr};  // frontier timing
    unsigned int* d_bar = nullptr;          // device-wide barrier flags
    int32_t* d_scratch = nullptr;           // this device's scratch array (ed_distance_noalloc)
    int32_t* d_gpart = nullptr;             // grid rounds: per-workgroup first mismatches of queued LCPs
    ed::DevPool pool;
};

struct ed_pair {
    ed_ctx* ctx = nullptr;
    uint64_t len[2] = {0, 0};
    uint32_t engine = 0;
    int32_t log2b = 5;
    int32_t force8 = 0;
    uint64_t r = 0;  // hash base its tables were built with
    void* w2[2] = {nullptr, nullptr};
    void* w4[2] = {nullptr, nullptr};  // direct engine with automatic packing only
    void* w8[2] = {nullptr, nullptr};
    void* tab[2] = {nullptr, nullptr};      // prefix tables: T[0] of each string
    void* tab_blk[2] = {nullptr, nullptr};  // their pool blocks (T[0] at kTabShift)
    void* stage[2] = {nullptr, nullptr};
    void* misc = nullptr;  // alphabet word, tile hashes and prefixes, chunk flags
    void* f0 = nullptr;    // unused (rows are per call)
    void* f1 = nullptr;
    uint64_t rounds = 0;
    // the last unbounded distance of this pair and the engine it ran on (-1: none)
    int64_t known_k = -1;
    uint32_t known_engine = 0;
    ed::CountersDev counters{};
    int launches_prepare = 0;
    int launches_distance = 0;
    double ns_prepare = 0, ns_distance = 0;
    // around the prepare kernels, and before the table kernels (ED_FLAG_TIMING)
    hipEvent_t ev_prep[3] = {nullptr, nullptr, nullptr};
    // recorded after the prepare's kernels on the caller's stream: the only
    // work on a pair that a call leaves queued (the others synchronise)
    hipEvent_t ev_done = nullptr;
    bool prep_timed = false;
    double gpu_ns_frontier = 0;
    double gpu_ns_lcp = 0;  // last ed_debug_lcp with the grid tier (ED_FLAG_TIMING)
    uint64_t certify_retries = 0;  // ED_FLAG_CERTIFY: hash results whose check failed
    uint64_t align_bytes = 0;      // last alignment: device bytes of kept rows, segment rows, path
    uint64_t align_seg = 0;        // last alignment: rounds per segment
    // ed_align: a script that did not fit the caller's buffer, kept for the retry
    std::vector<ed_op_run> script;
    uint64_t script_k = 0;
    bool script_kept = false;
    uint64_t rounds_phase_a = 0;
    double us_phase_a = 0, us_phase_b = 0;
};

namespace ed {
void set_error(const char* fmt, ...);
// hash base of a set of options (the seed's base, or 1 with ED_FLAG_WEAK_HASH)
uint64_t opt_base(const ed_options& o);
// power and lookup tables of base r on the context (no work when already there)
int ctx_set_hash(ed_ctx* c, uint64_t r);
void pair_free(ed_pair* p);
PairDev pair_dev(const ed_pair* p);
HashDev ctx_hash(const ed_ctx* c);
int prepare_locked(ed_ctx* c, const uint8_t* A, uint64_t n, const uint8_t* B, uint64_t m,
                   int on_device, hipStream_t s, ed_pair** out);
// The fields of a frontier launch that depend only on the context, its
// options and the pair (the hash tables of the pair's base made current);
// rows, t0, K, k_max and the dump are the caller's.
int frontier_setup(ed_ctx* c, ed_pair* p, FrontierParams& fp);
// One frontier launch, its control block reset first; the control block and
// the summed counters are left in c->h_ctl and c->h_cnt, and gpu_ns (if
// given) gains the kernel's time under ED_FLAG_TIMING.
int frontier_once(ed_ctx* c, const FrontierParams& fp, hipStream_t s, double* gpu_ns);
void counters_add(CountersDev& a, const CountersDev& b);
// rows: host copy of every round's frontier row (ed_distance_dump);
// fixed_rows: two rows of 2 fixed_K + 5 entries that the caller owns (no
// allocation and no growth; needs 0 <= k_max <= fixed_K)
int distance_locked(ed_ctx* c, ed_pair* p, int64_t k_max, uint64_t* k_out, int32_t* rows,
                    uint64_t rows_cap, hipStream_t s, int32_t* fixed_rows = nullptr, int64_t fixed_K = 0);
// device address of this device's scratch array (noalloc.hip), taken once at
// ed_init with the device current
int scratch_setup(ed_ctx* c);
// k, an optimal path (k + 1 steps) and the direct check of its runs of matches
int align_locked(ed_ctx* c, ed_pair* p, uint64_t* k_out, std::vector<PathStep>& path, hipStream_t s);
// One launch of the many-pair kernel over `st` (each pair's own k_max), the
// first tasks queued: started on stream s, then waited for (pair states
// copied back).  The run keeps its device block and host images in between.
struct TaskRun {
    void* blk = nullptr;
    TaskPair* d_pairs = nullptr;
    size_t pairs_bytes = 0;
    std::vector<unsigned long long> seq;
    std::vector<long long> task;
    unsigned long long ctr[2] = {0, 0};
    int32_t remaining = 0;
};
int tasks_start(ed_ctx* c, const std::vector<TaskPair>& st, const std::vector<long long>& first, uint32_t engine,
                hipStream_t s, TaskRun& run);
int tasks_wait(ed_ctx* c, std::vector<TaskPair>& st, hipStream_t s, TaskRun& run);
int tasks_run(ed_ctx* c, std::vector<TaskPair>& st, const std::vector<long long>& first, uint32_t engine,
              hipStream_t s);
long long task_solo(int32_t pi);
long long task_chunk(int32_t pi, int32_t c);
int32_t block_rounds_of(const ed_ctx* c);
uint32_t task_solo_rounds(const ed_ctx* c);
int32_t chunk_diags_of(const ed_ctx* c);
bool schedule_on_host(TaskPair& tp, int32_t pi, int32_t block_rounds, int32_t chunk, int64_t k_max,
                      std::vector<long long>& tasks);
int64_t batch_row_capacity(int64_t maxnm, int64_t k_max, uint32_t lds_rounds);
}  // namespace ed
