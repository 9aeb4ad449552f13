/*
 * ed.h -- exact output-sensitive edit distance on AMD Instinct MI355X (gfx950).
 *
 * C ABI of libed.so.  Plain pointers and sizes only; no C++ or framework types
 * cross this boundary and no exception leaves the library.
 *
 * The method is the breadth-first (Landau-Vishkin) frontier of "Efficient
 * Parallel Output-Sensitive Edit Distance" (Ding, Dong, Gu, Liu, Sun; ESA 2023):
 * round t computes, for every diagonal i = x - y in [-t, t], the furthest row
 * reachable with t edits, from the three neighbours of round t-1, followed by a
 * slide along the diagonal by a longest-common-prefix (LCP) query
 * (section 3.1, Algorithm 1; appendix A).  The LCP queries run on one of two
 * engines:
 *   ED_ENGINE_DIRECT  64-bit word XOR / count-trailing-zeros comparison of the
 *                     strings (the LCP definition of section 2, with the
 *                     leading-characters shortcut of section 5.1);
 *   ED_ENGINE_HASH    prefix-hash tables T[j] = h(S[0..jb)) mod 2^61-1
 *                     (sections 3.2 and 3.3, Algorithm 2) probed by a
 *                     wavefront-parallel galloping and 64-ary search; every
 *                     answer is confirmed by a direct comparison of the
 *                     characters around the reported mismatch, and a detected
 *                     hash collision falls back to the direct engine.
 *
 * Coordinates: strings are 0-based byte arrays A[0..n), B[0..m); the result is
 * the Levenshtein distance (minimum number of unit insertions, deletions and
 * substitutions; sections 1 and 2).  n and m must be below ED_MAX_LEN.
 *
 * Threading: every call on one context is serialised by the context's mutex.
 * Streams: `hip_stream` arguments are hipStream_t values (NULL = the null
 * stream).  A result written to host memory is valid when the call returns.
 */
#ifndef ED_H
#define ED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define ED_OK 0
#define ED_EINVAL (-1)     /* bad argument: NULL with length > 0, length >= ED_MAX_LEN,
                              a character > 3 with pack_bits = 2, bad option value */
#define ED_ENOMEM (-2)     /* device or host allocation failed */
#define ED_EDEVICE (-3)    /* a HIP call failed; ed_last_error() has the detail */
#define ED_ECOLLISION (-4) /* ed_align: a run of matches on the hash engine's traced path does not
                              match (a hash collision); the direct engine gives the exact answer */
#define ED_EBUSY (-5)      /* serving: host queue full */
#define ED_EINTERNAL (-6)  /* an internal consistency check failed (a bug) */

#define ED_MAX_LEN ((uint64_t)2146435072u) /* 2^31 - 2^20 characters */

/* ---- options ------------------------------------------------------------ */
#define ED_ENGINE_DIRECT 0u
#define ED_ENGINE_HASH 1u

#define ED_FLAG_DEBUG_DUMP 1u  /* keep per-round frontier rows (see ed_distance_dump) */
#define ED_FLAG_NO_PHASE_A 2u  /* run every round grid-wide (skip the one-workgroup phase) */
#define ED_FLAG_SHUFFLE 4u     /* batch: permute the work order with hash_seed (race test) */
#define ED_FLAG_TIMING 8u      /* time the prepare and frontier kernels with HIP events */
#define ED_FLAG_CERTIFY 16u    /* ed_distance, hash engine, no k_max: check the result as ed_align
                                * does, and answer with the direct engine if the check fails */
#define ED_FLAG_NO_GRID_ROUNDS 64u /* direct engine: never run the first rounds on every workgroup
                                   * (the grid tier for very long slides); workgroup 0 alone */
#define ED_FLAG_HASH_FIRST 128u /* hash engine: a slide that runs past the lane stage goes to the
                                 * wavefront's hash search at once (no direct steps); for pairs
                                 * with many long slides */
#define ED_FLAG_ALIGN_SEGMENTS 256u /* ed_align: keep rows in segments even when k is known and the
                                    * cone of rows fits (tests of the segmented form) */
#define ED_FLAG_WEAK_HASH 32u  /* fault injection for tests: hash base r = 1 (every permutation of
                                * a string hashes alike), so that collisions happen */

typedef struct ed_options {
    uint32_t engine;    /* ED_ENGINE_DIRECT or ED_ENGINE_HASH */
    uint32_t pack_bits; /* 0 = automatic (2-bit when every character is 0..3; direct engine:
                         * 4-bit when every character is 0..15), 2 or 8 */
    uint32_t block;     /* hash block size b (power of two, 1..4096); 0 = 32 */
    uint32_t flags;     /* ED_FLAG_* */
    uint64_t hash_seed; /* the hash base r is derived from this seed (see ed_hash_base) */
    /* tuning knobs; 0 = the library default or the autotuned value */
    uint32_t lds_rounds;   /* rounds kept in one workgroup's LDS before going grid-wide */
    uint32_t lane_words;   /* words compared per lane before a wave takes over an LCP */
    uint32_t grid_blocks;  /* workgroups of the persistent kernels */
    uint32_t init_rows;    /* initial frontier capacity in diagonals per side (grown on demand) */
    uint32_t block_rounds; /* grid-wide phase: rounds per device-wide barrier (temporal blocking) */
    /* knobs of the many-pair kernel (ed_batch, serving); 0 = default or autotuned */
    uint32_t chunk_diags;       /* diagonals per chunk task (64..8000) */
    uint32_t task_lds_rounds;   /* rounds a whole-pair task keeps in LDS (<= 4096) */
    uint32_t task_block_rounds; /* rounds per chunk task (<= 4096) */
} ed_options;

/* Fills *opt with the defaults: direct engine, automatic packing, b = 32,
 * seed 0x5EED, no flags, automatic tuning knobs. */
void ed_default_options(ed_options *opt);

/* Base r of the polynomial hash for a seed: one splitmix64 output z of
 * (seed + 0x9E3779B97F4A7C15), then r = 2^20 + z mod (2^61 - 1 - 2^21). */
uint64_t ed_hash_base(uint64_t seed);

/* ---- context -------------------------------------------------------------- */
typedef struct ed_ctx ed_ctx;
typedef struct ed_pair ed_pair;

/* Creates a context on HIP device `device`.  opt may be NULL (defaults).
 * Errors: ED_EINVAL (bad device or options), ED_EDEVICE, ED_ENOMEM. */
int ed_init(ed_ctx **out, int device, const ed_options *opt);

/* Replaces the context's options (pairs prepared later use them). */
int ed_set_options(ed_ctx *ctx, const ed_options *opt);
int ed_get_options(ed_ctx *ctx, ed_options *opt);

/* Releases the context and every device buffer it owns.  Pairs prepared on it
 * must be released first. */
int ed_shutdown(ed_ctx *ctx);

/* ---- single pair ------------------------------------------------------------ */
/*
 * Copies A[0..n) and B[0..m) into buffers owned by a new pair, detects the
 * alphabet (bitwise OR of all characters; 2-bit packing when it is <= 3 and
 * pack_bits is 0 or 2; for the direct engine with pack_bits = 0, 4-bit
 * packing when it is <= 15; else an 8-bit copy), packs, and -- for the hash
 * engine -- builds the prefix
 * tables T_A, T_B of section 3.3.  A and B are device pointers when
 * inputs_on_device != 0, host pointers otherwise; the caller keeps ownership
 * and may free them once `hip_stream` has synchronised.  A may be NULL iff
 * n = 0, B iff m = 0.  The work is queued on `hip_stream`; with pack_bits = 2
 * the call synchronises to report ED_EINVAL for characters above 3.
 * Errors: ED_EINVAL, ED_ENOMEM, ED_EDEVICE.
 */
int ed_prepare(ed_ctx *ctx, const uint8_t *A, uint64_t n, const uint8_t *B, uint64_t m,
               int inputs_on_device, void *hip_stream, ed_pair **out);

/* Frees the pair's device buffers (back to the context's pool).  Waits for the
 * pair's prepare kernels if they are still queued on the caller's stream (every
 * other call on a pair returns after its work), not for the whole device. */
int ed_release(ed_pair *pair);

/*
 * Edit distance of a prepared pair.  All rounds of the frontier run in one
 * persistent launch (device-wide barriers between rounds); the launch is
 * repeated only when the frontier outgrows its buffer.  With k_max >= 0 the
 * search stops after round k_max and reports k_max + 1 if the distance is
 * larger (the band |x - y| <= k of section 3.1).  Synchronous on hip_stream.
 */
int ed_distance(ed_ctx *ctx, ed_pair *pair, int64_t k_max, uint64_t *k_out, void *hip_stream);

/*
 * For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): ed_distance with every round's frontier
 * rows in a fixed device array of the library instead of memory from the
 * context's pool.  It calls no hipMalloc, hipFree or other allocating routine.
 * k_max is required and bounded: 0 <= k_max <= ED_NOALLOC_MAX_K, else
 * ED_EINVAL (the array holds the two rows of 2 k_max + 5 int32 entries, 8 MB);
 * as with ed_distance, *k_out = k_max + 1 when the distance is larger.  The
 * pair must have been prepared with the context's current hash base (else
 * ED_EINVAL).  The array is one per device, shared by every context and call
 * on that device: calls that overlap on one device race, and it keeps the
 * last call's contents (every entry a call reads it writes first).
 * Synchronous on hip_stream.  Errors: ED_EINVAL, ED_EDEVICE, ED_EINTERNAL.
 */
#define ED_NOALLOC_MAX_K ((uint64_t)500000u)
int ed_distance_noalloc(ed_ctx *ctx, ed_pair *pair, int64_t k_max, uint64_t *k_out, void *hip_stream);

/*
 * As ed_distance, and also copies the frontier of every round to `rows`
 * (host int32 array): row t (t = 0..k) starts at index t*t and holds the 2t+1
 * entries f_t[-t..t]; a diagonal without a cell holds ED_NONE.  Needs
 * (k+1)^2 <= rows_cap, else ED_EINVAL after computing k.
 */
#define ED_NONE (-(1 << 30))
int ed_distance_dump(ed_ctx *ctx, ed_pair *pair, int64_t k_max, uint64_t *k_out, int32_t *rows,
                     uint64_t rows_cap, void *hip_stream);

/* ---- alignment ---------------------------------------------------------------- */
/* One run of an edit script: `len` consecutive operations of one kind. */
typedef struct ed_op_run {
    uint32_t op; /* ED_OP_* */
    uint32_t pad;
    uint64_t len;
} ed_op_run;
#define ED_OP_MATCH 0u /* A[x] == B[y]; x and y advance */
#define ED_OP_SUB 1u   /* A[x] replaced by B[y]; x and y advance */
#define ED_OP_DEL 2u   /* A[x] deleted; x advances */
#define ED_OP_INS 3u   /* B[y] inserted; y advances */

/* Edit distance and an optimal edit script, checked.  The frontier rounds of
 * Algorithm 1 (section 3.1) are run twice: once for k (skipped when an
 * unbounded ed_distance on the pair with the same engine gave it), once
 * keeping every round's row in device memory ((k+1)^2 * 4 bytes, allocated
 * and freed by the call); from the row of round k at diagonal n - m the path is traced back on
 * the device (each round's start comes from one of the three neighbours of the
 * previous round, which names the edit), and every run of matches on it is
 * compared character by character on the device.  The script applied to A
 * gives B and has k edits.  With the hash engine this check makes the result
 * exact: a collision can only make an LCP too long (k too small), and a valid
 * script of k edits shows ED <= k.  runs: caller memory for `runs_cap`
 * entries (2k + 1 always suffice); *n_runs receives the count.  When runs_cap
 * is too small the call returns ED_EINVAL with *n_runs (and *k_out) set and
 * keeps the script with the pair: the next ed_align on the pair returns it
 * without recomputing.  Errors: ED_EINVAL, ED_ENOMEM (the rows do not fit),
 * ED_ECOLLISION (hash engine: a run
 * does not match; *k_out holds the unchecked k), ED_EINTERNAL (the traced path
 * is not a valid script: a bug), ED_EDEVICE. */
int ed_align(ed_ctx *ctx, ed_pair *pair, uint64_t *k_out, ed_op_run *runs, uint64_t runs_cap, uint64_t *n_runs,
             void *hip_stream);

/* ---- batch ---------------------------------------------------------------- */
/*
 * Edit distances of `count` prepared pairs in one persistent launch: the
 * workgroups take (pair, diagonal-chunk) work from a device queue, largest
 * pairs first.  k_out[i] and status_out[i] (either may be NULL) receive each
 * pair's result; the return value is the first error, or ED_OK.
 */
int ed_batch(ed_ctx *ctx, ed_pair *const *pairs, uint64_t count, int64_t k_max, uint64_t *k_out,
             int32_t *status_out, void *hip_stream);

/* ---- introspection ---------------------------------------------------------- */
typedef struct ed_stats {
    uint64_t n, m;
    uint32_t bits_per_char;  /* 2, 4 or 8, as detected */
    uint32_t engine;
    uint64_t rounds;          /* k of the last ed_distance (or batch) */
    uint64_t updates;         /* diagonal updates over all rounds */
    uint64_t lcp_chars;       /* sum of all slides */
    uint64_t wave_lcps;       /* LCPs handed from a lane to a whole wave */
    uint64_t grid_lcps;       /* LCPs handed to the whole grid (grid tier) */
    uint64_t hash_queries;    /* LCPs answered by the hash engine */
    uint64_t hash_probes;     /* hash equality tests */
    uint64_t collisions;      /* detected collisions (fell back to the direct engine) */
    double collision_bound;   /* hash engine: bound on the probability (over the base drawn from
                               * the seed) that the last run met an undetected collision: the sum
                               * of (L - 1) / (2^61 - 1 - 2^21) over the verdicts on strings of
                               * length L that decided a step of a hash search (Schwartz-Zippel) */
    uint64_t launches;        /* kernel launches of the last ed_distance */
    double ns_prepare, ns_distance; /* host wall time of the last calls */
    /* with ED_FLAG_TIMING: HIP-event time of the prepare kernel and of the
     * frontier kernel launches (summed over relaunches), on the call's stream */
    double gpu_ns_prepare_kernel, gpu_ns_frontier_kernel;
    /* device clock split of the last frontier launch: rounds and microseconds
     * in the one-workgroup phase and in the grid-wide phase */
    uint64_t rounds_phase_a;
    double us_phase_a, us_phase_b;
    /* with ED_FLAG_TIMING: HIP-event time of the last ed_debug_lcp call on the
     * grid tier (engine 3), all its queries */
    double gpu_ns_lcp_kernel;
    uint64_t wg_lcps;         /* LCPs extended by a whole workgroup (workgroup tier) */
    /* with ED_FLAG_TIMING, hash engine: HIP-event time of the prefix-table
     * kernels that follow the pack kernel (part of gpu_ns_prepare_kernel; at
     * b = 32 the pack kernel itself takes the block hashes, so this is the
     * scan and the emission of T; 0 for the direct engine) */
    double gpu_ns_table_kernel;
    /* ED_FLAG_CERTIFY: hash-engine distances whose check failed (then answered
     * by the direct engine) */
    uint64_t certify_retries;
    /* last ed_align (or certified distance): device bytes of its kept rows,
     * segment rows and path, and the rounds per segment between kept rows */
    uint64_t align_device_bytes;
    uint64_t align_segment_rounds;
} ed_stats;

int ed_pair_stats(const ed_pair *pair, ed_stats *out);

/* ---- autotuning ------------------------------------------------------------------ */
typedef struct ed_tune_result {
    ed_options best;    /* the context's options after tuning */
    double default_ms;  /* batch time with the options the call started from */
    double best_ms;     /* batch time with `best` */
    uint32_t evaluated; /* configurations timed */
    uint32_t pad;
} ed_tune_result;

/* Autotuner of the many-pair kernel (the batch form of section 3.1's rounds,
 * not a passage of the paper): times ed_batch on `pairs` for candidate values
 * of task_lds_rounds, task_block_rounds and chunk_diags by coordinate descent
 * (`passes` sweeps over the knobs, 0 = 2), requires every configuration to
 * return the same distances, and leaves the fastest configuration in the
 * context's options (ed_batch and the serving loop use it).  The pairs stay
 * prepared.  Each configuration runs the whole batch once; the call takes about
 * (3 + 18 * passes) batch times.  Errors: as ed_batch; ED_EINTERNAL when two
 * configurations disagree (the message names the pair). */
int ed_autotune_batch(ed_ctx *ctx, ed_pair *const *pairs, uint64_t count, int64_t k_max,
                      uint32_t passes, ed_tune_result *out, void *hip_stream);

/* ---- debug read-backs (used by the tests) ------------------------------------ */
#define ED_BUF_PACKED2 0 /* 2-bit words, char j at bits [2(j mod 32), +2) of word j/32 */
#define ED_BUF_BYTES 1   /* 8-bit copy (only when bits_per_char = 8) */
#define ED_BUF_TABLE 2   /* prefix table, floor(len/b) + 1 uint64 entries */
#define ED_BUF_PACKED4 3 /* 4-bit words, char j at bits [4(j mod 16), +4) of word j/16 (only when
                          * bits_per_char = 4) */
/* Copies a pair buffer of string `which` (0 = A, 1 = B) to host memory `out`
 * (cap bytes); *len_out receives the byte length of the valid part. */
int ed_pair_buffer(ed_ctx *ctx, const ed_pair *pair, int which, int kind, void *out, uint64_t cap,
                   uint64_t *len_out);

/* Runs the pair's LCP engine on `count` queries (x[i], y[i]) (host arrays) and
 * writes LCP(A, B, x[i], y[i]) to out[i] (section 2's LCP; 0 <= x[i] <= n,
 * 0 <= y[i] <= m, else ED_EINVAL).  engine: -1 = the prepared engine; 0 = the
 * direct engine's lane and wave tiers, one wavefront per query; 1 = the hash
 * engine (needs tables), one wavefront per query; 2 = the direct engine's
 * workgroup tier, one workgroup per query; 3 = the direct engine's grid tier,
 * every wavefront of the device on one query at a time (static segments taken
 * in increasing order, first mismatch by a shared minimum), timed with
 * ED_FLAG_TIMING into ed_stats.gpu_ns_lcp_kernel.  The same device code as
 * the frontier kernels. */
int ed_debug_lcp(ed_ctx *ctx, ed_pair *pair, int engine, const int64_t *x, const int64_t *y,
                 uint64_t count, int64_t *out, void *hip_stream);

/* The check behind ed_align on runs given by the caller: compares A[x[i] ..
 * x[i] + len[i]) with B[y[i] .. y[i] + len[i]) for i < count on the device and
 * sets *bad to 1 if any character differs, else 0 (runs inside the strings,
 * else ED_EINVAL). */
int ed_debug_check_runs(ed_ctx *ctx, ed_pair *pair, const int32_t *x, const int32_t *y, const int32_t *len,
                        uint64_t count, uint32_t *bad, void *hip_stream);

/* Dependent-access latency on this device, for measurement: a cycle of links
 * one per 128-byte line over a fresh region of region_bytes (a power of two,
 * 8 KiB .. 256 GiB; allocated and freed by the call), followed by one
 * wavefront whose every access reads the address of the next (64 chains),
 * `steps` links each (1 .. 2^24); with warm != 0 the same walk runs once
 * before the timed one, so a region that fits a cache is read from it.
 * *ns_per_access = HIP-event time / steps.  A frontier round (Algorithm 1)
 * needs at least one such access: its LCP loads take their addresses from
 * the previous round's row.  ED_EINVAL on bad sizes, ED_ENOMEM when the
 * region cannot be allocated, ED_EDEVICE on a HIP error. */
int ed_debug_mem_latency(ed_ctx *ctx, uint64_t region_bytes, uint32_t steps, int warm, double *ns_per_access);

/* ---- serving ---------------------------------------------------------------- */
typedef struct ed_server ed_server;
typedef struct ed_result {
    uint64_t tag;
    uint64_t k;
    int32_t status;
    int32_t pad;
    uint64_t t_arrive_ns; /* submit time (CLOCK_MONOTONIC) */
    uint64_t t_done_ns;   /* completion time */
} ed_result;

/* Opens a request loop on the context: requests are admitted while their
 * device bytes fit in hbm_budget_bytes and a slot is free (max_slots); admitted
 * requests advance together in shared launches, and finished slots are refilled
 * between launches (continuous batching).  The copies and packing of newly
 * admitted requests run on a second stream while the current launch runs. */
int ed_serve_open(ed_ctx *ctx, uint64_t hbm_budget_bytes, uint32_t max_slots, ed_server **out);
/* Copies the strings (host memory) and queues the request.  ED_EBUSY if the
 * host queue is full; ED_ENOMEM if the request alone exceeds the budget. */
int ed_serve_submit(ed_server *srv, const uint8_t *A, uint64_t n, const uint8_t *B, uint64_t m,
                    uint64_t tag);
/* As ed_serve_submit, with a bound of its own for this request: k_max >= 0
 * stops it after round k_max (the band |x - y| <= k_max of section 3.1), and
 * its result k is then k_max + 1 when the distance is larger (status ED_OK);
 * its frontier rows are sized for at most k_max rounds.  k_max = -1: no bound.
 * ED_EINVAL for k_max < -1. */
int ed_serve_submit_band(ed_server *srv, const uint8_t *A, uint64_t n, const uint8_t *B, uint64_t m,
                         uint64_t tag, int64_t k_max);
/* Moves up to max finished results into out; *got receives their number. */
int ed_serve_poll(ed_server *srv, ed_result *out, uint32_t max, uint32_t *got);
/* Blocks until every submitted request has finished. */
int ed_serve_drain(ed_server *srv);
int ed_serve_close(ed_server *srv);

/* ---- errors ----------------------------------------------------------------- */
const char *ed_strerror(int status);
/* Detail of the last error on the calling thread ("" if none). */
const char *ed_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ED_H */
