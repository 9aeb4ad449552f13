"""Benchmark: exact edit distance, chars/sec at n = 1e8 for k = 1e2, 1e3, 1e4, 1e5.

One step = the whole hot path for the four single pairs (A: 1e8 characters
uniform over {0,1,2,3}; B = A with k planted edits; seed 0): for each pair,
alphabet detection, 2-bit packing, [prefix tables], all frontier rounds with
LCP extension, and the distance read back to the host.  Inputs are resident in
device memory (torch uint8 tensors) when the timed region starts.

    value = 4e8 characters / (seconds per step)

Prints one JSON line.  With --gpus N > 1 it exits: the benchmark measures one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
KS = [100, 1000, 10000, 100000]
N = 10 ** 8


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def measured_traffic(kernel, engine, ks, n):
    """HBM bytes per launch from the committed rocprofv3 counter runs, or None
    when the kernel sources changed since they were taken (or another
    workload is being timed)."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
        src = b"".join(open(os.path.join(ROOT, "paper_2306_17461_amd", "csrc", f), "rb").read()
                       for f in rec["sources"])
    except (OSError, KeyError, ValueError):
        return None
    if hashlib.sha256(src).hexdigest() != rec["source_sha256"]:
        return None
    if engine != "direct" or ks != KS or n != N:
        return None
    return rec["per_launch_bytes"].get(kernel)


# The paper's own full-run times at n = 10^8 (table of full runs; BFS-B-Hash
# and BFS-Hash, build + query, median of 3), measured on 96 cores (4x Xeon Gold
# 6252) with |alphabet| = 256 and Monte Carlo hashing.  Context only: another
# machine, another alphabet.
PAPER_N1E8_SECONDS = {100: {"b_hash": 0.026, "hash": 0.052}, 1000: {"b_hash": 0.077, "hash": 0.079},
                      10000: {"b_hash": 0.625, "hash": 0.538}, 100000: {"b_hash": 11.8, "hash": 9.46}}


# The rest of that table (appendix, full runs): n = 10^6 .. 10^9, k = 1 .. 10^5,
# the better of BFS-B-Hash and BFS-Hash (build + query, seconds; None where the
# paper prints "< .001").
PAPER_GRID_SECONDS = {
    10 ** 6: {1: None, 10: None, 100: 0.002, 1000: 0.022, 10000: 0.362, 100000: 6.79},
    10 ** 7: {1: 0.005, 10: 0.004, 100: 0.007, 1000: 0.028, 10000: 0.391, 100000: 8.03},
    10 ** 8: {1: 0.022, 10: 0.028, 100: 0.026, 1000: 0.077, 10000: 0.538, 100000: 9.46},
    10 ** 9: {1: 0.200, 10: 0.204, 100: 0.214, 1000: 0.268, 10000: 0.978, 100000: 12.0},
}


def paper_context(ks, n):
    if n != N or any(k not in PAPER_N1E8_SECONDS for k in ks):
        return None
    best = {str(k): min(PAPER_N1E8_SECONDS[k].values()) for k in ks}
    total = sum(best.values())
    return {"hardware": "96 cores (4x Intel Xeon Gold 6252), ParlayLib", "alphabet": 256,
            "exact": False, "seconds_per_k_best_of_two": best,
            "chars_per_s_same_four_pairs": n * len(ks) / total,
            "note": "the paper's numbers on its machine and alphabet; not this workload"}


def host_cpu():
    """Model name and logical CPU count of the host (for the CPU baselines)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def stored_oracle():
    """Oracle distances of the workloads (tests/golden/fullsize.json), if present."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "fullsize.json")) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def batch_leg(ed, ctx, count=4096, seed=0, cpu_sample=0):
    """Batched workload: `count` pairs, n = floor(10^U) with U ~ U[3, 6], alphabet
    {0,1,2,3}, k ~ U{0..floor(0.01 n)} planted edits.  One ed_batch launch against
    a loop of one ed_distance launch per pair, on the same prepared pairs."""
    import synth
    log("batch leg: generating %d pairs" % count)
    specs = synth.batch_specs(count, seed)
    pairs = []
    chars = 0
    for n, k, ps in specs:
        A, B, _ = synth.single_pair(n, k, ps)
        pairs.append(ed.ed_prepare(ctx, A, B))
        chars += len(A)
    ed.ed_batch(ctx, pairs)  # warm-up
    t0 = time.perf_counter()
    k0, _ = ed.ed_batch(ctx, pairs)
    tb0 = time.perf_counter() - t0
    # the autotuner picks the many-pair kernel's knobs on this batch (untimed)
    log("batch leg: autotuning")
    tune = ed.ed_autotune_batch(ctx, pairs)
    t0 = time.perf_counter()
    kb, _ = ed.ed_batch(ctx, pairs)
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    kp = [ed.ed_distance(ctx, p) for p in pairs]
    tp = time.perf_counter() - t0
    if kb != kp or kb != k0:
        raise SystemExit("batch and per-pair distances differ")
    gold = stored_oracle()
    exact = None
    gb = next((b for b in (gold or {}).get("batch", []) if b["count"] == count and b["seed"] == seed), None)
    if gb is not None:
        exact = kb == gb["eds"]
        if not exact:
            raise SystemExit("batch distances differ from the stored oracle values")
    for p in pairs:
        ed.ed_release(p)
    cpu = None
    if cpu_sample:
        # the oracle on the first `cpu_sample` pairs (by default all), one pair per host thread
        import oracle
        from concurrent.futures import ThreadPoolExecutor
        log("batch leg: oracle on %d pairs" % cpu_sample)
        sample = [synth.single_pair(nn, kk, ps)[:2] for nn, kk, ps in specs[:cpu_sample]]
        t0 = time.perf_counter()
        with ThreadPoolExecutor(os.cpu_count() or 1) as ex:
            kc = list(ex.map(lambda ab: oracle.lv_omp(ab[0], ab[1], -1, 1), sample))
        tcpu = time.perf_counter() - t0
        if kc != list(kb[:cpu_sample]):
            raise SystemExit("batch: oracle and GPU distances differ")
        cpu = {"pairs_per_s": cpu_sample / tcpu, "cores": os.cpu_count(), "kind": "oracle",
               "sample": "oracle lv_omp, one thread per pair, on the first %d pairs of the batch, %.1f s"
                         % (cpu_sample, tcpu)}
    return {"workload": "%d pairs, n log-uniform [1e3, 1e6], alphabet {0,1,2,3}, k uniform "
                        "[0, 0.01 n], seed %d" % (count, seed),
            "cpu_baseline": cpu,
            "pairs": count, "chars_A": chars, "sum_k": int(sum(kb)),
            "batched_pairs_per_s": count / tb, "batched_s": tb,
            "untuned_batched_pairs_per_s": count / tb0,
            "autotune": {"knobs": tune["knobs"], "default_ms": round(tune["default_ms"], 3),
                         "best_ms": round(tune["best_ms"], 3), "evaluated": tune["evaluated"]},
            "per_pair_pairs_per_s": count / tp, "per_pair_s": tp,
            "speedup": tp / tb, "equal_to_stored_oracle": exact}


def lcp_leg(ed, n=10 ** 9):
    """LCP extension bandwidth at 2 and 8 bits per character.

    In the distance path: ed_distance on a pair whose first slide covers the
    whole string (B = A with its last character changed, distance 1), so the
    run is one LCP of n - 1 characters; with the grid rounds (every
    workgroup extends it) and, beside it, with workgroup 0's workgroup tier
    alone (ED_FLAG_NO_GRID_ROUNDS).  Bytes = both strings' packed words over
    the matched length; time = the frontier kernel (HIP events).
    Microbenchmark: the same LCP through the grid-tier query kernel of
    ed_debug_lcp (engine 3), which runs only that kernel."""
    import numpy as np
    import torch
    import synth
    out = []
    for bits, dist in ((2, synth.CharDist("uniform", 4)), (8, synth.CharDist("zipf", 256))):
        A = synth.random_string(n, dist, 7)
        B = A.copy()
        B[n - 1] = (int(B[n - 1]) + 1) % dist.sigma  # the single mismatch: LCP(0, 0) = n - 1
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        del A, B
        byts = 2 * (n - 1) * bits / 8
        row = {"bits_per_char": bits, "lcp_chars": n - 1, "bytes": byts}
        for name, flags in (("in_path_grid_rounds", ed.FLAG_TIMING),
                            ("in_path_workgroup_tier", ed.FLAG_TIMING | ed.FLAG_NO_GRID_ROUNDS)):
            ctx = ed.ed_init(0, pack_bits=bits, flags=flags)
            p = ed.ed_prepare(ctx, tA, tB)
            best = None
            for _ in range(3):
                k = ed.ed_distance(ctx, p)
                if k != 1:
                    raise SystemExit("lcp leg: distance %d, want 1" % k)
                ns = ed.ed_pair_stats(p)["gpu_ns_frontier_kernel"]
                best = ns if best is None else min(best, ns)
            row[name] = {"frontier_kernel_ms": round(best / 1e6, 4), "achieved_GBs": round(byts / best, 1),
                         "frac_of_hbm_peak": round(byts / best / PEAK_HBM_GBS, 4)}
            ed.ed_release(p)
            ed.ed_shutdown(ctx)
        ctx = ed.ed_init(0, pack_bits=bits, flags=ed.FLAG_TIMING)
        p = ed.ed_prepare(ctx, tA, tB)
        del tA, tB
        ed.ed_debug_lcp(ctx, p, [0], [0], engine=3)  # warm-up
        best = None
        for _ in range(3):
            got = ed.ed_debug_lcp(ctx, p, [0], [0], engine=3)
            ns = ed.ed_pair_stats(p)["gpu_ns_lcp_kernel"]
            best = ns if best is None else min(best, ns)
        if int(got[0]) != n - 1:
            raise SystemExit("grid LCP returned %d, want %d" % (int(got[0]), n - 1))
        row["microbenchmark_grid_query_kernel"] = {
            "kernel_ms": round(best / 1e6, 4), "achieved_GBs": round(byts / best, 1),
            "frac_of_hbm_peak": round(byts / best / PEAK_HBM_GBS, 4)}
        out.append(row)
        ed.ed_release(p)
        ed.ed_shutdown(ctx)
        torch.cuda.empty_cache()
    return out


def table_leg(ed, n=10 ** 9, k=1000, reps=3):
    """Prefix-table build at 8 bits per character: the n = 1e9 Zipf(1.0) pair
    over 256 symbols (k = 1000 planted edits, seed 0), hash engine, b = 32.
    At b = 32 the block hashes are taken by the pack kernel from the input
    bytes it reads anyway, so the table build is measured as the whole
    prepare: algorithmic bytes = the input read once, the 8-bit copy and the
    tables written.  Beside it the prepare of the same pair without tables
    (direct engine) and the table passes that run after the pack kernel
    (scan of the tile hashes, emission of the prefixes)."""
    import torch
    import synth
    log("table leg: generating the n=%d Zipf pair" % n)
    A, B, _ = synth.single_pair(n, k, 0, kind="zipf")
    lens = (len(A), len(B))
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    del A, B

    def best_of(engine):
        ctx = ed.ed_init(0, engine=engine, flags=ed.FLAG_TIMING)
        best = None
        for _ in range(reps + 1):
            p = ed.ed_prepare(ctx, tA, tB)
            st = ed.ed_pair_stats(p)
            ed.ed_release(p)
            cur = (st["gpu_ns_prepare_kernel"], st["gpu_ns_table_kernel"], st["bits_per_char"])
            best = cur if best is None or cur[0] < best[0] else best
        ed.ed_shutdown(ctx)
        return best

    with_t = best_of(ed.ENGINE_HASH)
    without = best_of(ed.ENGINE_DIRECT)
    del tA, tB
    torch.cuda.empty_cache()
    pbytes = sum(2 * L + 8 * (L // 32 + 1) for L in lens)
    return {"workload": "n=%d Zipf(1.0) over 256 symbols, k=%d, seed 0, hash engine, b=32" % (n, k),
            "bits_per_char": with_t[2],
            "prepare_ms": round(with_t[0] / 1e6, 4), "prepare_bytes": pbytes,
            "prepare_achieved_GBs": round(pbytes / with_t[0], 1),
            "prepare_frac_of_hbm_peak": round(pbytes / with_t[0] / PEAK_HBM_GBS, 4),
            "table_passes_after_pack_ms": round(with_t[1] / 1e6, 4),
            "prepare_without_tables_ms": round(without[0] / 1e6, 4)}


def engine_matrix(ed, dev, ks, want, stream, reps=3):
    """The single pairs on the other engine configurations: the direct engine
    at 8 bits per character, the hash engine with b = 1, and the hash engine's
    block size swept over b = 1 .. 64 at k = 1e5.  Kernel times (HIP events),
    median of `reps` runs; every distance must equal the main run's."""
    def run(ctx, i):
        tA, tB = dev[i]
        best = []
        for _ in range(reps):
            k, st = run_pair(ed, ctx, tA, tB, stream)
            if k != want[i]:
                raise SystemExit("engine matrix: distance %d != %d at k=%d" % (k, want[i], ks[i]))
            best.append((st["gpu_ns_prepare_kernel"] + st["gpu_ns_frontier_kernel"], st))
        best.sort(key=lambda x: x[0])
        st = best[len(best) // 2][1]
        return {"prepare_kernel_ms": round(st["gpu_ns_prepare_kernel"] / 1e6, 4),
                "table_kernel_ms": round(st["gpu_ns_table_kernel"] / 1e6, 4),
                "frontier_kernel_ms": round(st["gpu_ns_frontier_kernel"] / 1e6, 4),
                "bits_per_char": st["bits_per_char"]}

    out = {}
    log("engine matrix: direct 8-bit, hash b=1")
    for name, kw in (("direct_8bit", dict(engine=ed.ENGINE_DIRECT, pack_bits=8)),
                     ("hash_b1", dict(engine=ed.ENGINE_HASH, block=1))):
        ctx = ed.ed_init(0, flags=ed.FLAG_TIMING, **kw)
        out[name] = {str(k): run(ctx, i) for i, k in enumerate(ks)}
        ed.ed_shutdown(ctx)
    log("engine matrix: hash block sweep at k=1e5")
    i = ks.index(100000)
    sweep = {}
    for b in (1, 2, 4, 8, 16, 32, 64):
        ctx = ed.ed_init(0, engine=ed.ENGINE_HASH, block=b, flags=ed.FLAG_TIMING)
        sweep[str(b)] = run(ctx, i)
        ed.ed_shutdown(ctx)
    out["hash_block_sweep_k1e5"] = sweep
    return out


def paper_shape_leg(ed, stream, reps=3):
    """The paper's own synthetic workload: n = 1e8 characters uniform over 256
    symbols, B = A + k planted edits, k = 1e2 .. 1e5 (seed 0), 8 bits per
    character, both engines (hash: b = 32, as the paper's BFS-B-Hash).  Kernel
    times (prepare + frontier, median of `reps`) beside the paper's full-run
    times for the same n and k (its best of BFS-Hash and BFS-B-Hash, 96 cores).
    Distances checked against the stored oracle values."""
    import torch
    import synth
    gold = stored_oracle()
    want = {g["k"]: g["ed"] for g in gold["paper"]} if gold and "paper" in gold else {}
    ctxs = {"direct": ed.ed_init(0, engine=ed.ENGINE_DIRECT, flags=ed.FLAG_TIMING),
            "hash": ed.ed_init(0, engine=ed.ENGINE_HASH, flags=ed.FLAG_TIMING)}
    out = {}
    for k in KS:
        log("paper-shape leg: sigma=256 k=%d" % k)
        A, B, _ = synth.single_pair(N, k, 0, sigma=256)
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        del A, B
        row = {}
        for name, ctx in ctxs.items():
            ts = []
            for _ in range(reps):
                kk, st = run_pair(ed, ctx, tA, tB, stream)
                if k in want and kk != want[k]:
                    raise SystemExit("paper-shape leg: %s k=%d gave %d, oracle %d" % (name, k, kk, want[k]))
                ts.append((st["gpu_ns_prepare_kernel"] + st["gpu_ns_frontier_kernel"]) / 1e9)
            row[name + "_s"] = sorted(ts)[len(ts) // 2]
            row["ed"] = kk
        paper = min(PAPER_N1E8_SECONDS[k].values())
        best = min(row["direct_s"], row["hash_s"])
        row.update({"paper_s": paper, "paper_over_this": round(paper / best, 1),
                    "equal_to_stored_oracle": (row["ed"] == want[k]) if k in want else None})
        out[str(k)] = row
        del tA, tB
        torch.cuda.empty_cache()
    for c in ctxs.values():
        ed.ed_shutdown(c)
    return {"workload": "n=1e8 uniform over 256 symbols, B = A + k planted edits, seed 0, 8 bits per character",
            "paper_hardware": "96 cores (4x Intel Xeon Gold 6252), its best of BFS-Hash and BFS-B-Hash, "
                              "Monte Carlo hashing", "per_k": out}


def align_leg(ed, dev, ks, want, stream, only=(1000, 10000, 100000)):
    """Checked (certified) hash-engine results: ed_align on the single pairs
    (hash engine, b = 32): k, the edit script traced back, and every run of
    matches re-compared; wall time against the plain ed_distance, first on a
    pair whose k is known from that distance (one launch keeps the cone of rows
    the path can reach, when it fits an eighth of the free device memory), then
    on a fresh pair (segments: the row at every S-th round kept, k computed by
    the segments' launches, each segment run again with the rows kept for the
    diagonals the path can reach)."""
    ctx = ed.ed_init(0, engine=ed.ENGINE_HASH)
    out = {}
    for i, k in enumerate(ks):
        if k not in only:
            continue
        tA, tB = dev[i]
        log("align leg: k=%d" % k)
        p = ed.ed_prepare(ctx, tA, tB, stream=stream)
        t0 = time.perf_counter()
        kd = ed.ed_distance(ctx, p, stream=stream)
        td = time.perf_counter() - t0
        t0 = time.perf_counter()
        ka, script = ed.ed_align(ctx, p, stream=stream)
        ta = time.perf_counter() - t0
        st = ed.ed_pair_stats(p)
        ed.ed_release(p)
        p = ed.ed_prepare(ctx, tA, tB, stream=stream)
        t0 = time.perf_counter()
        kf, _ = ed.ed_align(ctx, p, stream=stream)
        tf = time.perf_counter() - t0
        ed.ed_release(p)
        edits = sum(L for op, L in script if op != ed.OP_MATCH)
        if not (kd == ka == kf == want[i] == edits):
            raise SystemExit("align leg: k=%d distance %d align %d/%d edits %d want %d" % (k, kd, ka, kf, edits,
                                                                                          want[i]))
        out[str(k)] = {"ed": ka, "script_runs": len(script), "distance_ms": round(td * 1e3, 3),
                       "align_after_distance_ms": round(ta * 1e3, 3), "align_fresh_pair_ms": round(tf * 1e3, 3),
                       "segment_rounds": st["align_segment_rounds"], "device_bytes": st["align_device_bytes"],
                       "every_row_bytes": (ka + 1) ** 2 * 4, "checked": True}
    ed.ed_shutdown(ctx)
    return out


def serve_leg(ed, ctx, count, seed=0, warmup=0):
    """Served workload: Poisson arrivals, n = floor(10^U), U ~ U[2, 7], alphabet 4
    or 20, k ~ U{0..floor(0.05 n)}.  The arrival rate is 0.7x the batched
    throughput measured on the same requests.  Latency = completion - arrival."""
    import threading
    import numpy as np
    import synth
    log("serve leg: generating %d requests" % count)
    trace = synth.arrival_trace(count, seed, rate_per_s=1.0)
    reqs = [synth.request_pair(r) for r in trace]
    gaps = np.diff([0.0] + [r["t_arrive_s"] for r in trace])
    pairs = [ed.ed_prepare(ctx, A, B) for A, B in reqs]
    t0 = time.perf_counter()
    want, _ = ed.ed_batch(ctx, pairs)
    tb = time.perf_counter() - t0
    for p in pairs:
        ed.ed_release(p)
    rate = 0.7 * count / tb
    arrive = np.cumsum(gaps / rate)
    log("serve leg: batched %.1f pairs/s -> arrival rate %.1f /s" % (count / tb, rate))

    def pct(lat):
        lat = np.sort(np.asarray(lat))
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    # served: a submitter thread follows the trace, the server batches
    srv = ed.ed_serve_open(ctx, 64 << 30, 256)
    start = time.perf_counter()

    def submit():
        for i, (A, B) in enumerate(reqs):
            d = start + arrive[i] - time.perf_counter()
            if d > 0:
                time.sleep(d)
            ed.ed_serve_submit(srv, A, B, i)

    th = threading.Thread(target=submit)
    th.start()
    th.join()
    ed.ed_serve_drain(srv)
    res = ed.ed_serve_poll(srv, count + 1)
    ed.ed_serve_close(srv)
    got = {r["tag"]: r["k"] for r in res}
    if [got[i] for i in range(count)] != list(want):
        raise SystemExit("served distances differ from the batch")
    lat = [(r["t_done_ns"] - r["t_arrive_ns"]) / 1e9 for r in res]
    span = (max(r["t_done_ns"] for r in res) - min(r["t_arrive_ns"] for r in res)) / 1e9
    p50, p99 = pct(lat)
    gold = stored_oracle()
    exact = None
    if gold and gold["serve"]["count"] == count and gold["serve"]["seed"] == seed:
        exact = list(want) == gold["serve"]["eds"]
        if not exact:
            raise SystemExit("served distances differ from the stored oracle values")
    # per-pair form on the same trace: one request at a time, in arrival order
    start = time.perf_counter()
    lat2 = []
    for i, (A, B) in enumerate(reqs):
        d = start + arrive[i] - time.perf_counter()
        if d > 0:
            time.sleep(d)
        p = ed.ed_prepare(ctx, A, B)
        k = ed.ed_distance(ctx, p)
        ed.ed_release(p)
        if k != want[i]:
            raise SystemExit("per-pair distance differs")
        lat2.append(time.perf_counter() - (start + arrive[i]))
    span2 = time.perf_counter() - start
    q50, q99 = pct(lat2)
    # served latency by n decade and by alphabet
    lat_by_tag = {r["tag"]: (r["t_done_ns"] - r["t_arrive_ns"]) / 1e9 for r in res}
    buckets = {}
    for i, r in enumerate(trace):
        for key in ("n=1e%d" % int(math.log10(max(1, r["n"]))), "sigma=%d" % r["sigma"]):
            buckets.setdefault(key, []).append((lat_by_tag[i], lat2[i]))
    by = {}
    for key in sorted(buckets):
        v = buckets[key]
        s50, s99 = pct([a for a, _ in v])
        p50_, p99_ = pct([b for _, b in v])
        by[key] = {"requests": len(v), "served_p50_s": s50, "served_p99_s": s99,
                   "per_pair_p50_s": p50_, "per_pair_p99_s": p99_}
    return {"workload": "quick check: %d requests, Poisson arrivals, n log-uniform [1e2, 1e7], alphabet 4 or "
                        "20, k uniform [0, 0.05 n], seed %d (the serving workload at its measured size is "
                        "bench.py --serve-full)" % (count, seed),
            "arrival_rate_per_s": rate, "batched_pairs_per_s": count / tb,
            "served": {"pairs_per_s": count / span, "p50_s": p50, "p99_s": p99},
            "per_pair": {"pairs_per_s": count / span2, "p50_s": q50, "p99_s": q99},
            "latency_by_bucket": by,
            "equal_to_stored_oracle": exact}


def serve_full(ed, seeds=(0, 1, 2), sigmas=(4, 20), count=2200, warmup=200, per_pair_seeds=(0,)):
    """The serving workload at its measured size: for each alphabet (4, 20) and
    trace seed, `count` requests (Poisson arrivals, n log-uniform in [1e2, 1e7],
    k uniform in [0, 0.05 n]), the first `warmup` of them excluded from the
    latency and throughput figures.  The arrival rate is 0.7x the batched
    throughput of the seed-0 trace of the alphabet (ed_batch over all its
    requests, prepared).  Served (continuous batching) on every trace; the
    per-pair form (one request at a time, prepare + ed_distance) on the same
    arrival times for the seeds in per_pair_seeds.  Every sampled request is
    compared with the stored oracle value, the others with the bounds of their
    planted edits."""
    import threading
    from concurrent.futures import ThreadPoolExecutor
    import numpy as np
    import synth
    gold = stored_oracle() or {}
    traces = {(t["sigma"], t["seed"]): t for t in gold.get("serve_trace", [])}
    ctx = ed.ed_init(0, engine=ed.ENGINE_DIRECT)
    out = {"workload": "%d requests per trace (%d warm-up), Poisson arrivals, n log-uniform [1e2, 1e7], "
                       "k uniform [0, 0.05 n], one alphabet per trace" % (count, warmup), "runs": []}

    def pct(lat):
        lat = np.asarray(lat)
        return float(np.percentile(lat, 50)), float(np.percentile(lat, 99))

    def check(sigma, seed, trace, reqs, got):
        t = traces.get((sigma, seed))
        if t is None or t["count"] != count:
            return None
        want = dict(zip(t["index"], t["eds"]))
        for i, (A, B) in enumerate(reqs):
            if i in want and got[i] != want[i]:
                raise SystemExit("serve: request %d of sigma=%d seed=%d: %d, oracle %d" % (i, sigma, seed, got[i], want[i]))
            if not (abs(len(A) - len(B)) <= got[i] <= trace[i]["k"]):
                raise SystemExit("serve: request %d outside its planted-edit bounds" % i)
        return {"sampled_equal_to_oracle": len(want), "bounded": count - len(want)}

    for sigma in sigmas:
        rate = None
        for seed in seeds:
            trace = synth.arrival_trace(count, seed, rate_per_s=1.0, sigmas=(sigma,))
            log("serve full: sigma=%d seed=%d generating" % (sigma, seed))
            with ThreadPoolExecutor(8) as ex:
                reqs = list(ex.map(synth.request_pair, trace))
            if rate is None:
                pairs = [ed.ed_prepare(ctx, A, B) for A, B in reqs]
                t0 = time.perf_counter()
                ed.ed_batch(ctx, pairs)
                tb = time.perf_counter() - t0
                for p in pairs:
                    ed.ed_release(p)
                batched = count / tb
                rate = 0.7 * batched
                log("serve full: sigma=%d batched %.1f pairs/s -> arrival rate %.1f /s" % (sigma, batched, rate))
            gaps = np.diff([0.0] + [r["t_arrive_s"] for r in trace])
            arrive = np.cumsum(gaps / rate)
            # served
            srv = ed.ed_serve_open(ctx, 128 << 30, 256)
            start = time.perf_counter()

            def submit():
                for i, (A, B) in enumerate(reqs):
                    d = start + arrive[i] - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    ed.ed_serve_submit(srv, A, B, i)

            th = threading.Thread(target=submit)
            th.start()
            th.join()
            ed.ed_serve_drain(srv)
            res = ed.ed_serve_poll(srv, count + 1)
            ed.ed_serve_close(srv)
            if len(res) != count or any(r["status"] != 0 for r in res):
                raise SystemExit("serve full: a request failed")
            got = {r["tag"]: r["k"] for r in res}
            exact = check(sigma, seed, trace, reqs, got)
            meas = [r for r in res if r["tag"] >= warmup]
            lat = [(r["t_done_ns"] - r["t_arrive_ns"]) / 1e9 for r in meas]
            span = (max(r["t_done_ns"] for r in meas) - min(r["t_arrive_ns"] for r in meas)) / 1e9
            p50, p99 = pct(lat)
            run = {"sigma": sigma, "seed": seed, "arrival_rate_per_s": round(rate, 2),
                   "served": {"pairs_per_s": round((count - warmup) / span, 2), "p50_s": p50, "p99_s": p99},
                   "exactness": exact}
            if seed in per_pair_seeds:
                start = time.perf_counter()
                lat2, done_t = [], []
                for i, (A, B) in enumerate(reqs):
                    d = start + arrive[i] - time.perf_counter()
                    if d > 0:
                        time.sleep(d)
                    p = ed.ed_prepare(ctx, A, B)
                    k = ed.ed_distance(ctx, p)
                    ed.ed_release(p)
                    if k != got[i]:
                        raise SystemExit("serve full: per-pair distance differs")
                    now = time.perf_counter()
                    if i >= warmup:
                        lat2.append(now - (start + arrive[i]))
                        done_t.append(now)
                q50, q99 = pct(lat2)
                span2 = max(done_t) - (start + arrive[warmup])
                run["per_pair"] = {"pairs_per_s": round((count - warmup) / span2, 2), "p50_s": q50, "p99_s": q99}
            log("serve full: %s" % json.dumps(run))
            out["runs"].append(run)
    ed.ed_shutdown(ctx)
    return out


def config3_leg(ed, seeds=(0, 1, 2)):
    """The n = 1e9 pairs (Zipf(1.0) over 256 symbols and its period-64
    variant, k in {1e3, 1e5}, seeds 0..2), both engines and the hash engine's
    long-LCP mode, from device-resident inputs: prepare and frontier kernel
    times (HIP events), chars/s over the host wall time, equal to the stored
    oracle values."""
    import torch
    import synth
    gold = stored_oracle() or {}
    want = {(g["periodic"], g["k"], g["seed"]): g["ed"] for g in gold.get("big", [])}
    ctxs = {"direct": ed.ed_init(0, engine=ed.ENGINE_DIRECT, flags=ed.FLAG_TIMING),
            "hash": ed.ed_init(0, engine=ed.ENGINE_HASH, flags=ed.FLAG_TIMING),
            # the long-LCP mode: full prefix tables (b = 1), every slide past the
            # lane stage straight to the hash search
            "hash_long_lcp": ed.ed_init(0, engine=ed.ENGINE_HASH, block=1,
                                        flags=ed.FLAG_TIMING | ed.FLAG_HASH_FIRST)}
    rows = []
    for seed in seeds:
        for periodic in (False, True):
            for k in (1000, 100000):
                A, B, _ = synth.single_pair(10 ** 9, k, seed, sigma=256, kind="zipf", periodic=periodic)
                tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
                del A, B
                for name, ctx in ctxs.items():
                    log("config3: %s k=%d seed=%d %s" % ("periodic" if periodic else "zipf", k, seed, name))
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    p = ed.ed_prepare(ctx, tA, tB)
                    d = ed.ed_distance(ctx, p)
                    wall = time.perf_counter() - t0
                    st = ed.ed_pair_stats(p)
                    ed.ed_release(p)
                    w = want.get((periodic, k, seed))
                    if w is not None and w != d:
                        raise SystemExit("config3: distance %d, oracle %d" % (d, w))
                    rows.append({"kind": "periodic64" if periodic else "zipf", "k_planted": k, "seed": seed,
                                 "engine": name, "ed": d, "equal_to_stored_oracle": None if w is None else True,
                                 "prepare_kernel_ms": round(st["gpu_ns_prepare_kernel"] / 1e6, 3),
                                 "frontier_kernel_ms": round(st["gpu_ns_frontier_kernel"] / 1e6, 3),
                                 "wall_ms": round(wall * 1e3, 3), "chars_per_s": 10 ** 9 / wall,
                                 "collision_bound": st["collision_bound"] if name != "direct" else None})
                del tA, tB
                torch.cuda.empty_cache()
    for c in ctxs.values():
        ed.ed_shutdown(c)
    return {"workload": "n=1e9, Zipf(1.0) over 256 symbols and its period-64 variant, k in {1e3, 1e5}, seeds %s, "
                        "8 bits per character, from device-resident inputs" % list(seeds), "runs": rows}


def paper_grid_leg(ed, reps=3):
    """The paper's synthetic grid (uniform over 256 symbols, n = 1e6 .. 1e9,
    k = 1 .. 1e5) and the stand-ins for its real-data rows (a DNA-like string of
    42.3M characters over 4 symbols; text-like strings over Zipf-256 of 0.56M
    and 6.47M characters), from device-resident inputs, both engines: prepare +
    distance wall time (best of `reps`), every distance equal to the stored
    oracle value, beside the paper's best full-run total where it has one."""
    import torch
    import synth
    gold = stored_oracle() or {}
    specs = ([("grid", g) for g in gold.get("paper_grid", [])] +
             [("grid", g) for g in gold.get("paper", [])] +
             [("shape", g) for g in gold.get("shapes", [])])
    ctxs = {"direct": ed.ed_init(0, engine=ed.ENGINE_DIRECT), "hash": ed.ed_init(0, engine=ed.ENGINE_HASH)}
    rows = []
    for group, g in sorted(specs, key=lambda s: (s[0], s[1]["n"], s[1]["k"])):
        A, B, _ = synth.single_pair(g["n"], g["k"], g["seed"], sigma=g["sigma"], kind=g["kind"])
        tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
        del A, B
        row = {"set": group, "name": g["name"], "n": g["n"], "k_planted": g["k"], "ed": g["ed"]}
        for name, ctx in ctxs.items():
            log("paper grid: %s %s" % (g["name"], name))
            best = None
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                p = ed.ed_prepare(ctx, tA, tB)
                d = ed.ed_distance(ctx, p)
                wall = time.perf_counter() - t0
                ed.ed_release(p)
                if d != g["ed"]:
                    raise SystemExit("paper grid: %s %s distance %d, oracle %d" % (g["name"], name, d, g["ed"]))
                best = wall if best is None else min(best, wall)
            row[name + "_s"] = round(best, 6)
        row["equal_to_stored_oracle"] = True
        if group == "grid":
            ps = PAPER_GRID_SECONDS.get(g["n"], {}).get(g["k"])
            row["paper_s"] = ps
            if ps:
                row["paper_over_this"] = round(ps / min(row["direct_s"], row["hash_s"]), 1)
        rows.append(row)
        del tA, tB
        torch.cuda.empty_cache()
    for c in ctxs.values():
        ed.ed_shutdown(c)
    return {"workload": "uniform over 256 symbols, n in {1e6 .. 1e9}, k in {1, 10, 1e2 .. 1e5}, seed 0; "
                        "DNA-like (42.3M, alphabet 4) and text-like (Zipf-256, 0.56M and 6.47M) pairs with the "
                        "edit counts of the paper's real-data rows; prepare + distance from device-resident "
                        "inputs, best of %d" % reps,
            "paper_hardware": "96 cores (4x Intel Xeon Gold 6252), better of BFS-B-Hash and BFS-Hash, "
                              "Monte Carlo hashing", "runs": rows}


def pair_stats(ed, pair):
    return ed.ed_pair_stats(pair)


def run_pair(ed, ctx, tA, tB, stream):
    pair = ed.ed_prepare(ctx, tA, tB, stream=stream)
    k = ed.ed_distance(ctx, pair, stream=stream)
    st = pair_stats(ed, pair)
    ed.ed_release(pair)
    return k, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--engine", choices=["direct", "hash"], default="direct")
    ap.add_argument("--ks", type=str, default=",".join(str(k) for k in KS))
    ap.add_argument("--n", type=int, default=N)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-other-engine", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4096-pair batch leg")
    ap.add_argument("--no-lcp", action="store_true", help="skip the long-LCP bandwidth leg")
    ap.add_argument("--no-table", action="store_true", help="skip the 8-bit table-build leg")
    ap.add_argument("--no-align", action="store_true", help="skip the checked alignment leg")
    ap.add_argument("--no-paper-shape", action="store_true",
                    help="skip the paper's own workload shape (alphabet 256) leg")
    ap.add_argument("--no-matrix", action="store_true",
                    help="skip the engine matrix (direct 8-bit, hash b=1, hash block sweep)")
    ap.add_argument("--serve", type=int, default=40, metavar="N",
                    help="requests of the serving leg (0 skips it)")
    ap.add_argument("--no-config3", action="store_true", help="skip the n=1e9 Zipf / periodic leg")
    ap.add_argument("--serve-full", action="store_true",
                    help="only the serving workload at its measured size (6 traces of 2200 requests)")
    ap.add_argument("--paper-grid", action="store_true",
                    help="only the paper's synthetic grid and the real-data shapes (stored oracle values)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: --gpus %d is not supported "
              "(pairs shard across GPUs without communication)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if args.calibrate_copy:
        nbytes = 1 << 30
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes_read": nbytes, "calibrate_copy_bytes_written": nbytes,
                          "launches": 3}))
        return
    import synth
    import paper_2306_17461_amd as ed
    if args.serve_full:
        print(json.dumps({"serve_full": serve_full(ed)}))
        return
    if args.paper_grid:
        print(json.dumps({"paper_grid": paper_grid_leg(ed)}))
        return

    ks = [int(x) for x in args.ks.split(",")]
    n = args.n
    log("generating %d pairs, n=%d" % (len(ks), n))
    host = []
    for k in ks:
        A, B, info = synth.single_pair(n, k, 0)
        host.append((A, B, info))
    dev = [(torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()) for A, B, _ in host]
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    engines = {"direct": ed.ENGINE_DIRECT, "hash": ed.ENGINE_HASH}
    ctxs = {name: ed.ed_init(0, engine=e, flags=ed.FLAG_TIMING) for name, e in engines.items()}

    def step(name):
        out = []
        for (tA, tB) in dev:
            out.append(run_pair(ed, ctxs[name], tA, tB, stream))
        return out

    main_engine = args.engine
    for w in range(args.warmup):
        log("warmup", w)
        step(main_engine)

    # K timed steps, each bracketed by synchronisations; the value is taken
    # from the median step (the mean is reported beside it)
    results = []
    times = []
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        results.append(step(main_engine))
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        log("step", s, "done")
    dt = sorted(times)[len(times) // 2]
    dt_mean = sum(times) / len(times)
    value = n * len(ks) / dt

    # per-k summary from the last step
    per_k = {}
    prep_ns = [0.0] * len(ks)
    front_ns = [0.0] * len(ks)
    for r in results:
        for i, (k, st) in enumerate(r):
            prep_ns[i] += st["gpu_ns_prepare_kernel"] / len(results)
            front_ns[i] += st["gpu_ns_frontier_kernel"] / len(results)
    last = results[-1]
    for i, (k, st) in enumerate(last):
        wall = (st["ns_prepare"] + st["ns_distance"]) / 1e6
        per_k[str(ks[i])] = {
            "ed": k, "m": int(host[i][2]["m"]), "bits_per_char": st["bits_per_char"],
            "prepare_kernel_ms": round(prep_ns[i] / 1e6, 4),
            "frontier_kernel_ms": round(front_ns[i] / 1e6, 4),
            "host_wall_ms": round(wall, 4),
            "rounds": st["rounds"], "updates": st["updates"],
            "us_per_round": round(front_ns[i] / 1e3 / max(1, st["rounds"]), 4),
            "updates_per_s": st["updates"] / (front_ns[i] / 1e9) if front_ns[i] else None,
            "lcp_chars": st["lcp_chars"], "wave_lcps": st["wave_lcps"], "wg_lcps": st["wg_lcps"],
            "grid_lcps": st["grid_lcps"],
            # the characters the run's slides matched, read once from each
            # string, over the frontier kernel's time
            "in_path_extension_GBs": round(2 * st["lcp_chars"] * st["bits_per_char"] / 8 / front_ns[i], 3)
            if front_ns[i] else None,
            "rounds_phase_a": st["rounds_phase_a"], "us_phase_a": round(st["us_phase_a"], 2),
            "us_phase_b": round(st["us_phase_b"], 2),
            "chars_per_s": n / (wall / 1e3) if wall else None,
        }

    # dominant kernel of the step, and its roofline (algorithmic bytes)
    tot_prep = sum(prep_ns)
    tot_front = sum(front_ns)
    bits = last[0][1]["bits_per_char"]
    if tot_front >= tot_prep:
        # frontier: compulsory bytes = every character of A and B read once
        # along the optimal path, (n + m) * bits / 8 per launch
        byts = sum((n + host[i][2]["m"]) * bits / 8 for i in range(len(ks))) / len(ks)
        avg_ns = tot_front / len(ks)
        dom = "frontier_kernel"
    else:
        # prepare: n bytes read + packed words (n/4) written per string, plus
        # the table for the hash engine
        byts = 0
        for i in range(len(ks)):
            for L in (n, host[i][2]["m"]):
                byts += L + L * bits / 8 + (8 * (L // 32 + 1) if main_engine == "hash" else 0)
        byts /= len(ks)
        avg_ns = tot_prep / len(ks)
        dom = "prepare_kernel"
    achieved = byts / avg_ns  # bytes/ns = GB/s
    roofline = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 3), "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 6),
                "traffic": measured_traffic(dom, main_engine, ks, n),
                "algorithmic_bytes_per_launch": byts, "avg_launch_ms": round(avg_ns / 1e6, 4)}
    if dom == "frontier_kernel":
        # the latency floor of a round: its LCP loads take their addresses
        # from the previous round's row, one dependent access at least
        lctx = ed.ed_init(0)
        try:
            cold = ed.ed_debug_mem_latency(lctx, 1 << 32, 4000)
            warm = ed.ed_debug_mem_latency(lctx, 1 << 20, 2000, warm=True)
        finally:
            ed.ed_shutdown(lctx)
        big = max(range(len(ks)), key=lambda i: ks[i])
        us_round = per_k[str(ks[big])]["us_per_round"]
        roofline["latency_floor"] = {
            "dependent_access_ns_4GiB_cold": round(cold, 1), "dependent_access_ns_1MiB_warm": round(warm, 1),
            "k": ks[big], "us_per_round": us_round,
            "frac_one_cold_access_per_round": round(cold / 1e3 / us_round, 3)}

    def prep_roofline(engine, prep_ms, table_ms=None):
        """Prepare kernels (pack, [table]) against the HBM peak: algorithmic
        bytes = input read once + packed words written [+ prefix table
        written]; for the hash engine also the time of the table passes after
        the pack kernel."""
        byts = 0
        for i in range(len(ks)):
            for L in (n, host[i][2]["m"]):
                byts += L + L * bits / 8 + (8 * (L // 32 + 1) if engine == "hash" else 0)
        byts /= len(ks)
        avg_ns = sum(prep_ms) / len(prep_ms) * 1e6
        out = {"engine": engine, "bound": "hbm", "achieved": round(byts / avg_ns, 3), "peak": PEAK_HBM_GBS,
               "unit": "GB/s", "frac": round(byts / avg_ns / PEAK_HBM_GBS, 4),
               "algorithmic_bytes_per_call": byts, "avg_ms": round(avg_ns / 1e6, 4)}
        if engine == "hash" and table_ms:
            # the block hashes come from the pack kernel (b = 32): the table
            # build is the whole prepare above; these are the passes after it
            tns = sum(table_ms) / len(table_ms) * 1e6
            out["table_passes_after_pack_ms"] = round(tns / 1e6, 4)
        return out

    table_ms = [st["gpu_ns_table_kernel"] / 1e6 for r in results for _, st in r]
    prepare_roofline = [prep_roofline(main_engine, [x / 1e6 for x in prep_ns], table_ms)]
    gold = stored_oracle()
    exact = None
    if gold and n == N:
        want = {g["k"]: g["ed"] for g in gold["single"] if g["seed"] == 0}
        if all(k in want for k in ks):
            exact = all(last[i][0] == want[ks[i]] for i in range(len(ks)))
            if not exact:
                raise SystemExit("distances differ from the stored oracle values")

    other = None
    if not args.no_other_engine:
        oname = "hash" if main_engine == "direct" else "direct"
        step(oname)
        r = step(oname)
        other = {"engine": oname, "per_k_ms": {}}
        for i, (k, st) in enumerate(r):
            other["per_k_ms"][str(ks[i])] = {
                "ed": k, "prepare_kernel_ms": round(st["gpu_ns_prepare_kernel"] / 1e6, 4),
                "frontier_kernel_ms": round(st["gpu_ns_frontier_kernel"] / 1e6, 4),
                "host_wall_ms": round((st["ns_prepare"] + st["ns_distance"]) / 1e6, 4)}
            if k != last[i][0]:
                raise SystemExit("engines disagree at k=%d: %d vs %d" % (ks[i], k, last[i][0]))
        prepare_roofline.append(prep_roofline(oname, [st["gpu_ns_prepare_kernel"] / 1e6 for _, st in r],
                                              [st["gpu_ns_table_kernel"] / 1e6 for _, st in r]))

    matrix = None
    if not args.no_matrix and n == N and 100000 in ks:
        matrix = engine_matrix(ed, dev, ks, [r[0] for r in last], stream)

    align = None
    if not args.no_align and n == N:
        align = align_leg(ed, dev, ks, [r[0] for r in last], stream)

    paper_shape = None
    if not args.no_paper_shape and n == N:
        paper_shape = paper_shape_leg(ed, stream)

    batch = None
    if not args.no_batch:
        batch = batch_leg(ed, ctxs["direct"], cpu_sample=0 if args.no_cpu else 4096)
    lcp = None
    if not args.no_lcp:
        log("lcp leg: one LCP of 1e9 characters in ed_distance (grid rounds, workgroup tier) and the grid query kernel")
        lcp = lcp_leg(ed)
    table = None
    if not args.no_table:
        table = table_leg(ed)
    config3 = None
    if not args.no_config3 and n == N:
        config3 = config3_leg(ed)
    serve = None
    if args.serve > 0:
        serve = serve_leg(ed, ctxs["direct"], args.serve)

    cpu = None
    if not args.no_cpu:
        import oracle
        log("cpu baseline (oracle lv_omp) on the same %d pairs" % len(ks))
        runs = []
        for rep in range(3):
            t1 = time.perf_counter()
            for i, (A, B, _) in enumerate(host):
                kc = oracle.lv_omp(A, B)
                if kc != last[i][0]:
                    raise SystemExit("GPU %d != oracle %d at k=%d" % (last[i][0], kc, ks[i]))
            runs.append(time.perf_counter() - t1)
        tc = sorted(runs)[1]
        cpu = {"value": n * len(ks) / tc, "unit": "chars/s", "cores": oracle.omp_max_threads(),
               "kind": "oracle",
               "sample": "oracle lv_omp (OpenMP Landau-Vishkin, 8-byte word LCP) on the same %d "
                         "pairs, median of 3 runs, %.1f s each" % (len(ks), tc),
               "host": host_cpu()}
        # the literal sequential Landau-Vishkin (character-by-character LCP), one thread:
        # the 10,000-character pair with 100 planted edits, and the n = 1e8 pairs with k <= 1e3
        naive = {}
        A1, B1, _ = synth.small_pair(0)
        t1 = time.perf_counter()
        k1 = oracle.lv_naive(A1, B1)
        naive["n1e4_k100"] = {"ed": k1, "s": round(time.perf_counter() - t1, 4)}
        for i, k in enumerate(ks):
            if k <= 1000:
                t1 = time.perf_counter()
                kc = oracle.lv_naive(host[i][0], host[i][1])
                if kc != last[i][0]:
                    raise SystemExit("GPU %d != lv_naive %d at k=%d" % (last[i][0], kc, k))
                naive["n1e8_k%d" % k] = {"ed": kc, "s": round(time.perf_counter() - t1, 3)}
        cpu["lv_naive_single_thread"] = naive

    for c in ctxs.values():
        ed.ed_shutdown(c)

    line = {
        "metric": "chars/sec at n=1e8, k=1e2..1e5 (exact); batched pairs/sec + p50/p99 latency",
        "value": value, "unit": "chars/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dt * 1e3, "ms_per_step_mean": dt_mean * 1e3, "timing": "median of the timed steps",
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8", "data": "synthetic",
        "config": {"workload": "single pairs n=1e8, alphabet {0,1,2,3} uniform, B = A + k planted "
                               "uniform edits, k in %s, seed 0, one launch per pair" % ks,
                   "engine": main_engine, "bits_per_char": bits},
        "per_k": per_k,
        "equal_to_stored_oracle": exact,
        "roofline": roofline,
        "prepare_roofline": prepare_roofline,
        "cpu_baseline": cpu,
        "paper_context": paper_context(ks, n),
        "paper_shape": paper_shape,
        "other_engine": other,
        "engine_matrix": matrix,
        "align_checked": align,
        "batch": batch,
        "lcp_extension": lcp,
        "table_build_8bit": table,
        "config3_n1e9": config3,
        "serve_quick": serve,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
