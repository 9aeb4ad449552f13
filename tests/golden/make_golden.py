"""Write tests/golden/fullsize.json: oracle distances of the full-size workloads.

Every value in the file comes from ``oracle.lv_omp`` (multicore Landau-Vishkin,
Algorithm 1 with an 8-byte word LCP) on inputs drawn by ``synth``; nothing here
touches the HIP library.  The full-size GPU tests regenerate the same inputs
from the same seeds and compare the library's distances with these values.

Workloads:
  * single pairs, n = 10^8, alphabet {0,1,2,3} uniform, k in {10^2 .. 10^5},
    seeds 0, 1, 2;
  * single pairs, n = 10^9, Zipf(1.0) over 256 symbols and its period-64
    variant, k in {10^3, 10^5}, seeds 0, 1, 2;
  * the paper's own synthetic shape: n = 10^8 uniform over 256 symbols,
    k in {10^2 .. 10^5}, seed 0 (the workload of its full-run table), and the
    rest of that table's grid: n in {10^6 .. 10^9}, k in {1, 10, 10^2 .. 10^5};
  * stand-ins for the shapes of the paper's real-data table (section 6): a
    DNA-like string (n = 42.3M, alphabet 4 uniform) and text-like ones
    (Zipf(1.0) over 256 symbols, n = 0.56M and 6.47M), each with three
    numbers of planted edits taken from that table;
  * a pair of the longest strings the library accepts (n = 2^31 - 2^20 - 64,
    alphabet 4, 10 planted edits);
  * the 4096-pair batch (n log-uniform in [10^3, 10^6], k uniform in
    [0, 0.01 n], alphabet 4), seeds 0, 1, 2;
  * the first 40 requests of the mixed-alphabet serving trace (n log-uniform
    in [10^2, 10^7], alphabet 4 or 20, k uniform in [0, 0.05 n]), seed 0;
  * the serving traces at their measured size: 2200 requests (200 warm-up +
    2000), one alphabet per trace (4 or 20), seeds 0, 1, 2.  The oracle takes
    about 2 hours of 8 cores per trace in full (the sum of k^2 is about
    8e12 diagonal updates), so a sample is stored: every request with
    k_planted <= SERVE_SMALL_K, plus SERVE_LARGE_PICK larger requests chosen
    by a seeded draw (stratified: the largest ones are represented).  The
    GPU test checks every sampled request against these values and the rest
    against properties that hold at any size.

Entries already in the file with the same specification are kept (the
script only computes what is missing); --force recomputes everything.

Usage: python tests/golden/make_golden.py [--only single|big|paper|grid|shapes|maxlen|batch|serve|trace] [--force]
(the single pairs at n = 10^9 need ~10 GB of RAM).
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")
SEEDS = (0, 1, 2)


def _sfx(seed):
    return "" if seed == 0 else "_seed%d" % seed


SINGLE = [dict(name="n1e8_sigma4_k%d%s" % (k, _sfx(s)), n=10 ** 8, k=k, seed=s, kind="uniform", sigma=4,
               periodic=False) for s in SEEDS for k in (100, 1000, 10000, 100000)]
BIG = [dict(name="n1e9_zipf%s_k%d%s" % ("_periodic" if p else "", k, _sfx(s)), n=10 ** 9, k=k, seed=s,
            kind="zipf", sigma=256, periodic=p) for s in SEEDS for p in (False, True) for k in (1000, 100000)]
PAPER = [dict(name="n1e8_sigma256_k%d" % k, n=10 ** 8, k=k, seed=0, kind="uniform", sigma=256,
              periodic=False) for k in (100, 1000, 10000, 100000)]
PAPER_GRID = [dict(name="n1e%d_sigma256_k%d" % (e, k), n=10 ** e, k=k, seed=0, kind="uniform", sigma=256,
                   periodic=False) for e in (6, 7, 8, 9) for k in (1, 10, 100, 1000, 10000, 100000)
              if not (e == 8 and k >= 100)]
# sizes and edit counts of the real-data table's rows (section 6); synthetic strings of those shapes
SHAPES = ([dict(name="dna_like_k%d" % k, n=42_300_000, k=k, seed=0, kind="uniform", sigma=4, periodic=False)
           for k in (928, 9162, 91419)] +
          [dict(name="wiki_like_k%d" % k, n=560_000, k=k, seed=0, kind="zipf", sigma=256, periodic=False)
           for k in (439, 5578, 15026)] +
          [dict(name="linux_like_k%d" % k, n=6_470_000, k=k, seed=0, kind="zipf", sigma=256, periodic=False)
           for k in (236, 1447, 9559)])
# the longest strings the library accepts (both below 2^31 - 2^20 characters)
MAXLEN = [dict(name="maxlen_sigma4_k10", n=2 ** 31 - 2 ** 20 - 64, k=10, seed=0, kind="uniform", sigma=4,
               periodic=False)]
BATCH = [dict(name="batch4096_seed%d" % s, count=4096, seed=s) for s in SEEDS]
SERVE = dict(name="serve40_seed0", count=40, seed=0)
TRACE_COUNT = 2200
TRACE_WARMUP = 200
SERVE_SMALL_K = 30000
SERVE_LARGE_PICK = 8
TRACES = [dict(name="serve%d_sigma%d_seed%d" % (TRACE_COUNT, sg, s), count=TRACE_COUNT, warmup=TRACE_WARMUP,
               seed=s, sigma=sg, small_k=SERVE_SMALL_K, large_pick=SERVE_LARGE_PICK)
          for sg in (4, 20) for s in SEEDS]


def log(*a):
    print(*a, flush=True)


def threads():
    return max(1, os.cpu_count() or 1)


def single(spec):
    t0 = time.time()
    A, B, info = synth.single_pair(spec["n"], spec["k"], spec["seed"], sigma=spec["sigma"],
                                   kind=spec["kind"], periodic=spec["periodic"])
    ed = oracle.lv_omp(A, B, -1, threads())
    dt = time.time() - t0
    out = dict(spec, m=len(B), ed=ed, k_planted=info["k_planted"], oracle_s=round(dt, 1))
    log("%-34s m=%d ed=%d (%.1f s)" % (spec["name"], len(B), ed, dt))
    return out


def many(pairs_of, count, name):
    """Oracle distances of `count` pairs, one single-threaded oracle per worker
    (ctypes releases the GIL during the call)."""
    t0 = time.time()

    def one(i):
        A, B = pairs_of(i)
        return oracle.lv_omp(A, B, -1, 1)

    with ThreadPoolExecutor(threads()) as ex:
        eds = list(ex.map(one, range(count)))
    log("%-34s %d pairs (%.1f s)" % (name, count, time.time() - t0))
    return eds, time.time() - t0


def batch(spec):
    specs = synth.batch_specs(spec["count"], spec["seed"])

    def pairs_of(i):
        n, k, ps = specs[i]
        A, B, _ = synth.single_pair(n, k, ps)
        return A, B

    eds, dt = many(pairs_of, spec["count"], spec["name"])
    return dict(spec, eds=eds, oracle_s=round(dt, 1))


def serve(spec):
    trace = synth.arrival_trace(spec["count"], spec["seed"], rate_per_s=1.0)
    eds, dt = many(lambda i: synth.request_pair(trace[i]), spec["count"], spec["name"])
    return dict(spec, eds=eds, oracle_s=round(dt, 1))


def trace_sample(spec):
    """Indices of a serving trace whose oracle values are stored: every request
    with k_planted <= small_k, and large_pick of the others, drawn with the
    trace's seed (half from the upper half of the larger k, half from the lower
    half, so that the heaviest requests are represented)."""
    trace = synth.arrival_trace(spec["count"], spec["seed"], rate_per_s=1.0, sigmas=(spec["sigma"],))
    small = [i for i, r in enumerate(trace) if r["k"] <= spec["small_k"]]
    large = sorted((i for i, r in enumerate(trace) if r["k"] > spec["small_k"]), key=lambda i: trace[i]["k"])
    half = len(large) // 2
    draws = synth.draws(spec["seed"] + 1000 * spec["sigma"], synth.S_REQ_SEED, spec["large_pick"])
    pick = []
    for j in range(spec["large_pick"]):
        lo, hi = (half, len(large)) if j % 2 == 0 else (0, half)
        pool = [i for i in large[lo:hi] if i not in pick]
        if pool:
            pick.append(pool[int(draws[j] % np.uint64(len(pool)))])
    return trace, sorted(small + pick)


def serve_trace(spec):
    trace, idx = trace_sample(spec)
    t0 = time.time()
    small = [i for i in idx if trace[i]["k"] <= spec["small_k"]]
    large = [i for i in idx if trace[i]["k"] > spec["small_k"]]
    got = {}
    with ThreadPoolExecutor(threads()) as ex:
        for i, e in zip(small, ex.map(lambda i: oracle.lv_omp(*synth.request_pair(trace[i]), -1, 1), small)):
            got[i] = e
    for i in large:
        t1 = time.time()
        got[i] = oracle.lv_omp(*synth.request_pair(trace[i]), -1, threads())
        log("  %s request %d: n=%d k=%d ed=%d (%.1f s)" % (spec["name"], i, trace[i]["n"], trace[i]["k"],
                                                          got[i], time.time() - t1))
    dt = time.time() - t0
    log("%-34s %d of %d requests (%.1f s)" % (spec["name"], len(idx), spec["count"], dt))
    return dict(spec, index=idx, eds=[got[i] for i in idx], oracle_s=round(dt, 1), threads=threads())


def _merge(old, specs, fn, force):
    """Entries of `specs`, reusing an old entry with the same specification."""
    have = {g["name"]: g for g in (old or [])}
    out = []
    for s in specs:
        g = have.get(s["name"])
        if g is not None and not force and all(g.get(k) == v for k, v in s.items()):
            out.append(g)
        else:
            out.append(fn(s))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["single", "big", "paper", "grid", "shapes", "maxlen", "batch", "serve",
                                       "trace"])
    ap.add_argument("--force", action="store_true")
    args = ap.parse_args()
    oracle.build(force=False)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    if isinstance(data.get("batch"), dict):  # older single-seed layout
        data["batch"] = [data["batch"]]
    data["source"] = ("oracle.lv_omp on synth inputs; written by tests/golden/make_golden.py")

    def save():
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1)
        os.replace(OUT + ".tmp", OUT)

    if args.only in (None, "single"):
        data["single"] = _merge(data.get("single"), SINGLE, single, args.force)
        save()
    if args.only in (None, "big"):
        data["big"] = _merge(data.get("big"), BIG, single, args.force)
        save()
    if args.only in (None, "paper"):
        data["paper"] = _merge(data.get("paper"), PAPER, single, args.force)
        save()
    if args.only in (None, "grid"):
        data["paper_grid"] = _merge(data.get("paper_grid"), PAPER_GRID, single, args.force)
        save()
    if args.only in (None, "shapes"):
        data["shapes"] = _merge(data.get("shapes"), SHAPES, single, args.force)
        save()
    if args.only in (None, "maxlen"):
        data["maxlen"] = _merge(data.get("maxlen"), MAXLEN, single, args.force)
        save()
    if args.only in (None, "batch"):
        data["batch"] = _merge(data.get("batch"), BATCH, batch, args.force)
        save()
    if args.only in (None, "serve"):
        data["serve"] = _merge([data["serve"]] if "serve" in data else [], [SERVE], serve, args.force)[0]
        save()
    if args.only in (None, "trace"):
        out = []
        for s in TRACES:
            out = _merge(data.get("serve_trace"), [s], serve_trace, args.force)
            data["serve_trace"] = [g for g in data.get("serve_trace", []) if g["name"] != s["name"]] + out
            save()
    log("wrote", OUT)


if __name__ == "__main__":
    main()
