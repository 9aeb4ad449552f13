"""Write tests/golden/fullsize.json: oracle distances of the full-size workloads.

Every value in the file comes from ``oracle.lv_omp`` (multicore Landau-Vishkin,
Algorithm 1 with an 8-byte word LCP) on inputs drawn by ``synth``; nothing here
touches the HIP library.  The full-size GPU tests regenerate the same inputs
from the same seeds and compare the library's distances with these values.

Workloads:
  * single pairs, n = 10^8, alphabet {0,1,2,3} uniform, k in {10^2 .. 10^5}, seed 0;
  * single pairs, n = 10^9, Zipf(1.0) over 256 symbols and its period-64
    variant, k in {10^3, 10^5}, seed 0;
  * the paper's own synthetic shape: n = 10^8 uniform over 256 symbols,
    k in {10^2 .. 10^5}, seed 0 (the workload of its full-run table);
  * the 4096-pair batch (n log-uniform in [10^3, 10^6], k uniform in
    [0, 0.01 n], alphabet 4), seed 0;
  * the first 40 requests of the serving trace (n log-uniform in [10^2, 10^7],
    alphabet 4 or 20, k uniform in [0, 0.05 n]), seed 0.

Usage: python tests/golden/make_golden.py [--only single|big|paper|batch|serve]
(several minutes on 8 cores; the single pairs at n = 10^9 need ~10 GB of RAM).
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize.json")

SINGLE = [dict(name="n1e8_sigma4_k%d" % k, n=10 ** 8, k=k, seed=0, kind="uniform", sigma=4,
               periodic=False) for k in (100, 1000, 10000, 100000)]
BIG = [dict(name="n1e9_zipf%s_k%d" % ("_periodic" if p else "", k), n=10 ** 9, k=k, seed=0,
            kind="zipf", sigma=256, periodic=p) for p in (False, True) for k in (1000, 100000)]
PAPER = [dict(name="n1e8_sigma256_k%d" % k, n=10 ** 8, k=k, seed=0, kind="uniform", sigma=256,
              periodic=False) for k in (100, 1000, 10000, 100000)]
BATCH = dict(name="batch4096_seed0", count=4096, seed=0)
SERVE = dict(name="serve40_seed0", count=40, seed=0)


def log(*a):
    print(*a, flush=True)


def threads():
    return max(1, os.cpu_count() or 1)


def single(spec):
    t0 = time.time()
    A, B, info = synth.single_pair(spec["n"], spec["k"], spec["seed"], sigma=spec["sigma"],
                                   kind=spec["kind"], periodic=spec["periodic"])
    ed = oracle.lv_omp(A, B, -1, threads())
    out = dict(spec, m=len(B), ed=ed, k_planted=info["k_planted"])
    log("%-28s m=%d ed=%d (%.1f s)" % (spec["name"], len(B), ed, time.time() - t0))
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
    log("%-28s %d pairs (%.1f s)" % (name, count, time.time() - t0))
    return eds


def batch(spec):
    specs = synth.batch_specs(spec["count"], spec["seed"])

    def pairs_of(i):
        n, k, ps = specs[i]
        A, B, _ = synth.single_pair(n, k, ps)
        return A, B

    return dict(spec, eds=many(pairs_of, spec["count"], spec["name"]))


def serve(spec):
    trace = synth.arrival_trace(spec["count"], spec["seed"], rate_per_s=1.0)
    return dict(spec, eds=many(lambda i: synth.request_pair(trace[i]), spec["count"],
                               spec["name"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", choices=["single", "big", "paper", "batch", "serve"])
    args = ap.parse_args()
    oracle.build(force=False)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data["source"] = ("oracle.lv_omp on synth inputs; written by tests/golden/make_golden.py")
    if args.only in (None, "single"):
        data["single"] = [single(s) for s in SINGLE]
    if args.only in (None, "big"):
        data["big"] = [single(s) for s in BIG]
    if args.only in (None, "paper"):
        data["paper"] = [single(s) for s in PAPER]
    if args.only in (None, "batch"):
        data["batch"] = batch(BATCH)
    if args.only in (None, "serve"):
        data["serve"] = serve(SERVE)
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1)
    os.replace(OUT + ".tmp", OUT)
    log("wrote", OUT)


if __name__ == "__main__":
    main()
