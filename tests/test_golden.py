"""The stored full-size oracle values and the input generators they rest on.

`tests/golden/fullsize.json` holds oracle distances of the full-size workloads
(written by `tests/golden/make_golden.py`).  These CPU tests recompute a cheap
part of it with the oracle, so a stale file or a change in the generators
fails here before any GPU comparison uses it.
"""
import json
import os

import numpy as np
import pytest

import synth

GOLD_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize.json")


@pytest.fixture(scope="module")
def gold():
    with open(GOLD_PATH) as f:
        return json.load(f)


def test_golden_file_complete(gold):
    seeds = (0, 1, 2)
    assert sorted((g["seed"], g["k"]) for g in gold["single"]) == [
        (s, k) for s in seeds for k in (100, 1000, 10000, 100000)]
    assert all(g["n"] == 10 ** 8 and g["sigma"] == 4 for g in gold["single"])
    assert sorted((g["seed"], g["periodic"], g["k"]) for g in gold["big"]) == [
        (s, p, k) for s in seeds for p in (False, True) for k in (1000, 100000)]
    assert all(g["n"] == 10 ** 9 and g["kind"] == "zipf" for g in gold["big"])
    assert [g["k"] for g in gold["paper"]] == [100, 1000, 10000, 100000]
    assert all(g["n"] == 10 ** 8 and g["sigma"] == 256 and g["kind"] == "uniform" for g in gold["paper"])
    assert sorted((g["n"], g["k"]) for g in gold["paper_grid"]) == sorted(
        (10 ** e, k) for e in (6, 7, 8, 9) for k in (1, 10, 100, 1000, 10000, 100000)
        if not (e == 8 and k >= 100))
    assert all(g["sigma"] == 256 and g["kind"] == "uniform" and g["seed"] == 0 for g in gold["paper_grid"])
    assert sorted((g["n"], g["k"]) for g in gold["shapes"]) == sorted(
        [(42_300_000, k) for k in (928, 9162, 91419)] + [(560_000, k) for k in (439, 5578, 15026)] +
        [(6_470_000, k) for k in (236, 1447, 9559)])
    assert [(g["n"], g["k"]) for g in gold["maxlen"]] == [(2 ** 31 - 2 ** 20 - 64, 10)]
    assert all(g["n"] < 2 ** 31 - 2 ** 20 and g["m"] < 2 ** 31 - 2 ** 20 for g in gold["maxlen"])
    assert [b["seed"] for b in gold["batch"]] == list(seeds)
    assert all(len(b["eds"]) == b["count"] == 4096 for b in gold["batch"])
    assert len(gold["serve"]["eds"]) == gold["serve"]["count"] == 40
    assert sorted((t["sigma"], t["seed"]) for t in gold["serve_trace"]) == [
        (sg, s) for sg in (4, 20) for s in seeds]
    for t in gold["serve_trace"]:
        assert t["count"] >= 2200 and t["warmup"] == 200 and len(t["index"]) == len(t["eds"])
    # distance bounds of planted edits: |n - m| <= ED <= k
    for g in gold["single"] + gold["big"] + gold["paper"] + gold["paper_grid"] + gold["shapes"] + gold["maxlen"]:
        assert abs(g["n"] - g["m"]) <= g["ed"] <= g["k_planted"]


def _trace_entry(gold, sigma, seed):
    return next(t for t in gold["serve_trace"] if t["sigma"] == sigma and t["seed"] == seed)


@pytest.mark.parametrize("sigma", [4, 20])
def test_serve_trace_sample_rule(gold, sigma):
    """The stored sample is the rule of make_golden.py: every request with
    k_planted <= small_k, plus large_pick larger ones, half of them from the
    upper half of the larger k."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_golden", os.path.join(os.path.dirname(GOLD_PATH), "make_golden.py"))
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    t = _trace_entry(gold, sigma, 0)
    trace, idx = mg.trace_sample(t)
    assert idx == t["index"]
    ks = sorted(r["k"] for r in trace if r["k"] > t["small_k"])
    picked = [trace[i]["k"] for i in idx if trace[i]["k"] > t["small_k"]]
    assert len(picked) == t["large_pick"]
    assert sum(k >= ks[len(ks) // 2] for k in picked) >= t["large_pick"] // 2
    for i, e in zip(t["index"], t["eds"]):
        r = trace[i]
        assert e <= r["k"]


@pytest.mark.parametrize("sigma", [4, 20])
def test_serve_trace_small_requests_recomputed(gold, orc, sigma):
    t = _trace_entry(gold, sigma, 1)
    trace = synth.arrival_trace(t["count"], t["seed"], rate_per_s=1.0, sigmas=(sigma,))
    got = dict(zip(t["index"], t["eds"]))
    small = [i for i in t["index"] if trace[i]["n"] <= 20000][:40]
    assert len(small) >= 20
    for i in small:
        A, B = synth.request_pair(trace[i])
        assert orc.lv_omp(A, B, -1, 1) == got[i], i


@pytest.mark.parametrize("idx", [0, 1])
def test_single_pairs_recomputed(gold, orc, idx):
    g = gold["single"][idx]
    A, B, info = synth.single_pair(g["n"], g["k"], g["seed"], sigma=g["sigma"], kind=g["kind"],
                                   periodic=g["periodic"])
    assert len(B) == g["m"] and info["k_planted"] == g["k_planted"]
    assert orc.lv_omp(A, B) == g["ed"]


@pytest.mark.parametrize("group,name", [("paper_grid", "n1e6_sigma256_k1000"), ("shapes", "wiki_like_k439")])
def test_grid_and_shape_entries_recomputed(gold, orc, group, name):
    g = next(e for e in gold[group] if e["name"] == name)
    A, B, info = synth.single_pair(g["n"], g["k"], g["seed"], sigma=g["sigma"], kind=g["kind"])
    assert len(B) == g["m"] and info["k_planted"] == g["k_planted"]
    assert orc.lv_omp(A, B) == g["ed"]


def test_paper_shape_recomputed(gold, orc):
    g = gold["paper"][0]
    A, B, info = synth.single_pair(g["n"], g["k"], g["seed"], sigma=g["sigma"], kind=g["kind"])
    assert len(B) == g["m"] and info["k_planted"] == g["k_planted"]
    assert orc.lv_omp(A, B) == g["ed"]


@pytest.mark.parametrize("which", [0, 2])
def test_batch_prefix_recomputed(gold, orc, which):
    b = gold["batch"][which]
    specs = synth.batch_specs(b["count"], b["seed"])
    for i in range(64):
        n, k, ps = specs[i]
        A, B, _ = synth.single_pair(n, k, ps)
        assert orc.lv_omp(A, B, -1, 1) == b["eds"][i], i
        assert abs(len(A) - len(B)) <= b["eds"][i] <= k


def test_serve_small_requests_recomputed(gold, orc):
    s = gold["serve"]
    trace = synth.arrival_trace(s["count"], s["seed"], rate_per_s=1.0)
    small = [i for i, r in enumerate(trace) if r["n"] <= 200000]
    assert len(small) >= 10
    for i in small:
        A, B = synth.request_pair(trace[i])
        assert orc.lv_omp(A, B, -1, 1) == s["eds"][i], i


def test_zipf_guide_table_equals_search():
    cdf = synth.zipf_cdf(256, 1.0)
    v = synth.draws(11, synth.S_CHARS, 1 << 20)
    u = synth._unit_float(v)
    want = np.minimum(np.searchsorted(cdf, u, side="right"), 255).astype(np.uint8)
    assert np.array_equal(synth._zipf_from(v, cdf), want)
    edge = np.array([0, 1, 2 ** 64 - 1, 2 ** 63, (5 << 48) - 1, 5 << 48], dtype=np.uint64)
    want = np.minimum(np.searchsorted(cdf, synth._unit_float(edge), side="right"), 255)
    assert np.array_equal(synth._zipf_from(edge, cdf), want.astype(np.uint8))


def test_threaded_sampling_matches_chunks():
    d = synth.CharDist("zipf", 256)
    n = 3 * (1 << 22) + 12345
    whole = d.sample(3, synth.S_CHARS, n)
    part = d.sample(3, synth.S_CHARS, 1000, start=(1 << 22) - 500)
    assert np.array_equal(whole[(1 << 22) - 500:(1 << 22) + 500], part)
