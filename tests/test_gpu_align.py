"""Alignment output and the checked (certified) hash-engine distance.

`ed_align` returns k and an edit script traced back through the frontier rows
(Algorithm 1, section 3.1); every run of matches on it is re-compared on the
device.  The script is checked here independently: applied to A it must give
B, its number of edits must equal the oracle's distance, every substitution
must replace a character by a different one and every match must match.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def ed():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2306_17461_amd as edmod
    return edmod


@pytest.fixture(scope="module")
def make_ctx(ed):
    made = []

    def make(**kw):
        c = ed.ed_init(0, **kw)
        made.append(c)
        return c

    yield make
    for c in made:
        ed.ed_shutdown(c)


def apply_script(ed, A, B, script):
    """Number of edits of the script; asserts that it turns A into B."""
    x = y = edits = 0
    for op, L in script:
        assert L > 0
        if op == ed.OP_MATCH:
            assert np.array_equal(A[x:x + L], B[y:y + L]), "match run at x=%d" % x
            x += L
            y += L
        elif op == ed.OP_SUB:
            assert np.all(A[x:x + L] != B[y:y + L]), "substitution of equal characters at x=%d" % x
            x += L
            y += L
            edits += L
        elif op == ed.OP_DEL:
            x += L
            edits += L
        elif op == ed.OP_INS:
            y += L
            edits += L
        else:
            raise AssertionError("unknown op %d" % op)
    assert x == len(A) and y == len(B)
    return edits


def _cases():
    d4 = synth.CharDist("uniform", 4)
    d256 = synth.CharDist("uniform", 256)
    A, B, _ = synth.single_pair(20000, 150, 3)
    yield "sigma4_planted", A, B
    A, B, _ = synth.single_pair(30000, 50, 4, sigma=256)
    yield "sigma256_planted", A, B
    yield "unrelated_unequal", synth.random_string(3000, d4, 5), synth.random_string(2500, d4, 6)
    P = synth.periodic_string(40000, d4, 7, period=64)
    Q, _ = synth.plant_edits(P, 40, d4, 8)
    yield "periodic", P, Q
    yield "identical", synth.random_string(5000, d256, 9), None
    A = synth.random_string(4097, d4, 10)
    B = A.copy()
    B[4096] ^= 1
    yield "last_char", A, B
    yield "empty_a", np.zeros(0, np.uint8), synth.random_string(37, d4, 11)
    yield "empty_b", synth.random_string(41, d256, 12), np.zeros(0, np.uint8)
    yield "both_empty", np.zeros(0, np.uint8), np.zeros(0, np.uint8)
    yield "one_char", np.array([2], np.uint8), np.array([3], np.uint8)


CASES = list(_cases())


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("pack_bits", [0, 8])
@pytest.mark.parametrize("name", [c[0] for c in CASES])
def test_align_script_is_optimal(ed, make_ctx, orc, engine, pack_bits, name):
    A, B = next((a, b) for n, a, b in CASES if n == name)
    if B is None:
        B = A.copy()
    say("align", name, engine, pack_bits, len(A), len(B))
    ctx = make_ctx(engine=engine, pack_bits=pack_bits)
    want = orc.lv_omp(A, B, -1, 1)
    for first in ("align", "distance"):
        # a fresh pair (segments) and one whose distance is known (the cone of rows)
        p = ed.ed_prepare(ctx, A, B)
        try:
            if first == "distance":
                assert ed.ed_distance(ctx, p) == want
            k, script = ed.ed_align(ctx, p)
        finally:
            ed.ed_release(p)
        assert k == want
        assert apply_script(ed, A, B, script) == k
        # runs are merged: no two neighbours share an operation
        assert all(script[j][0] != script[j + 1][0] for j in range(len(script) - 1))


@pytest.mark.parametrize("block", [1, 32])
def test_certified_hash_distance(ed, make_ctx, orc, block):
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=block, flags=ed.FLAG_CERTIFY)
    for seed in range(4):
        A, B, _ = synth.single_pair(12000, 100 + 40 * seed, 50 + seed)
        say("certify", block, seed)
        p = ed.ed_prepare(ctx, A, B)
        k = ed.ed_distance(ctx, p)
        st = ed.ed_pair_stats(p)
        ed.ed_release(p)
        assert k == orc.lv_omp(A, B, -1, 1)
        assert st["certify_retries"] == 0


def test_align_large_pair_both_engines(ed, make_ctx, orc):
    # 10^6 characters, about 2000 edits: two segments of 1024 rounds between kept rows
    A, B, _ = synth.single_pair(10 ** 6, 2000, 21)
    want = orc.lv_omp(A, B)
    for engine in (0, 1):
        say("align large", engine)
        ctx = make_ctx(engine=engine)
        p = ed.ed_prepare(ctx, A, B)
        k, script = ed.ed_align(ctx, p)
        ed.ed_release(p)
        assert k == want
        assert apply_script(ed, A, B, script) == k


@pytest.mark.parametrize("form", ["auto", "segments"])
@pytest.mark.parametrize("engine", [0, 1])
def test_align_segments_known_and_unknown_k(ed, make_ctx, orc, engine, form):
    # about 5000 edits: 5 segments of 1024 rounds; the path crosses every
    # segment boundary.  Without a distance before, the segments' launches
    # compute k; after one, k is known: the rows of the cone the path can
    # reach are kept in one launch ("auto"), or the segments run with the
    # last forward one skipped ("segments")
    A, B, _ = synth.single_pair(300000, 5000, 23, sigma=4)
    want = orc.lv_omp(A, B)
    ctx = make_ctx(engine=engine, flags=ed.FLAG_ALIGN_SEGMENTS if form == "segments" else 0)
    for first in ("align", "distance"):
        say("align segments", engine, form, first)
        p = ed.ed_prepare(ctx, A, B)
        try:
            if first == "distance":
                assert ed.ed_distance(ctx, p) == want
            k, script = ed.ed_align(ctx, p)
            st = ed.ed_pair_stats(p)
        finally:
            ed.ed_release(p)
        assert k == want
        assert st["rounds"] == want
        assert apply_script(ed, A, B, script) == k
        cone = first == "distance" and form == "auto"
        assert (st["align_segment_rounds"] == want) == cone


def test_align_beyond_every_row_in_memory(ed, make_ctx):
    # about 3e5 edits: every frontier row of every round would take (k + 1)^2
    # int32 = 360 GB, more than the device holds; the kept rows take ~130 MB.
    # The distance is the one of ed_distance (whose full-size values are pinned
    # to the oracle elsewhere), and the script, applied to A, gives B with
    # exactly that many edits.
    A, B, info = synth.single_pair(20_000_000, 300_000, 24, sigma=4)
    ctx = make_ctx(engine=ed.ENGINE_DIRECT)
    say("align k=3e5 distance")
    p = ed.ed_prepare(ctx, A, B)
    want = ed.ed_distance(ctx, p)
    ed.ed_release(p)
    assert abs(len(A) - len(B)) <= want <= info["k_planted"]
    assert want > 250_000
    say("align k=3e5 script")
    p = ed.ed_prepare(ctx, A, B)
    try:
        k, script = ed.ed_align(ctx, p)
    finally:
        ed.ed_release(p)
    assert k == want
    assert apply_script(ed, A, B, script) == k


@pytest.mark.parametrize("pack_bits", [0, 8])
def test_run_check_finds_every_difference(ed, make_ctx, pack_bits):
    # the check itself: equal runs pass; one differing character anywhere in a
    # run (first, inside a word, last, far into a long run) is found; a
    # difference just past a run's end is not counted
    d4 = synth.CharDist("uniform", 4)
    A = synth.random_string(50000, d4, 31)
    B = A.copy()
    ctx = make_ctx(pack_bits=pack_bits)
    p = ed.ed_prepare(ctx, A, B)
    runs = [(0, 0, 50000), (17, 17, 1000), (100, 100, 1), (49999, 49999, 1)]
    assert ed.ed_debug_check_runs(ctx, p, runs) == 0
    ed.ed_release(p)
    for pos in (0, 31, 32, 33, 4095, 20000, 49999):
        B2 = A.copy()
        B2[pos] ^= 1
        p = ed.ed_prepare(ctx, A, B2)
        say("check runs", pack_bits, pos)
        assert ed.ed_debug_check_runs(ctx, p, [(0, 0, 50000)]) == 1
        assert ed.ed_debug_check_runs(ctx, p, [(0, 0, pos)]) == 0  # ends just before
        if pos + 1 < 50000:
            assert ed.ed_debug_check_runs(ctx, p, [(pos + 1, pos + 1, 50000 - pos - 1)]) == 0
        assert ed.ed_debug_check_runs(ctx, p, [(pos, pos, 1)]) == 1
        ed.ed_release(p)
    # shifted runs compare A and B at different offsets
    P = synth.periodic_string(10000, d4, 32, period=64)
    p = ed.ed_prepare(ctx, P, P.copy())
    assert ed.ed_debug_check_runs(ctx, p, [(64, 0, 9000), (0, 128, 9000)]) == 0
    assert ed.ed_debug_check_runs(ctx, p, [(1, 0, 9000)]) == 1
    ed.ed_release(p)


def test_small_buffer_then_retry_returns_the_kept_script(ed, make_ctx, orc):
    import ctypes
    A, B, _ = synth.single_pair(30000, 300, 41)
    ctx = make_ctx(engine=ed.ENGINE_HASH)
    p = ed.ed_prepare(ctx, A, B)
    k = ctypes.c_uint64()
    cnt = ctypes.c_uint64()
    small = (ed.ed_op_run * 1)()
    rc = ed.lib.ed_align(ctx, p, ctypes.byref(k), small, 1, ctypes.byref(cnt), None)
    assert rc == ed.ED_EINVAL and cnt.value > 1 and k.value == orc.lv_omp(A, B, -1, 1)
    runs = (ed.ed_op_run * cnt.value)()
    cnt2 = ctypes.c_uint64()
    assert ed.lib.ed_align(ctx, p, ctypes.byref(k), runs, cnt.value, ctypes.byref(cnt2), None) == ed.ED_OK
    script = [(int(runs[i].op), int(runs[i].len)) for i in range(cnt2.value)]
    assert cnt2.value == cnt.value
    assert apply_script(ed, A, B, script) == k.value
    # a fresh call computes the same script again
    k3, script3 = ed.ed_align(ctx, p)
    assert k3 == k.value and script3 == script
    ed.ed_release(p)


def test_weak_hash_collisions_are_caught(ed, make_ctx, orc):
    # fault injection: with the hash base r = 1 a string hashes like any of its
    # permutations.  B is A with one pair of neighbouring characters swapped
    # (ED = 2); the weak hash sees equal prefixes past the swap, so the plain
    # hash distance comes out too small (one-sided, never too large).  The check
    # of ed_align must reject it, and ED_FLAG_CERTIFY must answer the exact 2.
    # (the swap lies past the first 16384 + 131072 + 3 x 262144 characters,
    # which the lane, wavefront and workgroup tiers compare directly before the
    # hash search)
    d4 = synth.CharDist("uniform", 4)
    A = synth.random_string(3000000, d4, 61)
    pos = next(i for i in range(1500000, 3000000) if A[i] != A[i + 1])
    B = A.copy()
    B[pos], B[pos + 1] = A[pos + 1], A[pos]
    assert orc.lv_omp(A, B, -1, 1) == 2
    weak = make_ctx(engine=ed.ENGINE_HASH, flags=ed.FLAG_WEAK_HASH)
    p = ed.ed_prepare(weak, A, B)
    k_weak = ed.ed_distance(weak, p)
    assert k_weak < 2  # the collision made an LCP too long
    with pytest.raises(ed.EdError) as ei:
        ed.ed_align(weak, p)
    assert ei.value.status == ed.ED_ECOLLISION
    ed.ed_release(p)
    cert = make_ctx(engine=ed.ENGINE_HASH, flags=ed.FLAG_WEAK_HASH | ed.FLAG_CERTIFY)
    p = ed.ed_prepare(cert, A, B)
    assert ed.ed_distance(cert, p) == 2
    assert ed.ed_pair_stats(p)["certify_retries"] == 1
    ed.ed_release(p)
    # the engines of a strong context agree with the oracle on the same pair
    strong = make_ctx(engine=ed.ENGINE_HASH)
    p = ed.ed_prepare(strong, A, B)
    assert ed.ed_distance(strong, p) == 2
    ed.ed_release(p)


def test_pairs_keep_their_hash_base_across_option_changes(ed, make_ctx, orc):
    # a pair's tables are built with the base of the options at prepare time;
    # queries on pairs of different bases (in any order) each use their own
    ctx = make_ctx(engine=ed.ENGINE_HASH, hash_seed=1)
    pairs = []
    for s in range(4):
        A, B, _ = synth.single_pair(20000, 150, 70 + s)
        if s:
            o = ed.ed_get_options(ctx)
            o["hash_seed"] = 1 + s
            ed.ed_set_options(ctx, **o)
        pairs.append((ed.ed_prepare(ctx, A, B), orc.lv_omp(A, B, -1, 1)))
    for p, want in pairs + pairs[::-1]:
        assert ed.ed_distance(ctx, p) == want
        assert ed.ed_pair_stats(p)["collisions"] == 0
    for p, _ in pairs:
        ed.ed_release(p)
