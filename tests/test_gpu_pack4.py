"""The 4-bit layout (direct engine, every character below 16; survey row f3).

Strings over at most 16 symbols are read at 4 bits per character: 16
characters per 64-bit word, so every LCP tier compares twice the characters
of the 8-bit copy per load.  The pack kernel writes a chunk's 4-bit words
when its characters fit; a second pass fills in the chunks written at 2 bits
once the pair's alphabet is known, or the 8-bit copies when a character is
above 15 after all.  Every check here is against the input bytes or the
oracle.
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


def unpack4(words_u8, n):
    w = words_u8.view(np.uint64)
    out = np.empty(len(w) * 16, dtype=np.uint8)
    for j in range(16):
        out[j::16] = ((w >> np.uint64(4 * j)) & np.uint64(15)).astype(np.uint8)
    return out[:n]


D4 = synth.CharDist("uniform", 4)
D16 = synth.CharDist("uniform", 16)


def _pack_cases():
    for n in (1, 15, 16, 17, 4095, 4096, 4097, 16384, 16385, 3 * 16384 + 1000):
        yield "sigma16_n%d" % n, synth.random_string(n, D16, n), synth.random_string(n // 2 + 5, D16, n + 1)
    # 2-bit chunks in a pair whose alphabet needs 4 bits: the second pass writes them
    A = synth.random_string(50000, D4, 3)
    B = synth.random_string(50000, D4, 4)
    B[40000] = 9
    yield "mixed", A, B
    A = synth.random_string(50017, D4, 5)
    B = synth.random_string(49997, D4, 6)
    A[-1] = 15
    yield "mixed_tail", A, B


@pytest.mark.parametrize("name", [c[0] for c in _pack_cases()])
def test_pack4_roundtrip(ed, make_ctx, name):
    A, B = next((a, b) for n, a, b in _pack_cases() if n == name)
    say("pack4", name)
    ctx = make_ctx(engine=ed.ENGINE_DIRECT)
    p = ed.ed_prepare(ctx, A, B)
    try:
        assert ed.ed_pair_stats(p)["bits_per_char"] == 4
        assert np.array_equal(unpack4(ed.ed_pair_buffer(ctx, p, 0, ed.BUF_PACKED4), len(A)), A)
        assert np.array_equal(unpack4(ed.ed_pair_buffer(ctx, p, 1, ed.BUF_PACKED4), len(B)), B)
    finally:
        ed.ed_release(p)


@pytest.mark.parametrize("case", ["above15", "hash_engine", "force8"])
def test_wider_alphabets_keep_the_byte_copy(ed, make_ctx, orc, case):
    # chunks written at 4 bits whose pair turns out to need 8 (a 16 in the
    # last tile), the hash engine (no 4-bit layout), and pack_bits = 8
    A = synth.random_string(60000, D16, 7)
    B, _ = synth.plant_edits(A, 30, D16, 8)
    if case == "above15":
        B[-3] = 16
    ctx = make_ctx(engine=ed.ENGINE_HASH if case == "hash_engine" else ed.ENGINE_DIRECT,
                   pack_bits=8 if case == "force8" else 0)
    say("wider", case)
    p = ed.ed_prepare(ctx, A, B)
    try:
        assert ed.ed_pair_stats(p)["bits_per_char"] == 8
        assert np.array_equal(ed.ed_pair_buffer(ctx, p, 0, ed.BUF_BYTES), A)
        assert np.array_equal(ed.ed_pair_buffer(ctx, p, 1, ed.BUF_BYTES), B)
        assert ed.ed_distance(ctx, p) == orc.lv_omp(A, B, -1, 1)
    finally:
        ed.ed_release(p)


def _lcp_cases16():
    A = synth.random_string(30000, D16, 11)
    B, _ = synth.plant_edits(A, 12, D16, 12)
    yield "planted", A, B
    A = synth.random_string(70000, D16, 13)
    yield "equal", A, A.copy()
    P = synth.periodic_string(50000, D16, 14, period=64)
    yield "periodic", P, P.copy()
    A = synth.random_string(40000, D4, 15)
    B = A.copy()
    B[20000] = 12
    yield "mixed", A, B


@pytest.mark.parametrize("engine", [0, 2, 3])
def test_lcp_engines_4bit(ed, make_ctx, orc, engine):
    """engine 0: lane + wave tiers; 2: workgroup tier; 3: grid tier, at 4 bits."""
    rng = np.random.default_rng(400 + engine)
    ctx = make_ctx(engine=ed.ENGINE_DIRECT)
    for name, A, B in _lcp_cases16():
        say("lcp4", engine, name)
        n, m = len(A), len(B)
        xs, ys = [], []
        for a in range(16):
            for c in range(0, 16, 3):
                xs.append(a); ys.append(c)
                xs.append(max(0, n - 32 + a)); ys.append(max(0, m - 32 + c))
        xs += [n, 0, n, 0]; ys += [m, m, 0, 0]
        for _ in range(200):
            x = int(rng.integers(0, n + 1))
            d = int(rng.integers(-15, 16))
            xs.append(x); ys.append(min(m, max(0, x + d)))
        for _ in range(200):
            xs.append(int(rng.integers(0, n + 1))); ys.append(int(rng.integers(0, m + 1)))
        p = ed.ed_prepare(ctx, A, B)
        try:
            assert ed.ed_pair_stats(p)["bits_per_char"] == 4
            got = ed.ed_debug_lcp(ctx, p, xs, ys, engine=engine)
        finally:
            ed.ed_release(p)
        want = np.array([orc.lcp(A, B, x, y) for x, y in zip(xs, ys)])
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, [(xs[i], ys[i], int(got[i]), int(want[i])) for i in bad[:10]]


@pytest.mark.parametrize("mode", ["lds", "grid7", "blk7g3"])
def test_frontier_rows_4bit(ed, make_ctx, orc, mode):
    kw = {"lds": dict(), "grid7": dict(flags=ed.FLAG_NO_PHASE_A, block_rounds=7),
          "blk7g3": dict(lds_rounds=4, block_rounds=7, grid_blocks=3)}[mode]
    ctx = make_ctx(engine=ed.ENGINE_DIRECT, **kw)
    rng = np.random.default_rng(16)
    for ci in range(12):
        n = int(rng.integers(1, 300))
        A = synth.random_string(n, D16, int(rng.integers(1 << 30)))
        B, _ = synth.plant_edits(A, int(rng.integers(0, 40)), D16, int(rng.integers(1 << 30)))
        say("rows4", mode, ci, len(A), len(B))
        ed_ref, rows_ref = orc.rt_dump(A, B)
        p = ed.ed_prepare(ctx, A, B)
        try:
            if max(A.max(initial=0), B.max(initial=0)) > 3:
                assert ed.ed_pair_stats(p)["bits_per_char"] == 4
            k, rows = ed.ed_distance_dump(ctx, p, (max(len(A), len(B)) + 2) ** 2)
        finally:
            ed.ed_release(p)
        assert k == ed_ref
        np.testing.assert_array_equal(rows, rows_ref, err_msg="case %d" % ci)


def test_distances_4bit_single_batch_and_align(ed, make_ctx, orc):
    ctx = make_ctx(engine=ed.ENGINE_DIRECT)
    pairs_h = []
    for seed, (n, k) in enumerate([(200000, 1000), (1_000_000, 50), (50000, 3000), (3_000_000, 20)]):
        A = synth.random_string(n, D16, 50 + seed)
        B, _ = synth.plant_edits(A, k, D16, 60 + seed)
        pairs_h.append((A, B))
    # a periodic pair: long slides through the wavefront, workgroup and grid tiers
    P = synth.periodic_string(2_000_000, D16, 70, period=64)
    Q, _ = synth.plant_edits(P, 40, D16, 71)
    pairs_h.append((P, Q))
    want = [orc.lv_omp(A, B) for A, B in pairs_h]
    for i, (A, B) in enumerate(pairs_h):
        say("distance4", i, len(A))
        p = ed.ed_prepare(ctx, A, B)
        try:
            assert ed.ed_pair_stats(p)["bits_per_char"] == 4
            assert ed.ed_distance(ctx, p) == want[i], i
        finally:
            ed.ed_release(p)
    say("batch4")
    pairs = [ed.ed_prepare(ctx, A, B) for A, B in pairs_h]
    try:
        got, st = ed.ed_batch(ctx, pairs)
    finally:
        for p in pairs:
            ed.ed_release(p)
    assert st == [0] * len(pairs) and list(got) == want
    say("align4")
    A, B = pairs_h[2]
    p = ed.ed_prepare(ctx, A, B)
    try:
        k, script = ed.ed_align(ctx, p)
    finally:
        ed.ed_release(p)
    assert k == want[2]
    x = y = edits = 0
    for op, L in script:
        if op == ed.OP_MATCH:
            assert np.array_equal(A[x:x + L], B[y:y + L])
            x += L; y += L
        elif op == ed.OP_SUB:
            x += L; y += L; edits += L
        elif op == ed.OP_DEL:
            x += L; edits += L
        else:
            y += L; edits += L
    assert (x, y, edits) == (len(A), len(B), k)


def test_serving_4bit_requests(ed, make_ctx, orc):
    # requests over 16 symbols through the serving loop (the many-pair kernel
    # reads the 4-bit words), mixed with requests over 4 symbols
    ctx = make_ctx(engine=ed.ENGINE_DIRECT)
    reqs = []
    for i in range(24):
        n = [300, 5000, 40000, 200000][i % 4]
        d = D16 if i % 3 else D4
        A = synth.random_string(n, d, 700 + i)
        B, _ = synth.plant_edits(A, max(1, n // 200), d, 800 + i)
        reqs.append((A, B))
    say("serve 4-bit", len(reqs))
    srv = ed.ed_serve_open(ctx, 8 << 30, 32)
    try:
        for tag, (A, B) in enumerate(reqs):
            assert ed.ed_serve_submit(srv, A, B, tag) == 0, ed.ed_last_error()
        ed.ed_serve_drain(srv)
        res = ed.ed_serve_poll(srv, len(reqs) + 1)
    finally:
        ed.ed_serve_close(srv)
    assert len(res) == len(reqs) and all(r["status"] == 0 for r in res)
    got = {r["tag"]: r["k"] for r in res}
    for tag, (A, B) in enumerate(reqs):
        assert got[tag] == orc.lv_omp(A, B, -1, 1), tag
