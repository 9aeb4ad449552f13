"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is exact: the edit distance, the frontier rows, the LCPs, the
packed strings and the prefix tables are integers.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


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


def gpu_ed(ed, ctx, A, B, k_max=-1):
    p = ed.ed_prepare(ctx, A, B)
    try:
        return ed.ed_distance(ctx, p, k_max)
    finally:
        ed.ed_release(p)


def unpack2(words_u8, n):
    w = words_u8.view(np.uint64)
    out = np.empty(len(w) * 32, dtype=np.uint8)
    for j in range(32):
        out[j::32] = ((w >> np.uint64(2 * j)) & np.uint64(3)).astype(np.uint8)
    return out[:n]


# ---------------------------------------------------------------------------
# pack, copy, alphabet detection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", [0, 1, 31, 32, 33, 1000, 4095, 4096, 4097, 8193, 16383, 16384, 16385,
                               100003])
def test_pack_roundtrip(ed, make_ctx, n):
    say("pack", n)
    ctx = make_ctx()
    A = synth.random_string(n, synth.CharDist("uniform", 4), 7)
    B = synth.random_string(n // 2 + 3, synth.CharDist("uniform", 4), 8)
    p = ed.ed_prepare(ctx, A, B)
    st = ed.ed_pair_stats(p)
    assert st["bits_per_char"] == 2
    assert np.array_equal(unpack2(ed.ed_pair_buffer(ctx, p, 0, ed.BUF_PACKED2), n), A)
    assert np.array_equal(unpack2(ed.ed_pair_buffer(ctx, p, 1, ed.BUF_PACKED2), len(B)), B)
    ed.ed_release(p)


@pytest.mark.parametrize("case", ["sigma256", "mixed", "mixed_tail", "force8"])
def test_byte_copy(ed, make_ctx, case):
    say("bytes", case)
    n = 50000
    if case == "sigma256":
        ctx = make_ctx()
        A = synth.random_string(n, synth.CharDist("uniform", 256), 1)
        B = synth.random_string(n + 7, synth.CharDist("uniform", 256), 2)
    elif case == "mixed":
        # one string packable everywhere, the other with a large character in one tile only
        ctx = make_ctx()
        A = synth.random_string(n, synth.CharDist("uniform", 4), 3)
        B = synth.random_string(n, synth.CharDist("uniform", 4), 4)
        B[40000] = 200
    elif case == "mixed_tail":
        # large characters only in the last, partial chunk of A and the first chunk of B
        ctx = make_ctx()
        A = synth.random_string(n + 17, synth.CharDist("uniform", 4), 9)
        B = synth.random_string(n - 3, synth.CharDist("uniform", 4), 10)
        A[-1] = 4
        B[0] = 255
    else:
        ctx = make_ctx(pack_bits=8)
        A = synth.random_string(n, synth.CharDist("uniform", 4), 5)
        B = synth.random_string(n - 5, synth.CharDist("uniform", 4), 6)
    p = ed.ed_prepare(ctx, A, B)
    assert ed.ed_pair_stats(p)["bits_per_char"] == 8
    assert np.array_equal(ed.ed_pair_buffer(ctx, p, 0, ed.BUF_BYTES), A)
    assert np.array_equal(ed.ed_pair_buffer(ctx, p, 1, ed.BUF_BYTES), B)
    ed.ed_release(p)


def test_pack2_rejects_large_characters(ed, make_ctx):
    say("pack2 reject")
    ctx = make_ctx(pack_bits=2)
    A = np.array([0, 1, 2, 3, 7], np.uint8)
    with pytest.raises(ed.EdError) as ei:
        ed.ed_prepare(ctx, A, A)
    assert ei.value.status == ed.ED_EINVAL


# ---------------------------------------------------------------------------
# prefix tables: bit-exact against Horner's rule (sections 3.2, 3.3)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("b", [1, 2, 4, 8, 16, 32, 64, 128, 1024, 4096])
@pytest.mark.parametrize("alpha", ["sigma4", "sigma256", "mixed"])
def test_table_bit_exact(ed, make_ctx, orc, b, alpha):
    say("table", b, alpha)
    seed = 1000 + b
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=b, hash_seed=seed)
    base = orc.hash_base(seed)
    for n in [0, 1, b - 1, b, b + 1, 16384 + 3 * b + 1, 3 * 16384, 70001]:
        if n < 0:
            continue
        if alpha == "sigma256":
            A = synth.random_string(n, synth.CharDist("uniform", 256), n + 1)
        else:
            A = synth.random_string(n, synth.CharDist("uniform", 4), n + 1)
            if alpha == "mixed" and n > 20000:
                A[20000] = 255
        B = synth.random_string(n // 3 + 1, synth.CharDist("uniform", 4), n + 2)
        p = ed.ed_prepare(ctx, A, B)
        TA = ed.ed_pair_buffer(ctx, p, 0, ed.BUF_TABLE)
        TB = ed.ed_pair_buffer(ctx, p, 1, ed.BUF_TABLE)
        np.testing.assert_array_equal(TA, orc.horner_table(A, b, base), err_msg="A n=%d" % n)
        np.testing.assert_array_equal(TB, orc.horner_table(B, b, base), err_msg="B n=%d" % n)
        ed.ed_release(p)


def test_base_switch_after_prepare_on_side_stream(ed, make_ctx, orc):
    # a prepare queued on a stream that does not wait for the null stream,
    # then a new hash base at once: the pair's tables must still be those of
    # its own base (the context's power tables are rewritten only after the
    # queued kernels that read them)
    import torch
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=32, hash_seed=501)
    A = synth.random_string(1 << 25, synth.CharDist("uniform", 256), 41)
    B = synth.random_string(5000, synth.CharDist("uniform", 4), 42)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    say("base switch on side stream")
    p = ed.ed_prepare(ctx, tA, tB, stream=side)
    ed.ed_set_options(ctx, engine=ed.ENGINE_HASH, block=32, hash_seed=502)
    side.synchronize()
    TA = ed.ed_pair_buffer(ctx, p, 0, ed.BUF_TABLE)
    ed.ed_release(p)
    np.testing.assert_array_equal(TA, orc.horner_table(A, 32, orc.hash_base(501)))


def test_release_right_after_prepare_on_side_stream(ed, make_ctx, orc):
    # a pair released while its prepare is still queued on a stream that does
    # not wait for the null stream: the release waits for that work, and the
    # next pair, which reuses the pooled buffers, is exact
    import torch
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=32, hash_seed=503)
    side = torch.cuda.Stream()
    A = synth.random_string(1 << 25, synth.CharDist("uniform", 4), 43)
    B, _ = synth.plant_edits(A, 20, synth.CharDist("uniform", 4), 44)
    tA, tB = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    torch.cuda.synchronize()
    for r in range(3):
        say("release on side stream", r)
        p = ed.ed_prepare(ctx, tA, tB, stream=side)
        ed.ed_release(p)
    C = synth.random_string(1 << 25, synth.CharDist("uniform", 4), 45)
    D, _ = synth.plant_edits(C, 30, synth.CharDist("uniform", 4), 46)
    tC, tD = torch.from_numpy(C).cuda(), torch.from_numpy(D).cuda()
    torch.cuda.synchronize()
    p = ed.ed_prepare(ctx, tC, tD, stream=side)
    try:
        TA = ed.ed_pair_buffer(ctx, p, 0, ed.BUF_TABLE)
        k = ed.ed_distance(ctx, p, stream=side)
    finally:
        ed.ed_release(p)
    np.testing.assert_array_equal(TA, orc.horner_table(C, 32, orc.hash_base(503)))
    assert k == orc.lv_omp(C, D, -1, 1)


@pytest.mark.parametrize("b,sigma", [(32, 4), (4096, 4), (32, 256), (64, 256)])
def test_table_bit_exact_multi_chunk_scan(ed, make_ctx, orc, b, sigma):
    # more than 8192 tiles of 16384 characters: the scan of the tile hashes
    # runs over several chunks and carries the prefix from one to the next
    n = 8193 * 16384 + 77
    say("table multi-chunk", b, sigma, n)
    seed = 77 + b
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=b, hash_seed=seed)
    A = synth.random_string(n, synth.CharDist("uniform", sigma), 5)
    B = synth.random_string(1000, synth.CharDist("uniform", 4), 6)
    p = ed.ed_prepare(ctx, A, B)
    TA = ed.ed_pair_buffer(ctx, p, 0, ed.BUF_TABLE)
    ed.ed_release(p)
    np.testing.assert_array_equal(TA, orc.horner_table(A, b, orc.hash_base(seed)))


@pytest.mark.parametrize("b", [32, 64])
def test_table_and_distance_with_forced_8bit_copy(ed, make_ctx, orc, b):
    # alphabet {0,1,2,3} kept at 8 bits per character (pack_bits=8): the
    # block hashes come from the input bytes whatever the packing, and the
    # tables must equal Horner's rule over the characters either way
    say("table force8", b)
    seed = 31 + b
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=b, hash_seed=seed, pack_bits=8)
    d4 = synth.CharDist("uniform", 4)
    for n in [1, 31, 32, 33, 16384 * 3 + 17]:
        A = synth.random_string(n, d4, n + 7)
        B, _ = synth.plant_edits(A, max(1, n // 500), d4, n + 8)
        p = ed.ed_prepare(ctx, A, B)
        try:
            assert ed.ed_pair_stats(p)["bits_per_char"] == 8
            np.testing.assert_array_equal(ed.ed_pair_buffer(ctx, p, 0, ed.BUF_TABLE),
                                          orc.horner_table(A, b, orc.hash_base(seed)), err_msg="A n=%d" % n)
            np.testing.assert_array_equal(ed.ed_pair_buffer(ctx, p, 1, ed.BUF_TABLE),
                                          orc.horner_table(B, b, orc.hash_base(seed)), err_msg="B n=%d" % n)
            assert ed.ed_distance(ctx, p) == orc.lv_omp(A, B)
        finally:
            ed.ed_release(p)


# ---------------------------------------------------------------------------
# LCP engines against the character loop (section 2)
# ---------------------------------------------------------------------------
def _lcp_cases():
    d4 = synth.CharDist("uniform", 4)
    d256 = synth.CharDist("uniform", 256)
    A = synth.random_string(30000, d4, 11)
    B, _ = synth.plant_edits(A, 12, d4, 12)
    yield "sigma4_planted", A, B
    A = synth.random_string(30000, d256, 13)
    B, _ = synth.plant_edits(A, 12, d256, 14)
    yield "sigma256_planted", A, B
    A = synth.random_string(70000, d4, 15)
    yield "equal", A, A.copy()
    P = synth.periodic_string(50000, d4, 16, period=64)
    yield "periodic", P, P.copy()
    Z = np.zeros(5000, np.uint8)
    yield "zeros", Z, Z.copy()


@pytest.mark.parametrize("engine", [0, 1, 2, 3])
@pytest.mark.parametrize("pack_bits", [0, 8])
@pytest.mark.parametrize("block", [32, 1, 4, 256])
def test_lcp_engines(ed, make_ctx, orc, engine, pack_bits, block):
    """engine 0: lane + wave tiers; 1: hash search; 2: direct workgroup tier; 3: grid tier."""
    if engine != 1 and block != 32:
        pytest.skip("block size only matters for the hash engine")
    rng = np.random.default_rng(engine * 100 + pack_bits + block)
    ctx = make_ctx(engine=min(engine, 1), pack_bits=pack_bits, block=block, hash_seed=77)
    for name, A, B in _lcp_cases():
        say("lcp", engine, pack_bits, block, name)
        n, m = len(A), len(B)
        xs, ys = [], []
        # every alignment pair mod 32 near the start, near the end, and the ends themselves
        for a in range(32):
            for c in range(0, 32, 3):
                xs.append(a); ys.append(c)
                xs.append(max(0, n - 64 + a)); ys.append(max(0, m - 64 + c))
        xs += [n, 0, n, 0]; ys += [m, m, 0, 0]
        # diagonal-aligned queries (long LCPs on planted pairs)
        for _ in range(200):
            x = int(rng.integers(0, n + 1))
            d = int(rng.integers(-15, 16))
            xs.append(x); ys.append(min(m, max(0, x + d)))
        for _ in range(200):
            xs.append(int(rng.integers(0, n + 1))); ys.append(int(rng.integers(0, m + 1)))
        p = ed.ed_prepare(ctx, A, B)
        got = ed.ed_debug_lcp(ctx, p, xs, ys, engine=engine)
        want = np.array([orc.lcp(A, B, x, y) for x, y in zip(xs, ys)])
        bad = np.nonzero(got != want)[0]
        assert len(bad) == 0, [(xs[i], ys[i], int(got[i]), int(want[i])) for i in bad[:10]]
        ed.ed_release(p)


@pytest.mark.parametrize("pack_bits", [0, 8])
def test_lcp_grid_tier_long(ed, make_ctx, orc, pack_bits):
    # one mismatch planted around segment boundaries of the grid tier (1024
    # threads x 8 words: 262144 characters at 2 bits, 65536 at 8 bits)
    n = 3_000_000
    seg = 1024 * 8 * (32 if pack_bits == 0 else 8)
    A = synth.random_string(n, synth.CharDist("uniform", 4), 31)
    ctx = make_ctx(pack_bits=pack_bits, flags=ed.FLAG_TIMING)
    spots = [0, 1, seg - 1, seg, seg + 1, 3 * seg + 17, 7 * seg - 1, n - 2, n - 1]
    for pos in spots + [None]:
        B = A.copy()
        if pos is not None:
            B[pos] ^= 1
        say("grid lcp", pack_bits, pos)
        p = ed.ed_prepare(ctx, A, B)
        xs = [0, 5, 0, 1000]
        ys = [0, 5, 3, 1000]
        got = ed.ed_debug_lcp(ctx, p, xs, ys, engine=3)
        want = [orc.lcp(A, B, x, y) for x, y in zip(xs, ys)]
        assert list(got) == want
        assert ed.ed_pair_stats(p)["gpu_ns_lcp_kernel"] > 0
        ed.ed_release(p)


# ---------------------------------------------------------------------------
# frontier rows: every f_t[i] against R_t from the DP matrix
# ---------------------------------------------------------------------------
FRONTIER_MODES = [
    ("lds", dict()),
    ("grid", dict(flags=2)),
    ("lds3", dict(lds_rounds=3)),
    ("grow", dict(lds_rounds=2, init_rows=4)),
    ("blk1", dict(lds_rounds=4, block_rounds=1)),
    ("blk7g3", dict(lds_rounds=4, block_rounds=7, grid_blocks=3)),
    ("g1", dict(lds_rounds=2, block_rounds=5, grid_blocks=1)),
    ("grid7", dict(flags=2, block_rounds=7)),
    # hash engine: long slides straight to the hash search, full table (no-op for the direct engine)
    ("hfirst", dict(flags=128, block=1, lds_rounds=4, block_rounds=5)),
]


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("mode", [m[0] for m in FRONTIER_MODES])
def test_frontier_rows(ed, make_ctx, orc, engine, mode):
    kw = dict(FRONTIER_MODES)[mode]
    ctx = make_ctx(engine=engine, **kw)
    rng = np.random.default_rng(1 + engine)
    cases = [(np.zeros(0, np.uint8), np.zeros(0, np.uint8)),
             (np.zeros(0, np.uint8), np.array([1, 2, 3], np.uint8)),
             (np.array([3, 2, 1, 0], np.uint8), np.zeros(0, np.uint8)),
             (np.array([1], np.uint8), np.array([1], np.uint8))]
    for _ in range(25):
        sigma = int(rng.choice([2, 4, 20, 256]))
        n = int(rng.integers(0, 300))
        d = synth.CharDist("uniform", sigma)
        A = synth.random_string(n, d, int(rng.integers(1 << 30)))
        B, _ = synth.plant_edits(A, int(rng.integers(0, 40)), d, int(rng.integers(1 << 30)))
        cases.append((A, B))
    for ci, (A, B) in enumerate(cases):
        say("rows", engine, mode, ci, len(A), len(B))
        ed_ref, rows_ref = orc.rt_dump(A, B)
        p = ed.ed_prepare(ctx, A, B)
        cap = (max(len(A), len(B)) + 2) ** 2
        k, rows = ed.ed_distance_dump(ctx, p, cap)
        ed.ed_release(p)
        assert k == ed_ref
        np.testing.assert_array_equal(rows, rows_ref, err_msg="case %d" % ci)


# ---------------------------------------------------------------------------
# distances
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("block", [1, 32])
def test_hash_first_mode_distances(ed, make_ctx, orc, block):
    # the long-LCP mode: every slide past the lane stage goes to the hash
    # search (alphabet 4 and 256, a period-64 string, long planted runs)
    ctx = make_ctx(engine=ed.ENGINE_HASH, block=block, flags=ed.FLAG_HASH_FIRST)
    d4, d256 = synth.CharDist("uniform", 4), synth.CharDist("uniform", 256)
    cases = [synth.single_pair(200000, 300, 61), synth.single_pair(300000, 50, 62, sigma=256)]
    P = synth.periodic_string(400000, d4, 63, period=64)
    Q, _ = synth.plant_edits(P, 80, d4, 64)
    cases.append((P, Q, None))
    for i, (A, B, _) in enumerate(cases):
        say("hash first", block, i)
        p = ed.ed_prepare(ctx, A, B)
        try:
            k = ed.ed_distance(ctx, p)
            st = ed.ed_pair_stats(p)
        finally:
            ed.ed_release(p)
        assert k == orc.lv_omp(A, B, -1, 1), i
        assert st["wg_lcps"] == 0
def test_config1_all_seeds_direct(ed, make_ctx, orc):
    ctx = make_ctx(engine=0)
    for seed in range(100):
        A, B, info = synth.small_pair(seed)
        say("config1 direct", seed)
        assert gpu_ed(ed, ctx, A, B) == orc.lv_naive(A, B), seed


def test_config1_seeds_hash(ed, make_ctx, orc):
    ctx = make_ctx(engine=1)
    for seed in range(30):
        A, B, info = synth.small_pair(seed)
        say("config1 hash", seed)
        assert gpu_ed(ed, ctx, A, B) == orc.lv_naive(A, B), seed


@pytest.mark.parametrize("engine", [0, 1])
def test_edge_cases(ed, make_ctx, orc, engine):
    ctx = make_ctx(engine=engine)
    d4 = synth.CharDist("uniform", 4)
    X = synth.random_string(5000, d4, 1)
    Y = synth.random_string(3000, d4, 2)
    cases = {
        "empty": (np.zeros(0, np.uint8), np.zeros(0, np.uint8)),
        "emptyA": (np.zeros(0, np.uint8), X),
        "emptyB": (X, np.zeros(0, np.uint8)),
        "identical": (X, X.copy()),
        "prefix": (X, X[:4000].copy()),
        "suffix": (X[1000:].copy(), X),
        "unrelated": (X[:1500].copy(), Y[:1500].copy()),
        "lengths": (X, Y[:200].copy()),
        "ones": (np.array([1], np.uint8), np.array([2], np.uint8)),
        "zeros_vs_ones": (np.zeros(700, np.uint8), np.ones(900, np.uint8)),
        "periodic": (synth.periodic_string(9000, d4, 3, 64), synth.periodic_string(9050, d4, 3, 64)),
        # almost every diagonal has a long LCP: more long LCPs per round than the queue holds
        "zeros_edits": (np.zeros(20000, np.uint8),
                        synth.plant_edits(np.zeros(20000, np.uint8), 300, synth.CharDist("uniform", 2), 4)[0]),
    }
    for name, (A, B) in cases.items():
        say("edge", engine, name)
        want = orc.lv_omp(A, B)
        assert gpu_ed(ed, ctx, A, B) == want, name
        assert gpu_ed(ed, ctx, B, A) == want, name + " swapped"


@pytest.mark.parametrize("engine", [0, 1])
def test_k_max_cutoff(ed, make_ctx, orc, engine):
    ctx = make_ctx(engine=engine)
    A, B, _ = synth.single_pair(20000, 300, 5)
    k = orc.lv_omp(A, B)
    say("kmax", engine, k)
    assert gpu_ed(ed, ctx, A, B, k_max=k) == k
    assert gpu_ed(ed, ctx, A, B, k_max=k + 10) == k
    assert gpu_ed(ed, ctx, A, B, k_max=k - 1) == k
    assert gpu_ed(ed, ctx, A, B, k_max=k // 3) == k // 3 + 1


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("mode", ["default", "grid", "grow", "narrow"])
def test_medium_pairs(ed, make_ctx, orc, engine, mode):
    kw = {"default": {}, "grid": dict(flags=2), "grow": dict(lds_rounds=64, init_rows=100),
          "narrow": dict(grid_blocks=1, lds_rounds=16, block_rounds=8)}[mode]
    ctx = make_ctx(engine=engine, **kw)
    for (n, k, sigma, seed) in [(200000, 3000, 4, 1), (100000, 9000, 4, 2), (150000, 2000, 20, 3),
                                (300000, 500, 256, 4), (60000, 6000, 2, 5)]:
        A, B, _ = synth.single_pair(n, k, seed, sigma=sigma)
        say("medium", engine, mode, n, k, sigma)
        assert gpu_ed(ed, ctx, A, B) == orc.lv_omp(A, B)


@pytest.mark.parametrize("case", ["sigma4", "sigma256", "force8"])
def test_long_lcps_in_phase_a(ed, make_ctx, orc, case):
    # few edits on long strings: the one-workgroup phase meets LCPs of many
    # workgroup-tier steps (and, with k = 0, one LCP over the whole string)
    if case == "sigma4":
        ctx = make_ctx(flags=ed.FLAG_TIMING)
        specs = [(4_000_000, 3, 4, 1), (3_000_000, 6, 4, 2), (2_500_000, 0, 4, 3)]
    elif case == "sigma256":
        ctx = make_ctx(flags=ed.FLAG_TIMING)
        specs = [(1_000_000, 5, 256, 4), (800_000, 9, 256, 5)]
    else:
        ctx = make_ctx(pack_bits=8, flags=ed.FLAG_TIMING)
        specs = [(1_200_000, 4, 4, 6)]
    for n, k, sigma, seed in specs:
        A, B, _ = synth.single_pair(n, k, seed, sigma=sigma)
        say("long lcps", case, n, k)
        p = ed.ed_prepare(ctx, A, B)
        got = ed.ed_distance(ctx, p)
        st = ed.ed_pair_stats(p)
        ed.ed_release(p)
        assert got == orc.lv_omp(A, B)
        # extended by the workgroup tier, or by every workgroup (grid rounds)
        assert st["wg_lcps"] + st["grid_lcps"] > 0


@pytest.mark.parametrize("engine", [0, 1])
@pytest.mark.parametrize("case", ["sigma4", "sigma256", "periodic"])
def test_long_lcps_in_grid_rounds(ed, make_ctx, orc, engine, case):
    # every round grid-wide (no one-workgroup phase), short blocks: slides
    # longer than the wavefront steps go to the workgroup tier (or the hash
    # search) inside the temporal blocks
    ctx = make_ctx(engine=engine, flags=ed.FLAG_NO_PHASE_A | ed.FLAG_TIMING, block_rounds=9)
    if case == "sigma4":
        specs = [(600_000, 25, 4, 11), (300_000, 700, 4, 12)]
    elif case == "sigma256":
        specs = [(300_000, 30, 256, 13), (200_000, 900, 256, 14)]
    else:
        specs = [(250_000, 150, 0, 15)]
    for n, k, sigma, seed in specs:
        if sigma:
            A, B, _ = synth.single_pair(n, k, seed, sigma=sigma)
        else:
            A = synth.periodic_string(n, synth.CharDist("uniform", 4), seed, 64)
            B, _ = synth.plant_edits(A, k, synth.CharDist("uniform", 4), seed + 1)
        say("long lcps grid", engine, case, n, k)
        assert gpu_ed(ed, ctx, A, B) == orc.lv_omp(A, B)


@pytest.mark.parametrize("case", ["sigma4", "sigma256", "force8", "to_grid_blocks", "kmax", "grow"])
def test_grid_rounds(ed, make_ctx, orc, case):
    # pairs within few edits of identity: slides far past a workgroup step,
    # extended by every workgroup in the first rounds (direct engine); the
    # same distances with those rounds switched off, and equal to the oracle
    kw = {"sigma4": {}, "sigma256": {}, "force8": dict(pack_bits=8),
          "to_grid_blocks": dict(lds_rounds=2, block_rounds=3), "kmax": {},
          "grow": dict(lds_rounds=8, init_rows=6)}[case]
    ctx = make_ctx(flags=ed.FLAG_TIMING, **kw)
    ref = make_ctx(flags=ed.FLAG_TIMING | ed.FLAG_NO_GRID_ROUNDS, **kw)
    sigma = 256 if case == "sigma256" else 4
    specs = {"to_grid_blocks": [(24_000_000, 3, 7)], "grow": [(24_000_000, 4, 8)]}.get(
        case, [(6_000_000, 0, 1), (6_000_000, 1, 2), (5_000_000, 5, 3), (30_000_000, 3, 4)])
    for n, k, seed in specs:
        A, B, _ = synth.single_pair(n, k, seed, sigma=sigma)
        want = orc.lv_omp(A, B)
        say("grid rounds", case, n, k, want)
        kmax = max(want // 2, 0) if case == "kmax" else -1
        p = ed.ed_prepare(ctx, A, B)
        got = ed.ed_distance(ctx, p, kmax)
        st = ed.ed_pair_stats(p)
        ed.ed_release(p)
        q = ed.ed_prepare(ref, A, B)
        alone = ed.ed_distance(ref, q, kmax)
        ed.ed_release(q)
        expect = want if kmax < 0 or want <= kmax else kmax + 1
        assert got == alone == expect
        # the first slide runs past the wavefront steps: extended by the grid
        assert st["grid_lcps"] > 0


@pytest.mark.parametrize("first", ["align", "distance"])
def test_grid_rounds_alignment(ed, make_ctx, orc, first):
    # the per-round rows that the grid rounds write back are traced and
    # checked, in segments (a fresh pair) and in the cone of one launch (k known)
    ctx = make_ctx()
    A, B, _ = synth.single_pair(6_000_000, 7, 21)
    want = orc.lv_omp(A, B)
    p = ed.ed_prepare(ctx, A, B)
    try:
        if first == "distance":
            assert ed.ed_distance(ctx, p) == want
        k, script = ed.ed_align(ctx, p)
        st = ed.ed_pair_stats(p)
    finally:
        ed.ed_release(p)
    assert k == want
    assert st["grid_lcps"] > 0
    assert sum(ln for op, ln in script if op != ed.OP_MATCH) == k
    x = y = 0
    for op, ln in script:
        if op == ed.OP_MATCH:
            assert np.array_equal(A[x:x + ln], B[y:y + ln])
        if op in (ed.OP_MATCH, ed.OP_SUB, ed.OP_DEL):
            x += ln
        if op in (ed.OP_MATCH, ed.OP_SUB, ed.OP_INS):
            y += ln
    assert (x, y) == (len(A), len(B))


# ---------------------------------------------------------------------------
# batch
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("engine", [0, 1])
def test_batch_matches_oracle_and_single(ed, make_ctx, orc, engine):
    ctx = make_ctx(engine=engine)
    specs = synth.batch_specs(300, 9, lo_exp=1.0, hi_exp=4.7, kfrac=0.05)
    pairs, want = [], []
    for n, k, ps in specs:
        A, B, _ = synth.single_pair(n, k, ps)
        pairs.append(ed.ed_prepare(ctx, A, B))
        want.append(orc.lv_omp(A, B))
    # unrelated strings: the distance outgrows the rows a batch reserves
    d4 = synth.CharDist("uniform", 4)
    for seed in (1, 2):
        A = synth.random_string(12000, d4, 100 + seed)
        B = synth.random_string(11000, d4, 200 + seed)
        pairs.append(ed.ed_prepare(ctx, A, B))
        want.append(orc.lv_omp(A, B))
    say("batch", engine, len(pairs))
    got, st = ed.ed_batch(ctx, pairs)
    assert st == [0] * len(pairs)
    assert got == want
    single = [ed.ed_distance(ctx, p) for p in pairs[:40]]
    assert single == want[:40]
    ed.ed_set_options(ctx, engine=engine, flags=4, hash_seed=0x5EED)
    got2, _ = ed.ed_batch(ctx, pairs)
    assert got2 == want
    ed.ed_set_options(ctx, engine=engine, lds_rounds=16, flags=4, hash_seed=0x5EED)
    got3, _ = ed.ed_batch(ctx, pairs)
    assert got3 == want
    # one-workgroup grid, tiny chunks of rounds: many super-steps per pair
    ed.ed_set_options(ctx, engine=engine, lds_rounds=8, block_rounds=3, grid_blocks=1, hash_seed=0x5EED)
    got4, _ = ed.ed_batch(ctx, pairs[:60] + pairs[-2:])
    assert got4 == want[:60] + want[-2:]
    # k_max cutoff inside the batch
    got5, _ = ed.ed_batch(ctx, pairs, k_max=50)
    assert got5 == [min(w, 51) for w in want]
    for p in pairs:
        ed.ed_release(p)


@pytest.mark.parametrize("engine", [0, 1])
def test_autotune_batch(ed, make_ctx, orc, engine):
    # the tuner times every candidate, keeps the distances identical and
    # leaves the winner in the context; the batch still matches the oracle
    ctx = make_ctx(engine=engine)
    specs = synth.batch_specs(96, 17, lo_exp=2.0, hi_exp=4.5, kfrac=0.05)
    pairs, want = [], []
    for n, k, ps in specs:
        A, B, _ = synth.single_pair(n, k, ps)
        pairs.append(ed.ed_prepare(ctx, A, B))
        want.append(orc.lv_omp(A, B))
    say("autotune", engine, len(pairs))
    r = ed.ed_autotune_batch(ctx, pairs, passes=1)
    kn = r["knobs"]
    assert r["evaluated"] >= 3 and r["best_ms"] > 0 and r["best_ms"] <= r["default_ms"] * 1.0001
    assert kn["chunk_diags"] + 2 * kn["task_block_rounds"] <= 2 * 4096 + 5
    opts = ed.ed_get_options(ctx)
    assert {k: opts[k] for k in kn} == kn
    got, st = ed.ed_batch(ctx, pairs)
    assert st == [0] * len(pairs) and got == want
    # k_max is honoured while tuning
    r2 = ed.ed_autotune_batch(ctx, pairs[:20], k_max=5, passes=1)
    assert r2["evaluated"] >= 3
    got2, _ = ed.ed_batch(ctx, pairs[:20], k_max=5)
    assert got2 == [min(w, 6) for w in want[:20]]
    for p in pairs:
        ed.ed_release(p)


def test_batch_superstep_wider_than_workgroup(ed, make_ctx, orc):
    # 64-diagonal chunks: the late super-steps of the large pair hold more
    # chunk tasks than the workgroup that schedules them has threads, so each
    # thread pushes several; the rows the batch reserves (n / 16 rounds) hold
    # the whole distance, so the pair stays in the many-pair kernel
    ctx = make_ctx(engine=0)
    A, B, _ = synth.single_pair(700000, 40000, 31)
    want = [orc.lv_omp(A, B)]
    assert (2 * want[0] + 5 + 63) // 64 > 1024 and want[0] <= len(A) // 16
    pairs = [ed.ed_prepare(ctx, A, B)]
    for n, k, ps in synth.batch_specs(40, 23, lo_exp=3.0, hi_exp=5.0, kfrac=0.05):
        A2, B2, _ = synth.single_pair(n, k, ps)
        pairs.append(ed.ed_prepare(ctx, A2, B2))
        want.append(orc.lv_omp(A2, B2))
    say("batch, 64-diagonal chunks", len(pairs))
    ed.ed_set_options(ctx, engine=0, chunk_diags=64, task_block_rounds=16)
    try:
        got, st = ed.ed_batch(ctx, pairs)
    finally:
        for p in pairs:
            ed.ed_release(p)
    assert st == [0] * len(pairs)
    assert got == want


def test_device_inputs_and_unaligned(ed, make_ctx, orc):
    import torch
    ctx = make_ctx()
    A, B, _ = synth.single_pair(30000, 200, 21)
    want = orc.lv_omp(A, B)
    tA = torch.from_numpy(A).cuda()
    tB = torch.from_numpy(B).cuda()
    say("device inputs")
    assert gpu_ed(ed, ctx, tA, tB) == want
    # unaligned device views go through a staging copy
    tA2 = torch.zeros(len(A) + 3, dtype=torch.uint8, device="cuda")
    tA2[3:] = tA
    assert gpu_ed(ed, ctx, tA2[3:], tB) == want


# ---------------------------------------------------------------------------
# serving: continuous batching under an HBM budget
# ---------------------------------------------------------------------------
def _serve_all(ed, ctx, reqs, budget, slots, gap_s=0.0):
    import time
    srv = ed.ed_serve_open(ctx, budget, slots)
    for tag, (A, B) in enumerate(reqs):
        rc = ed.ed_serve_submit(srv, A, B, tag)
        assert rc == 0, ed.ed_last_error()
        if gap_s:
            time.sleep(gap_s)
    ed.ed_serve_drain(srv)
    res = ed.ed_serve_poll(srv, len(reqs) + 10)
    ed.ed_serve_close(srv)
    return res


@pytest.mark.parametrize("engine", [0, 1])
def test_serve_matches_oracle_and_alone(ed, make_ctx, orc, engine):
    ctx = make_ctx(engine=engine)
    trace = synth.arrival_trace(120, 3, rate_per_s=1e4, lo_exp=1.0, hi_exp=4.6, kfrac=0.05)
    reqs = [synth.request_pair(r) for r in trace]
    want = [orc.lv_omp(A, B) for A, B in reqs]
    say("serve", engine, len(reqs))
    res = _serve_all(ed, ctx, reqs, 8 << 30, 64)
    assert sorted(r["tag"] for r in res) == list(range(len(reqs)))
    got = {r["tag"]: r["k"] for r in res}
    assert all(r["status"] == 0 for r in res)
    assert [got[i] for i in range(len(reqs))] == want
    assert all(r["t_done_ns"] >= r["t_arrive_ns"] for r in res)
    # the same requests alone (one slot at a time) give the same answers
    alone = _serve_all(ed, ctx, reqs[:25], 8 << 30, 1)
    got1 = {r["tag"]: r["k"] for r in alone}
    assert [got1[i] for i in range(25)] == want[:25]


@pytest.mark.parametrize("engine", [0, 1])
def test_serve_band_per_request(ed, make_ctx, orc, engine):
    # every request with a k_max of its own, in one mix: the distance when it
    # is at most k_max, else k_max + 1; requests without a bound beside them
    ctx = make_ctx(engine=engine)
    srv = ed.ed_serve_open(ctx, 8 << 30, 64)
    want = {}
    for tag in range(48):
        n = [300, 5000, 40000, 200000][tag % 4]
        A, B, _ = synth.single_pair(n, max(1, n // 40), 700 + tag, sigma=4 if tag % 3 else 20)
        ed_ = orc.lv_omp(A, B)
        kmax = [-1, 0, ed_ // 2, ed_, ed_ + 3, max(ed_ - 1, 0)][tag % 6]
        assert ed.ed_serve_submit_band(srv, A, B, tag, kmax) == 0, ed.ed_last_error()
        want[tag] = ed_ if kmax < 0 or ed_ <= kmax else kmax + 1
    say("serve band", engine)
    ed.ed_serve_drain(srv)
    res = ed.ed_serve_poll(srv, 100)
    ed.ed_serve_close(srv)
    assert all(r["status"] == 0 for r in res)
    assert {r["tag"]: r["k"] for r in res} == want
    assert ed.lib.ed_serve_submit_band(None, None, 0, None, 0, 0, -1) == ed.ED_EINVAL


def test_serve_tiny_budget_and_growth(ed, make_ctx, orc):
    # a budget that fits about one request at a time still completes them all,
    # and a slow-converging pair outgrows its rows and keeps going
    ctx = make_ctx(lds_rounds=64, block_rounds=8)
    d4 = synth.CharDist("uniform", 4)
    reqs = []
    for s in range(6):
        A, B, _ = synth.single_pair(20000, 300 + 50 * s, 40 + s)
        reqs.append((A, B))
    reqs.append((synth.random_string(9000, d4, 77), synth.random_string(8000, d4, 78)))
    want = [orc.lv_omp(A, B) for A, B in reqs]
    say("serve tiny budget")
    res = _serve_all(ed, ctx, reqs, 400 << 10, 8)
    got = {r["tag"]: r["k"] for r in res}
    assert [got[i] for i in range(len(reqs))] == want
    assert all(r["status"] == 0 for r in res)
    srv = ed.ed_serve_open(ctx, 1 << 10, 4)
    A, B = reqs[0]
    assert ed.ed_serve_submit(srv, A, B, 0) == ed.ED_ENOMEM
    ed.ed_serve_close(srv)


def test_invalid_argument_matrix(ed, make_ctx):
    # every entry point refuses bad arguments with ED_EINVAL before touching memory
    import ctypes
    say("invalid arguments")
    ctx = make_ctx()
    other = make_ctx()
    A = synth.random_string(100, synth.CharDist("uniform", 4), 1)
    keep = (ctypes.c_uint8 * 100).from_buffer_copy(A.tobytes())
    out = ctypes.c_void_p()
    # NULL string with a positive length, and lengths at or past the limit
    assert ed.lib.ed_prepare(ctx, None, 5, keep, 100, 0, None, ctypes.byref(out)) == ed.ED_EINVAL
    assert ed.lib.ed_prepare(ctx, keep, 100, None, 1, 0, None, ctypes.byref(out)) == ed.ED_EINVAL
    assert ed.lib.ed_prepare(ctx, keep, ed.ED_MAX_LEN, keep, 100, 0, None, ctypes.byref(out)) == ed.ED_EINVAL
    assert ed.lib.ed_prepare(ctx, keep, 100, keep, 1 << 40, 0, None, ctypes.byref(out)) == ed.ED_EINVAL
    p = ed.ed_prepare(ctx, A, A)
    k = ctypes.c_uint64()
    cnt = ctypes.c_uint64()
    # a pair used with another context
    assert ed.lib.ed_distance(other, p, -1, ctypes.byref(k), None) == ed.ED_EINVAL
    assert ed.lib.ed_align(other, p, ctypes.byref(k), None, 0, ctypes.byref(cnt), None) == ed.ED_EINVAL
    # ed_align: missing outputs, a capacity without a buffer
    assert ed.lib.ed_align(ctx, p, None, None, 0, ctypes.byref(cnt), None) == ed.ED_EINVAL
    assert ed.lib.ed_align(ctx, p, ctypes.byref(k), None, 4, ctypes.byref(cnt), None) == ed.ED_EINVAL
    # runs outside the strings
    with pytest.raises(ed.EdError) as ei:
        ed.ed_debug_check_runs(ctx, p, [(90, 0, 20)])
    assert ei.value.status == ed.ED_EINVAL
    with pytest.raises(ed.EdError) as ei:
        ed.ed_debug_check_runs(ctx, p, [(-1, 0, 5)])
    assert ei.value.status == ed.ED_EINVAL
    # a batch mixing engines
    hctx = make_ctx(engine=ed.ENGINE_HASH)
    q = ed.ed_prepare(hctx, A, A)
    arr = (ctypes.c_void_p * 2)(p.value, q.value)
    kout = (ctypes.c_uint64 * 2)()
    st = (ctypes.c_int32 * 2)()
    assert ed.lib.ed_batch(ctx, arr, 2, -1, kout, st, None) == ed.ED_EINVAL
    ed.ed_release(q)
    ed.ed_release(p)


# ---------------------------------------------------------------------------
# dependent-access latency probe (the floor of a frontier round)
# ---------------------------------------------------------------------------
def test_dependent_access_latency_probe(ed, make_ctx):
    say("latency probe")
    ctx = make_ctx()
    cached = ed.ed_debug_mem_latency(ctx, 1 << 20, 2000, warm=True)
    cold = ed.ed_debug_mem_latency(ctx, 1 << 32, 4000, warm=False)
    print("dependent access: 1 MiB warm %.0f ns, 4 GiB cold %.0f ns" % (cached, cold))
    assert 20 < cached < cold < 50000
    for bad in [(3 << 20, 10), (1 << 12, 10), (1 << 20, 0)]:
        with pytest.raises(ed.EdError) as ei:
            ed.ed_debug_mem_latency(ctx, *bad)
        assert ei.value.status == ed.ED_EINVAL
