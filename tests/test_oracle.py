"""Pins for the CPU oracle: each oracle function is checked against something
other than itself -- brute force over strings, closed forms, identities that
the edit distance must satisfy, and published generator outputs.

Runs on the CPU only (no GPU marker).
"""
import itertools

import numpy as np
import pytest

import synth

P61 = (1 << 61) - 1


def all_strings(sigma, maxlen):
    for l in range(maxlen + 1):
        for s in itertools.product(range(sigma), repeat=l):
            yield np.array(s, dtype=np.uint8)


# ---------------------------------------------------------------------------
# DP (section 1) against breadth-first search over strings (definition).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("sigma,maxlen", [(2, 8), (3, 5)])
def test_dp_equals_brute_exhaustive(orc, sigma, maxlen):
    strs = list(all_strings(sigma, maxlen))
    idx = [orc.brute_index(s, sigma) for s in strs]
    for A in strs:
        dist = orc.brute_from(A, sigma, maxlen)
        for B, j in zip(strs, idx):
            assert orc.dp_ed(A, B) == dist[j], (A, B)


def test_dp_equals_brute_sampled_sigma4(orc):
    rng = np.random.default_rng(7)
    sigma, maxlen = 4, 7
    for _ in range(40):
        la = int(rng.integers(0, maxlen + 1))
        A = rng.integers(0, sigma, la).astype(np.uint8)
        dist = orc.brute_from(A, sigma, maxlen)
        for _ in range(50):
            lb = int(rng.integers(0, maxlen + 1))
            B = rng.integers(0, sigma, lb).astype(np.uint8)
            assert orc.dp_ed(A, B) == dist[orc.brute_index(B, sigma)]


def test_dp_matrix_prefixes_equal_brute(orc):
    """G[x][y] = ED(A[:x], B[:y]) for every prefix pair, checked by BFS."""
    rng = np.random.default_rng(3)
    sigma, maxlen = 3, 7
    for _ in range(12):
        A = rng.integers(0, sigma, int(rng.integers(0, 8))).astype(np.uint8)
        B = rng.integers(0, sigma, int(rng.integers(0, 8))).astype(np.uint8)
        G = orc.dp_matrix(A, B)
        assert G[len(A), len(B)] == orc.dp_ed(A, B)
        for x in range(len(A) + 1):
            dist = orc.brute_from(A[:x], sigma, maxlen)
            for y in range(len(B) + 1):
                assert G[x, y] == dist[orc.brute_index(B[:y], sigma)]


# ---------------------------------------------------------------------------
# Identities of the edit distance.
# ---------------------------------------------------------------------------
def _rand_pair(rng, sigma, n, k):
    A = rng.integers(0, sigma, n).astype(np.uint8)
    B, _ = synth.plant_edits(A, k, synth.CharDist("uniform", sigma), int(rng.integers(1 << 30)))
    return A, B


def test_identities(orc):
    rng = np.random.default_rng(11)
    for sigma in (2, 4, 20, 256):
        for _ in range(8):
            n = int(rng.integers(0, 300))
            A, B = _rand_pair(rng, sigma, n, int(rng.integers(0, 30)))
            d = orc.dp_ed(A, B)
            assert d == orc.dp_ed(B, A)
            assert orc.dp_ed(A, A) == 0
            assert orc.dp_ed(A, A[:0]) == len(A)
            assert abs(len(A) - len(B)) <= d <= max(len(A), len(B))
            if len(A) == len(B):
                assert d <= int(np.count_nonzero(A != B))
            if len(A):
                C = A.copy()
                p = int(rng.integers(len(A)))
                C[p] = (int(C[p]) + 1) % 256
                assert orc.dp_ed(A, C) == 1


def test_triangle_inequality(orc):
    rng = np.random.default_rng(5)
    for _ in range(60):
        X = rng.integers(0, 3, int(rng.integers(0, 40))).astype(np.uint8)
        Y = rng.integers(0, 3, int(rng.integers(0, 40))).astype(np.uint8)
        Z = rng.integers(0, 3, int(rng.integers(0, 40))).astype(np.uint8)
        assert orc.dp_ed(X, Z) <= orc.dp_ed(X, Y) + orc.dp_ed(Y, Z)


def test_planted_edit_bounds(orc):
    for seed in range(10):
        A, B, info = synth.single_pair(3000, 60, seed)
        d = orc.dp_ed(A, B)
        assert info["m"] == info["n"] + info["ins"] - info["del"]
        assert abs(info["ins"] - info["del"]) <= d <= info["k_planted"] - info["noop_sub"]


# ---------------------------------------------------------------------------
# LCP character loop (section 2) against slicing.
# ---------------------------------------------------------------------------
def test_lcp_char_loop(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        n, m = int(rng.integers(0, 60)), int(rng.integers(0, 60))
        sigma = int(rng.choice([1, 2, 4]))
        A = rng.integers(0, sigma, n).astype(np.uint8)
        B = rng.integers(0, sigma, m).astype(np.uint8)
        x, y = int(rng.integers(0, n + 1)), int(rng.integers(0, m + 1))
        L = 0
        while L <= min(n - x, m - y) and np.array_equal(A[x:x + L], B[y:y + L]):
            L += 1
        assert orc.lcp(A, B, x, y) == L - 1


# ---------------------------------------------------------------------------
# Algorithm 1 (naive LV) against the DP, and its frontier against R_t.
# ---------------------------------------------------------------------------
def test_lv_naive_equals_dp(orc):
    rng = np.random.default_rng(17)
    for sigma in (2, 4, 20, 256):
        for _ in range(10):
            n = int(rng.integers(0, 2000))
            A, B = _rand_pair(rng, sigma, n, int(rng.integers(0, max(1, n // 10) + 1)))
            assert orc.lv_naive(A, B) == orc.dp_ed(A, B)


def test_lv_naive_tiny_exhaustive(orc):
    strs = list(all_strings(2, 5))
    for A in strs:
        for B in strs:
            assert orc.lv_naive(A, B) == orc.dp_ed(A, B)


def test_rt_dump_against_brute(orc):
    """R_t[i] = max{x : ED(A[:x], B[:x-i]) <= t}, computed from BFS distances."""
    rng = np.random.default_rng(23)
    sigma, maxlen = 3, 7
    for _ in range(10):
        A = rng.integers(0, sigma, int(rng.integers(0, 8))).astype(np.uint8)
        B = rng.integers(0, sigma, int(rng.integers(0, 8))).astype(np.uint8)
        n, m = len(A), len(B)
        ed, rows = orc.rt_dump(A, B)
        E = np.empty((n + 1, m + 1), dtype=np.int64)
        for x in range(n + 1):
            dist = orc.brute_from(A[:x], sigma, maxlen)
            for y in range(m + 1):
                E[x, y] = dist[orc.brute_index(B[:y], sigma)]
        assert ed == E[n, m]
        for t in range(ed + 1):
            for i in range(-t, t + 1):
                xs = [x for x in range(n + 1) if 0 <= x - i <= m and E[x, x - i] <= t]
                want = max(xs) if xs else orc.NONE
                assert rows[t * t + i + t] == want, (t, i)


def test_lv_naive_frontier_equals_rt(orc):
    rng = np.random.default_rng(29)
    cases = [(np.zeros(0, np.uint8), np.zeros(0, np.uint8)),
             (np.zeros(0, np.uint8), np.array([1, 2, 3], np.uint8)),
             (np.array([1, 2, 3, 4], np.uint8), np.zeros(0, np.uint8))]
    for _ in range(60):
        sigma = int(rng.choice([2, 4, 20]))
        n = int(rng.integers(0, 90))
        A, B = _rand_pair(rng, sigma, n, int(rng.integers(0, 20)))
        cases.append((A, B))
    for A, B in cases:
        ed, rows = orc.rt_dump(A, B)
        ed2, rows2 = orc.lv_naive(A, B, dump=True)
        assert ed == ed2
        np.testing.assert_array_equal(rows, rows2)
        # the frontier only moves forward: f_t[i] >= f_{t-1}[i] where both exist
        for t in range(1, ed + 1):
            for i in range(-(t - 1), t):
                a, b = rows2[(t - 1) ** 2 + i + t - 1], rows2[t * t + i + t]
                if a != orc.NONE:
                    assert b >= a


def test_lv_naive_kmax_cutoff(orc):
    A, B, _ = synth.single_pair(500, 40, 1)
    ed = orc.dp_ed(A, B)
    assert orc.lv_naive(A, B, k_max=ed) == ed
    assert orc.lv_naive(A, B, k_max=ed - 1) == ed
    assert orc.lv_naive(A, B, k_max=ed // 2) == ed // 2 + 1


def test_lv_omp_equals_naive(orc):
    rng = np.random.default_rng(31)
    for sigma in (2, 4, 256):
        for _ in range(6):
            n = int(rng.integers(0, 3000))
            A, B = _rand_pair(rng, sigma, n, int(rng.integers(0, max(1, n // 20) + 1)))
            want = orc.dp_ed(A, B)
            assert orc.lv_naive(A, B) == want
            assert orc.lv_omp(A, B, threads=4) == want
    A, B, _ = synth.single_pair(10 ** 6, 300, 4)
    assert orc.lv_omp(A, B) == orc.lv_naive(A, B)
    assert orc.lv_omp(A, B, k_max=10) == 11


# ---------------------------------------------------------------------------
# Hash (section 2) and prefix tables (sections 3.2, 3.3).
# ---------------------------------------------------------------------------
def test_hash_base_splitmix_vector(orc):
    # splitmix64 published first output for state 0 is 0xE220A8397B1DCDAF
    z = 0xE220A8397B1DCDAF
    assert orc.hash_base(0) == (1 << 20) + z % (P61 - (1 << 21))
    for s in range(50):
        r = orc.hash_base(s * 7919 + 1)
        assert (1 << 20) <= r < P61 - (1 << 20)


def test_hash_closed_forms(orc):
    r = orc.hash_base(42)
    for L in (1, 2, 5, 64, 1000):
        ones = np.ones(L, np.uint8)
        geo = (pow(r, L, P61) - 1) * pow(r - 1, P61 - 2, P61) % P61
        assert orc.substr_hash(ones, 0, L, r) == geo
        single = np.zeros(L, np.uint8)
        single[0] = 200
        assert orc.substr_hash(single, 0, L, r) == 200 * pow(r, L - 1, P61) % P61


def test_hash_power_sum_and_concat(orc):
    rng = np.random.default_rng(13)
    r = orc.hash_base(9)
    for _ in range(20):
        A = rng.integers(0, 256, int(rng.integers(1, 300))).astype(np.uint8)
        n = len(A)
        want = sum(int(A[i]) * pow(r, n - 1 - i, P61) for i in range(n)) % P61
        assert orc.substr_hash(A, 0, n, r) == want
        s = int(rng.integers(0, n + 1))
        h1, h2 = orc.substr_hash(A, 0, s, r), orc.substr_hash(A, s, n, r)
        assert (h1 * pow(r, n - s, P61) + h2) % P61 == want
        # linearity in the characters
        B = rng.integers(0, 100, n).astype(np.uint8)
        C = (A.astype(np.int64) % 100 + B).astype(np.uint8)
        lin = (orc.substr_hash((A % 100).astype(np.uint8), 0, n, r) + orc.substr_hash(B, 0, n, r)) % P61
        assert orc.substr_hash(C, 0, n, r) == lin


@pytest.mark.parametrize("b", [1, 2, 8, 32, 64])
def test_horner_table_blocks(orc, b):
    rng = np.random.default_rng(b)
    r = orc.hash_base(b + 100)
    for n in [0, 1, b - 1, b, b + 1, 3 * b + (b // 2), 257]:
        if n < 0:
            continue
        A = rng.integers(0, 256, n).astype(np.uint8)
        T = orc.horner_table(A, b, r)
        assert len(T) == n // b + 1 and T[0] == 0
        for j in range(1, n // b + 1):
            L = j * b
            want = sum(int(A[i]) * pow(r, L - 1 - i, P61) for i in range(L)) % P61
            assert int(T[j]) == want
        T1 = orc.horner_table(A, 1, r)
        np.testing.assert_array_equal(T1[::b][: len(T)], T)


# ---------------------------------------------------------------------------
# Generator sanity.
# ---------------------------------------------------------------------------
def test_generator_determinism_and_shape():
    A1, B1, i1 = synth.single_pair(5000, 50, 3)
    A2, B2, i2 = synth.single_pair(5000, 50, 3)
    assert np.array_equal(A1, A2) and np.array_equal(B1, B2) and i1 == i2
    assert A1.max() <= 3
    Az, _, _ = synth.single_pair(20000, 10, 1, kind="zipf")
    counts = np.bincount(Az, minlength=256)
    assert counts[0] > counts[1] > counts[3]  # rank 1 is the most frequent
    Ap, _, _ = synth.single_pair(1000, 0, 2, kind="zipf", periodic=True)
    assert np.array_equal(Ap[:64], Ap[64:128])
    specs = synth.batch_specs(100, 0)
    assert all(1000 <= n <= 10 ** 6 and 0 <= k <= n // 100 for n, k, _ in specs)
