"""Seeded synthetic inputs for the edit-distance workloads.

This module holds no edit-distance arithmetic: it only draws strings and
planted edits.  Both the oracle-driven tests and the GPU path take their inputs
from here, so that the two sides see identical bytes.

Random numbers come from a counter-based generator built on splitmix64's output
function (Steele, Lea, Flood 2014; constants as published by Vigna):

    mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
            z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
    key(seed, stream) = mix(mix(seed + G) + (stream + 1) * G),  G = 0x9E3779B97F4A7C15
    value(seed, stream, c) = mix(key + (c + 1) * G)             (counter c = 0, 1, ...)

Every quantity below draws from its own stream id, so changing one size never
shifts the numbers drawn for another quantity.

Planted edits follow the paper's synthetic workload: random characters, then k
edits whose types are uniform over insertion, deletion and substitution
(section 6, "Tested Algorithms and Datasets").  Where the paper leaves details
open, this module reads them as follows:
  * the k positions are distinct, uniform without replacement over [0, n);
  * an insertion puts the new character before A[p] and keeps A[p];
  * a deletion drops A[p];
  * a substitution replaces A[p] by a fresh draw, which may equal A[p] (a no-op);
  * new characters come from the same distribution as A;
  * the edits are applied in one left-to-right pass, so m = n + #ins - #del.
"""
import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

G = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22

# stream ids
S_CHARS = 1
S_POS = 2
S_TYPE = 3
S_NEWCH = 4
S_PERIOD = 5
S_PAIR_N = 10
S_PAIR_K = 11
S_PAIR_SEED = 12
S_ARRIVAL = 20
S_REQ_N = 21
S_REQ_K = 22
S_REQ_SEED = 23
S_REQ_SIGMA = 24


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z ^ (z >> np.uint64(30))
        z = z * _M1
        z = z ^ (z >> np.uint64(27))
        z = z * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _key(seed, stream):
    with np.errstate(over="ignore"):
        s = _mix(np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64) + G)
        k = _mix(s + np.uint64(stream + 1) * G)
    return k[0]


def draws(seed, stream, count, start=0):
    """uint64 values value(seed, stream, c) for c in [start, start+count)."""
    key = _key(seed, stream)
    c = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + c * G)


def _uniform_from(v, sigma):
    # multiply-shift on the high 32 bits: exact for powers of two
    return (((v >> np.uint64(32)) * np.uint64(sigma)) >> np.uint64(32)).astype(np.uint8)


def _unit_float(v):
    return (v >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def zipf_cdf(nsym=256, s=1.0):
    w = 1.0 / np.arange(1, nsym + 1, dtype=np.float64) ** s
    return np.cumsum(w) / w.sum()


def _zipf_guide(cdf):
    """Guide table (Chen and Asau): g[j] = #{cdf <= j / 2^16}, plus the cdf with a sentinel."""
    g = np.searchsorted(cdf, np.arange(1 << 16, dtype=np.float64) / 65536.0, side="right")
    return g.astype(np.int64), np.append(cdf, np.inf)


def _zipf_from(v, cdf, guide=None):
    """Symbol = #{cdf <= u} (clamped to the last symbol), u = top 53 bits of v.

    The guide table starts the count at the bucket of u's top 16 bits (which are
    the top 16 bits of v); a short forward scan finishes it.  The result equals
    searchsorted(cdf, u, side="right") exactly.
    """
    u = _unit_float(v)
    if guide is None:
        guide = _zipf_guide(cdf)
    g, ext = guide
    idx = g[(v >> np.uint64(48)).astype(np.int64)]
    while True:
        adv = ext[idx] <= u
        if not adv.any():
            break
        idx += adv
    return np.minimum(idx, len(cdf) - 1).astype(np.uint8)


def _threads():
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return max(1, min(16, n or os.cpu_count() or 1))


class CharDist:
    """A character distribution: 'uniform' over sigma symbols or 'zipf'."""

    def __init__(self, kind="uniform", sigma=4, s=1.0):
        self.kind = kind
        self.sigma = sigma
        self.s = s
        self._cdf = zipf_cdf(sigma, s) if kind == "zipf" else None
        self._guide = _zipf_guide(self._cdf) if kind == "zipf" else None

    def from_draws(self, v):
        if self.kind == "uniform":
            return _uniform_from(v, self.sigma)
        return _zipf_from(v, self._cdf, self._guide)

    def sample(self, seed, stream, count, start=0):
        out = np.empty(count, dtype=np.uint8)

        def fill(a):
            b = min(count, a + _CHUNK)
            out[a:b] = self.from_draws(draws(seed, stream, b - a, start + a))

        starts = range(0, count, _CHUNK)
        if count > 2 * _CHUNK and _threads() > 1:
            # chunks are independent (counter-based draws); numpy releases the GIL
            with ThreadPoolExecutor(_threads()) as ex:
                list(ex.map(fill, starts))
        else:
            for a in starts:
                fill(a)
        return out


def random_string(n, dist, seed, stream=S_CHARS):
    return dist.sample(seed, stream, n)


def periodic_string(n, dist, seed, period=64):
    block = dist.sample(seed, S_PERIOD, period)
    reps = -(-n // period) if n else 0
    return np.tile(block, reps)[:n].copy()


def _distinct_positions(n, k, seed, stream):
    """k distinct positions uniform without replacement over [0, n), in draw order."""
    if k <= 0 or n <= 0:
        return np.empty(0, dtype=np.int64)
    k = min(k, n)
    if k * 2 > n:
        # dense case: a seeded permutation by sorting random keys
        v = draws(seed, stream, n)
        return np.argsort(v, kind="stable")[:k].astype(np.int64)
    got = np.empty(0, dtype=np.int64)
    start = 0
    want = k + k // 8 + 16
    while True:
        v = draws(seed, stream, want, start)
        start += want
        cand = (v % np.uint64(n)).astype(np.int64)
        allc = np.concatenate([got, cand])
        _, first = np.unique(allc, return_index=True)
        first.sort()
        uniq = allc[first]
        if len(uniq) >= k:
            return uniq[:k]
        got = uniq
        want = 2 * (k - len(got)) + 16


def plant_edits(A, k, dist, seed):
    """Apply k planted unit edits to A; returns (B, info dict)."""
    A = np.ascontiguousarray(A, dtype=np.uint8)
    n = len(A)
    pos = _distinct_positions(n, k, seed, S_POS)
    kk = len(pos)
    types = (draws(seed, S_TYPE, kk) % np.uint64(3)).astype(np.int8)  # 0 ins, 1 del, 2 sub
    newc = dist.sample(seed, S_NEWCH, kk)
    ins = types == 0
    dele = types == 1
    sub = types == 2
    B = A.copy()
    B[pos[sub]] = newc[sub]
    noop = int(np.count_nonzero(A[pos[sub]] == newc[sub]))
    keep = np.ones(n, dtype=bool)
    keep[pos[dele]] = False
    reduced = B[keep]
    ipos = np.sort(pos[ins])
    order = np.argsort(pos[ins], kind="stable")
    ichars = newc[ins][order]
    # index of A[p] inside the reduced array = p - #deleted positions before p
    dsorted = np.sort(pos[dele])
    shift = np.searchsorted(dsorted, ipos, side="left")
    B = np.insert(reduced, ipos - shift, ichars)
    info = {"k_planted": kk, "ins": int(ins.sum()), "del": int(dele.sum()),
            "sub": int(sub.sum()), "noop_sub": noop}
    return np.ascontiguousarray(B, dtype=np.uint8), info


# --------------------------------------------------------------------------
# Workloads.  Each returns numpy uint8 arrays and a description.
# --------------------------------------------------------------------------

def single_pair(n, k, seed, sigma=4, kind="uniform", periodic=False):
    """A: n chars (uniform over sigma, or Zipf(1.0) over 256); B = A + k edits."""
    dist = CharDist(kind, sigma if kind == "uniform" else 256)
    A = periodic_string(n, dist, seed) if periodic else random_string(n, dist, seed)
    B, info = plant_edits(A, k, dist, seed)
    info.update({"n": n, "m": len(B), "dist": kind, "sigma": dist.sigma, "periodic": periodic})
    return A, B, info


def small_pair(seed):
    """n = 10,000 uniform over {0,1,2,3}, 100 planted edits."""
    return single_pair(10_000, 100, seed)


def batch_specs(count, seed, lo_exp=3.0, hi_exp=6.0, kfrac=0.01):
    """(n, k, pair_seed) for a batch: n = floor(10^U), U ~ U[lo, hi]; k ~ U{0..floor(kfrac n)}."""
    u = _unit_float(draws(seed, S_PAIR_N, count))
    n = np.floor(10.0 ** (lo_exp + (hi_exp - lo_exp) * u)).astype(np.int64)
    kv = draws(seed, S_PAIR_K, count)
    kmax = np.floor(kfrac * n).astype(np.int64)
    k = (kv % (kmax + 1).astype(np.uint64)).astype(np.int64)
    ps = draws(seed, S_PAIR_SEED, count)
    return [(int(n[i]), int(k[i]), int(ps[i])) for i in range(count)]


def batch_pairs(count, seed, lo_exp=3.0, hi_exp=6.0, kfrac=0.01, sigma=4):
    """Materialise the pairs of batch_specs (list of (A, B))."""
    out = []
    for n, k, ps in batch_specs(count, seed, lo_exp, hi_exp, kfrac):
        A, B, _ = single_pair(n, k, ps, sigma=sigma)
        out.append((A, B))
    return out


def arrival_trace(count, seed, rate_per_s, lo_exp=2.0, hi_exp=7.0, kfrac=0.05, sigmas=(4, 20)):
    """Poisson arrivals: list of dicts {t_arrive_s, n, k, sigma, seed}."""
    u = _unit_float(draws(seed, S_ARRIVAL, count))
    gaps = -np.log1p(-u) / float(rate_per_s)
    t = np.cumsum(gaps)
    un = _unit_float(draws(seed, S_REQ_N, count))
    n = np.floor(10.0 ** (lo_exp + (hi_exp - lo_exp) * un)).astype(np.int64)
    kmax = np.floor(kfrac * n).astype(np.int64)
    k = (draws(seed, S_REQ_K, count) % (kmax + 1).astype(np.uint64)).astype(np.int64)
    sg = draws(seed, S_REQ_SIGMA, count) % np.uint64(len(sigmas))
    rs = draws(seed, S_REQ_SEED, count)
    return [{"t_arrive_s": float(t[i]), "n": int(n[i]), "k": int(k[i]),
             "sigma": int(sigmas[int(sg[i])]), "seed": int(rs[i])} for i in range(count)]


def request_pair(req):
    return single_pair(req["n"], req["k"], req["seed"], sigma=req["sigma"])[:2]


def log_uniform_mean(lo_exp, hi_exp):
    """E[10^U] for U ~ U[lo, hi] (used to size workloads)."""
    a, b = 10.0 ** lo_exp, 10.0 ** hi_exp
    return (b - a) / (math.log(b) - math.log(a))
