"""CPU oracle for exact edit distance: ctypes wrapper around ``oracle.c``.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product library never does.
It shares no code with the HIP path.

Every function follows a passage of "Efficient Parallel Output-Sensitive Edit
Distance" (ESA 2023); the C file lists which.  ``build()`` compiles the shared
object with gcc (OpenMP on) next to this file.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ORACLE_SANITIZED=1 loads the AddressSanitizer / UndefinedBehaviorSanitizer
# build instead (the process must preload libasan; see tests/test_oracle_sanitized.py)
_SANITIZED = os.environ.get("ORACLE_SANITIZED") == "1"
_LIB = os.path.join(_HERE, "liboracle_san.so" if _SANITIZED else "liboracle.so")

NONE = -(1 << 30)

_lib = None


def build(force=True, sanitized=None):
    """Compile liboracle.so (gcc -O2 -fopenmp), or with sanitized=True the
    AddressSanitizer + UndefinedBehaviorSanitizer build liboracle_san.so."""
    san = _SANITIZED if sanitized is None else sanitized
    lib = os.path.join(_HERE, "liboracle_san.so" if san else "liboracle.so")
    if not force and os.path.exists(lib) and os.path.getmtime(lib) >= os.path.getmtime(_SRC):
        return lib
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]
    if san:
        cmd += ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.check_call(cmd + ["-o", tmp, _SRC])
    os.replace(tmp, lib)
    return lib


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i32p = ctypes.POINTER(ctypes.c_int32)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i64 = ctypes.c_int64
    lib.orc_dp_ed.argtypes = [u8p, i64, u8p, i64]
    lib.orc_dp_ed.restype = i64
    lib.orc_dp_matrix.argtypes = [u8p, i64, u8p, i64, i32p]
    lib.orc_dp_matrix.restype = ctypes.c_int
    lib.orc_rt_dump.argtypes = [u8p, i64, u8p, i64, i32p, i64]
    lib.orc_rt_dump.restype = i64
    lib.orc_brute_count.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.orc_brute_count.restype = i64
    lib.orc_brute_from.argtypes = [u8p, ctypes.c_int, ctypes.c_int, ctypes.c_int, i32p]
    lib.orc_brute_from.restype = i64
    lib.orc_lcp.argtypes = [u8p, i64, u8p, i64, i64, i64]
    lib.orc_lcp.restype = i64
    lib.orc_lv_naive.argtypes = [u8p, i64, u8p, i64, i64, i32p, i64]
    lib.orc_lv_naive.restype = i64
    lib.orc_hash_base.argtypes = [ctypes.c_uint64]
    lib.orc_hash_base.restype = ctypes.c_uint64
    lib.orc_substr_hash.argtypes = [u8p, i64, i64, ctypes.c_uint64]
    lib.orc_substr_hash.restype = ctypes.c_uint64
    lib.orc_horner_table.argtypes = [u8p, i64, i64, ctypes.c_uint64, u64p]
    lib.orc_horner_table.restype = ctypes.c_int
    lib.orc_lv_omp.argtypes = [u8p, i64, u8p, i64, i64, ctypes.c_int]
    lib.orc_lv_omp.restype = i64
    lib.orc_omp_max_threads.argtypes = []
    lib.orc_omp_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _u8(a):
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def dp_ed(A, B):
    """Edit distance by the two-row DP of section 1."""
    A, pa = _u8(A)
    B, pb = _u8(B)
    r = _load().orc_dp_ed(pa, len(A), pb, len(B))
    if r < 0:
        raise MemoryError("orc_dp_ed")
    return int(r)


def dp_matrix(A, B):
    """Full DP matrix G (section 1), shape (n+1, m+1), int32."""
    A, pa = _u8(A)
    B, pb = _u8(B)
    G = np.empty((len(A) + 1, len(B) + 1), dtype=np.int32)
    _load().orc_dp_matrix(pa, len(A), pb, len(B), G.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return G


def rt_dump(A, B):
    """Frontier rows R_t[i] = max{x : G[x][x-i] <= t} for t = 0..ED.

    Returns (ed, flat int32 array); row t sits at offset t*t, entries i=-t..t.
    """
    A, pa = _u8(A)
    B, pb = _u8(B)
    cap = (max(len(A), len(B)) + 1) ** 2
    out = np.empty(cap, dtype=np.int32)
    ed = _load().orc_rt_dump(pa, len(A), pb, len(B),
                             out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    if ed < 0:
        raise MemoryError("orc_rt_dump")
    return int(ed), out[: (ed + 1) ** 2].copy()


def brute_count(sigma, maxlen):
    return int(_load().orc_brute_count(sigma, maxlen))


def brute_index(s, sigma):
    """Vertex index of string s in orc_brute_from's numbering."""
    off = sum(sigma ** l for l in range(len(s)))
    v = 0
    for c in s:
        v = v * sigma + int(c)
    return off + v


def brute_from(A, sigma, maxlen):
    """Distances from A to every string of length <= maxlen (BFS over strings)."""
    A, pa = _u8(A)
    total = brute_count(sigma, maxlen)
    dist = np.empty(total, dtype=np.int32)
    r = _load().orc_brute_from(pa, len(A), sigma, maxlen,
                               dist.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if r < 0:
        raise ValueError("orc_brute_from: bad arguments")
    return dist


def lcp(A, B, x, y):
    """LCP(A, B, x, y) by the character loop of section 2."""
    A, pa = _u8(A)
    B, pb = _u8(B)
    return int(_load().orc_lcp(pa, len(A), pb, len(B), x, y))


def lv_naive(A, B, k_max=-1, dump=False):
    """Algorithm 1, sequential and literal; returns ED (or k_max+1).

    With dump=True returns (ed, rows) where rows has (ed+1)^2 int32 entries.
    """
    A, pa = _u8(A)
    B, pb = _u8(B)
    lib = _load()
    if not dump:
        r = lib.orc_lv_naive(pa, len(A), pb, len(B), k_max, None, 0)
        if r < 0:
            raise RuntimeError("orc_lv_naive failed")
        return int(r)
    kcap = max(len(A), len(B)) + 1
    if k_max >= 0:
        kcap = min(kcap, k_max + 1)
    cap = (kcap + 1) ** 2
    out = np.empty(cap, dtype=np.int32)
    r = lib.orc_lv_naive(pa, len(A), pb, len(B), k_max,
                         out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
    if r < 0:
        raise RuntimeError("orc_lv_naive failed")
    rows = min(r, kcap - 1) if k_max >= 0 and r > k_max else r
    return int(r), out[: (rows + 1) ** 2].copy()


def hash_base(seed):
    """Base r of the hash, derived from a 64-bit seed (splitmix64, clamped)."""
    return int(_load().orc_hash_base(ctypes.c_uint64(seed & (2 ** 64 - 1))))


def substr_hash(A, l, r, base):
    A, pa = _u8(A)
    return int(_load().orc_substr_hash(pa, l, r, ctypes.c_uint64(base)))


def horner_table(A, b, base):
    """Blocked prefix table T[j] = h(A[0..jb)), j = 0..floor(n/b) (section 3.3)."""
    A, pa = _u8(A)
    T = np.empty(len(A) // b + 1, dtype=np.uint64)
    r = _load().orc_horner_table(pa, len(A), b, ctypes.c_uint64(base),
                                 T.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if r != 0:
        raise ValueError("orc_horner_table: bad block size")
    return T


def lv_omp(A, B, k_max=-1, threads=0):
    """Multicore Landau-Vishkin (the timed CPU baseline)."""
    A, pa = _u8(A)
    B, pb = _u8(B)
    r = _load().orc_lv_omp(pa, len(A), pb, len(B), k_max, threads)
    if r < 0:
        raise RuntimeError("orc_lv_omp failed")
    return int(r)


def omp_max_threads():
    return int(_load().orc_omp_max_threads())
