"""Exact output-sensitive edit distance on AMD MI355X: Python binding of libed.so.

The binding only marshals arguments: every step of the computation runs in the
HIP kernels of ``libed.so`` (see ``include/ed.h``).  PyTorch supplies device
memory and streams; numpy arrays are accepted as host inputs.

    import paper_2306_17461_amd as ed
    ctx = ed.ed_init(0, engine=ed.ENGINE_DIRECT)
    pair = ed.ed_prepare(ctx, A, B)          # torch uint8 tensors (cuda or cpu) or numpy
    k = ed.ed_distance(ctx, pair)
    ed.ed_release(pair); ed.ed_shutdown(ctx)

Importing this module loads libed.so and raises ImportError if it is missing:
there is no fallback implementation.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libed.so")

ED_OK = 0
ED_EINVAL = -1
ED_ENOMEM = -2
ED_EDEVICE = -3
ED_ECOLLISION = -4
ED_EBUSY = -5
ED_EINTERNAL = -6
ENGINE_DIRECT = 0
ENGINE_HASH = 1
FLAG_DEBUG_DUMP = 1
FLAG_NO_PHASE_A = 2
FLAG_SHUFFLE = 4
FLAG_TIMING = 8
FLAG_CERTIFY = 16
FLAG_WEAK_HASH = 32
FLAG_NO_GRID_ROUNDS = 64
FLAG_HASH_FIRST = 128
FLAG_ALIGN_SEGMENTS = 256
ED_MAX_LEN = 2146435072  # 2^31 - 2^20 characters
OP_MATCH, OP_SUB, OP_DEL, OP_INS = 0, 1, 2, 3
BUF_PACKED2 = 0
BUF_BYTES = 1
BUF_TABLE = 2
BUF_PACKED4 = 3
NONE = -(1 << 30)
NOALLOC_MAX_K = 500000
MAX_LEN = 2146435072


class EdError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        super().__init__("%s: %s (%d): %s" % (where, _strerror(status), status, _last_error()))


class ed_options(ctypes.Structure):
    _fields_ = [("engine", ctypes.c_uint32), ("pack_bits", ctypes.c_uint32),
                ("block", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("hash_seed", ctypes.c_uint64), ("lds_rounds", ctypes.c_uint32),
                ("lane_words", ctypes.c_uint32), ("grid_blocks", ctypes.c_uint32),
                ("init_rows", ctypes.c_uint32), ("block_rounds", ctypes.c_uint32),
                ("chunk_diags", ctypes.c_uint32), ("task_lds_rounds", ctypes.c_uint32),
                ("task_block_rounds", ctypes.c_uint32)]


class ed_tune_result(ctypes.Structure):
    _fields_ = [("best", ed_options), ("default_ms", ctypes.c_double), ("best_ms", ctypes.c_double),
                ("evaluated", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class ed_stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("m", ctypes.c_uint64),
                ("bits_per_char", ctypes.c_uint32), ("engine", ctypes.c_uint32),
                ("rounds", ctypes.c_uint64), ("updates", ctypes.c_uint64),
                ("lcp_chars", ctypes.c_uint64), ("wave_lcps", ctypes.c_uint64),
                ("grid_lcps", ctypes.c_uint64), ("hash_queries", ctypes.c_uint64),
                ("hash_probes", ctypes.c_uint64), ("collisions", ctypes.c_uint64),
                ("collision_bound", ctypes.c_double), ("launches", ctypes.c_uint64),
                ("ns_prepare", ctypes.c_double), ("ns_distance", ctypes.c_double),
                ("gpu_ns_prepare_kernel", ctypes.c_double),
                ("gpu_ns_frontier_kernel", ctypes.c_double),
                ("rounds_phase_a", ctypes.c_uint64), ("us_phase_a", ctypes.c_double),
                ("us_phase_b", ctypes.c_double), ("gpu_ns_lcp_kernel", ctypes.c_double),
                ("wg_lcps", ctypes.c_uint64), ("gpu_ns_table_kernel", ctypes.c_double),
                ("certify_retries", ctypes.c_uint64), ("align_device_bytes", ctypes.c_uint64),
                ("align_segment_rounds", ctypes.c_uint64)]


class ed_op_run(ctypes.Structure):
    _fields_ = [("op", ctypes.c_uint32), ("pad", ctypes.c_uint32), ("len", ctypes.c_uint64)]


class ed_result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("k", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("t_arrive_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64)]


# every symbol declared in include/ed.h
EXPORTS = [
    "ed_default_options", "ed_hash_base", "ed_init", "ed_set_options", "ed_get_options",
    "ed_shutdown", "ed_prepare", "ed_release", "ed_distance", "ed_distance_noalloc", "ed_distance_dump", "ed_align", "ed_batch",
    "ed_autotune_batch", "ed_pair_stats", "ed_pair_buffer", "ed_debug_lcp", "ed_debug_check_runs",
    "ed_debug_mem_latency", "ed_serve_open",
    "ed_serve_submit", "ed_serve_submit_band",
    "ed_serve_poll", "ed_serve_drain", "ed_serve_close", "ed_strerror", "ed_last_error",
]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libed.so not built at %s (run __graft_entry__.build() or "
                          "python paper_2306_17461_amd/build.py)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    u64 = ctypes.c_uint64
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "ed_default_options": (None, [P(ed_options)]),
        "ed_hash_base": (u64, [u64]),
        "ed_init": (i32, [P(vp), i32, P(ed_options)]),
        "ed_set_options": (i32, [vp, P(ed_options)]),
        "ed_get_options": (i32, [vp, P(ed_options)]),
        "ed_shutdown": (i32, [vp]),
        "ed_prepare": (i32, [vp, vp, u64, vp, u64, i32, vp, P(vp)]),
        "ed_release": (i32, [vp]),
        "ed_distance": (i32, [vp, vp, i64, P(u64), vp]),
        "ed_distance_noalloc": (i32, [vp, vp, i64, P(u64), vp]),
        "ed_distance_dump": (i32, [vp, vp, i64, P(u64), vp, u64, vp]),
        "ed_align": (i32, [vp, vp, P(u64), P(ed_op_run), u64, P(u64), vp]),
        "ed_batch": (i32, [vp, P(vp), u64, i64, P(u64), P(ctypes.c_int32), vp]),
        "ed_autotune_batch": (i32, [vp, P(vp), u64, i64, ctypes.c_uint32, P(ed_tune_result), vp]),
        "ed_pair_stats": (i32, [vp, P(ed_stats)]),
        "ed_pair_buffer": (i32, [vp, vp, i32, i32, vp, u64, P(u64)]),
        "ed_debug_lcp": (i32, [vp, vp, i32, vp, vp, u64, vp, vp]),
        "ed_debug_check_runs": (i32, [vp, vp, vp, vp, vp, u64, P(ctypes.c_uint32), vp]),
        "ed_debug_mem_latency": (i32, [vp, u64, ctypes.c_uint32, i32, P(ctypes.c_double)]),
        "ed_serve_open": (i32, [vp, u64, ctypes.c_uint32, P(vp)]),
        "ed_serve_submit": (i32, [vp, vp, u64, vp, u64, u64]),
        "ed_serve_submit_band": (i32, [vp, vp, u64, vp, u64, u64, i64]),
        "ed_serve_poll": (i32, [vp, P(ed_result), ctypes.c_uint32, P(ctypes.c_uint32)]),
        "ed_serve_drain": (i32, [vp]),
        "ed_serve_close": (i32, [vp]),
        "ed_strerror": (ctypes.c_char_p, [i32]),
        "ed_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


lib = _load()


def _strerror(s):
    return lib.ed_strerror(s).decode()


def _last_error():
    return lib.ed_last_error().decode()


def _check(rc, where):
    if rc != ED_OK:
        raise EdError(rc, where)


def _stream_handle(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available() and torch.cuda.is_initialized():
                return torch.cuda.current_stream().cuda_stream
        except Exception:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _buffer(x):
    """(pointer, length, on_device, keepalive) for a torch tensor or numpy array."""
    if x is None:
        return None, 0, 1, None
    try:
        import torch
        if isinstance(x, torch.Tensor):
            if x.dtype != torch.uint8:
                raise TypeError("expected a uint8 tensor")
            if not x.is_contiguous():
                x = x.contiguous()
            return (x.data_ptr() if x.numel() else None), x.numel(), 1 if x.is_cuda else 0, x
    except ImportError:
        pass
    a = np.ascontiguousarray(x, dtype=np.uint8)
    return (a.ctypes.data if a.size else None), a.size, 0, a


def options(**kw):
    o = ed_options()
    lib.ed_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError("unknown option %r" % k)
        setattr(o, k, v)
    return o


def ed_hash_base(seed):
    return int(lib.ed_hash_base(seed & 0xFFFFFFFFFFFFFFFF))


def ed_init(device=0, **kw):
    o = options(**kw)
    h = ctypes.c_void_p()
    _check(lib.ed_init(ctypes.byref(h), device, ctypes.byref(o)), "ed_init")
    return h


def ed_set_options(ctx, **kw):
    o = options(**kw)
    _check(lib.ed_set_options(ctx, ctypes.byref(o)), "ed_set_options")


def ed_get_options(ctx):
    o = ed_options()
    _check(lib.ed_get_options(ctx, ctypes.byref(o)), "ed_get_options")
    return {f: getattr(o, f) for f, _ in o._fields_}


def ed_shutdown(ctx):
    _check(lib.ed_shutdown(ctx), "ed_shutdown")


def ed_prepare(ctx, A, B, stream=None):
    pa, n, da, ka = _buffer(A)
    pb, m, db, kb = _buffer(B)
    if n and m and da != db:
        raise ValueError("A and B must both be on the device or both on the host")
    on_dev = da if n else db
    h = ctypes.c_void_p()
    _check(lib.ed_prepare(ctx, pa, n, pb, m, on_dev, _stream_handle(stream), ctypes.byref(h)),
           "ed_prepare")
    return h


def ed_release(pair):
    _check(lib.ed_release(pair), "ed_release")


def ed_distance(ctx, pair, k_max=-1, stream=None):
    k = ctypes.c_uint64()
    _check(lib.ed_distance(ctx, pair, k_max, ctypes.byref(k), _stream_handle(stream)), "ed_distance")
    return int(k.value)


def ed_distance_noalloc(ctx, pair, k_max, stream=None):
    """ed_distance without device allocation: rows in the library's fixed
    array, 0 <= k_max <= NOALLOC_MAX_K."""
    k = ctypes.c_uint64()
    _check(lib.ed_distance_noalloc(ctx, pair, k_max, ctypes.byref(k), _stream_handle(stream)),
           "ed_distance_noalloc")
    return int(k.value)


def ed_distance_dump(ctx, pair, rows_cap, k_max=-1, stream=None):
    rows = np.empty(rows_cap, dtype=np.int32)
    k = ctypes.c_uint64()
    _check(lib.ed_distance_dump(ctx, pair, k_max, ctypes.byref(k), rows.ctypes.data, rows_cap,
                                _stream_handle(stream)), "ed_distance_dump")
    k = int(k.value)
    return k, rows[: (k + 1) ** 2].copy()


def ed_align(ctx, pair, stream=None):
    """(k, script): the edit distance and an optimal edit script, every run of
    matches checked on the device; script = [(op, length), ...] with op one of
    OP_MATCH, OP_SUB, OP_DEL, OP_INS."""
    k = ctypes.c_uint64()
    cnt = ctypes.c_uint64()
    cap = 4096
    while True:
        runs = (ed_op_run * cap)()
        rc = lib.ed_align(ctx, pair, ctypes.byref(k), runs, cap, ctypes.byref(cnt), _stream_handle(stream))
        if rc == ED_EINVAL and cnt.value > cap:
            cap = int(cnt.value)
            continue
        _check(rc, "ed_align")
        return int(k.value), [(int(runs[i].op), int(runs[i].len)) for i in range(cnt.value)]


def ed_debug_check_runs(ctx, pair, runs, stream=None):
    """runs = [(x, y, length), ...]: 1 if some A[x + j] != B[y + j], else 0."""
    r = np.asarray(runs, dtype=np.int32).reshape(-1, 3)
    x, y, ln = (np.ascontiguousarray(r[:, j]) for j in range(3))
    bad = ctypes.c_uint32()
    _check(lib.ed_debug_check_runs(ctx, pair, x.ctypes.data, y.ctypes.data, ln.ctypes.data, len(r),
                                   ctypes.byref(bad), _stream_handle(stream)), "ed_debug_check_runs")
    return int(bad.value)


def ed_debug_mem_latency(ctx, region_bytes, steps, warm=False):
    """Nanoseconds per dependent global access over a region of region_bytes."""
    ns = ctypes.c_double()
    _check(lib.ed_debug_mem_latency(ctx, region_bytes, steps, 1 if warm else 0, ctypes.byref(ns)),
           "ed_debug_mem_latency")
    return ns.value


def ed_batch(ctx, pairs, k_max=-1, stream=None, check=True):
    cnt = len(pairs)
    arr = (ctypes.c_void_p * max(cnt, 1))(*[p.value for p in pairs])
    kout = (ctypes.c_uint64 * max(cnt, 1))()
    st = (ctypes.c_int32 * max(cnt, 1))()
    rc = lib.ed_batch(ctx, arr, cnt, k_max, kout, st, _stream_handle(stream))
    if check:
        _check(rc, "ed_batch")
    return [int(kout[i]) for i in range(cnt)], [int(st[i]) for i in range(cnt)]


def ed_autotune_batch(ctx, pairs, k_max=-1, passes=0, stream=None):
    """Tunes the many-pair kernel on these pairs; returns the chosen knobs and timings."""
    cnt = len(pairs)
    arr = (ctypes.c_void_p * max(cnt, 1))(*[p.value for p in pairs])
    r = ed_tune_result()
    _check(lib.ed_autotune_batch(ctx, arr, cnt, k_max, passes, ctypes.byref(r), _stream_handle(stream)),
           "ed_autotune_batch")
    best = {f: getattr(r.best, f) for f, _ in r.best._fields_}
    return {"best": best, "default_ms": r.default_ms, "best_ms": r.best_ms, "evaluated": r.evaluated,
            "knobs": {k: best[k] for k in ("task_lds_rounds", "task_block_rounds", "chunk_diags")}}


def ed_pair_stats(pair):
    s = ed_stats()
    _check(lib.ed_pair_stats(pair, ctypes.byref(s)), "ed_pair_stats")
    return {f: getattr(s, f) for f, _ in s._fields_}


def ed_pair_buffer(ctx, pair, which, kind):
    ln = ctypes.c_uint64()
    _check(lib.ed_pair_buffer(ctx, pair, which, kind, None, 0, ctypes.byref(ln)), "ed_pair_buffer")
    out = np.empty(int(ln.value), dtype=np.uint8)
    _check(lib.ed_pair_buffer(ctx, pair, which, kind, out.ctypes.data if out.size else None,
                              out.size, ctypes.byref(ln)), "ed_pair_buffer")
    if kind == BUF_TABLE:
        return out.view(np.uint64)
    return out


def ed_debug_lcp(ctx, pair, x, y, engine=-1, stream=None):
    x = np.ascontiguousarray(x, dtype=np.int64)
    y = np.ascontiguousarray(y, dtype=np.int64)
    out = np.empty(len(x), dtype=np.int64)
    _check(lib.ed_debug_lcp(ctx, pair, engine, x.ctypes.data, y.ctypes.data, len(x),
                            out.ctypes.data, _stream_handle(stream)), "ed_debug_lcp")
    return out


def ed_serve_open(ctx, hbm_budget_bytes, max_slots):
    h = ctypes.c_void_p()
    _check(lib.ed_serve_open(ctx, hbm_budget_bytes, max_slots, ctypes.byref(h)), "ed_serve_open")
    return h


def ed_serve_submit(srv, A, B, tag):
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    return lib.ed_serve_submit(srv, A.ctypes.data if A.size else None, A.size,
                               B.ctypes.data if B.size else None, B.size, tag)


def ed_serve_submit_band(srv, A, B, tag, k_max):
    A = np.ascontiguousarray(A, dtype=np.uint8)
    B = np.ascontiguousarray(B, dtype=np.uint8)
    return lib.ed_serve_submit_band(srv, A.ctypes.data if A.size else None, A.size,
                                    B.ctypes.data if B.size else None, B.size, tag, k_max)


def ed_serve_poll(srv, max_results=1024):
    buf = (ed_result * max_results)()
    got = ctypes.c_uint32()
    _check(lib.ed_serve_poll(srv, buf, max_results, ctypes.byref(got)), "ed_serve_poll")
    return [{f: getattr(buf[i], f) for f, _ in ed_result._fields_} for i in range(got.value)]


def ed_serve_drain(srv):
    _check(lib.ed_serve_drain(srv), "ed_serve_drain")


def ed_serve_close(srv):
    _check(lib.ed_serve_close(srv), "ed_serve_close")


def ed_strerror(status):
    return _strerror(status)


def ed_last_error():
    return _last_error()
