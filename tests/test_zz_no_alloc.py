"""ed_distance_noalloc (rows in the library's fixed device array) against
ed_distance (rows from the pool) and the oracle, through the C ABI.

Two calls in a row on each engine, the second on a smaller pair, so that the
second call runs over the contents the first one left in the array; a k_max
cutoff; and the argument checks (k_max outside [0, ED_NOALLOC_MAX_K]).
"""
import ctypes
import sys

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


@pytest.mark.parametrize("engine", [0, 1])
def test_noalloc_matches_distance_twice(ed, orc, engine):
    ctx = ed.ed_init(0, engine=engine)
    try:
        # first a pair whose frontier leaves the one-workgroup phase (about
        # 1800 rounds), then a smaller one over the rows the first one left
        for n, k, seed in ((1_000_000, 2000, 41), (10_000, 100, 42)):
            A, B, _ = synth.single_pair(n, k, seed)
            want = orc.lv_omp(A, B)
            say("noalloc", engine, n, k, "oracle", want)
            p = ed.ed_prepare(ctx, A, B)
            try:
                kmax = ed.NOALLOC_MAX_K
                got = ed.ed_distance_noalloc(ctx, p, kmax)
                ref = ed.ed_distance(ctx, p, kmax)
                assert got == ref == want
                # the band cutoff: k_max + 1 when the distance is larger
                cut = want // 2
                assert ed.ed_distance_noalloc(ctx, p, cut) == ed.ed_distance(ctx, p, cut) == cut + 1
                assert ed.ed_distance_noalloc(ctx, p, want) == want
            finally:
                ed.ed_release(p)
    finally:
        ed.ed_shutdown(ctx)


def test_noalloc_rejects_k_max_outside_the_array(ed):
    ctx = ed.ed_init(0)
    try:
        A, B, _ = synth.single_pair(1000, 10, 3)
        p = ed.ed_prepare(ctx, A, B)
        try:
            k = ctypes.c_uint64()
            for bad in (-1, ed.NOALLOC_MAX_K + 1):
                assert ed.lib.ed_distance_noalloc(ctx, p, bad, ctypes.byref(k), None) == ed.ED_EINVAL
            assert ed.lib.ed_distance_noalloc(ctx, p, 0, None, None) == ed.ED_EINVAL
            assert ed.lib.ed_distance_noalloc(None, p, 0, ctypes.byref(k), None) == ed.ED_EINVAL
            # still usable after the rejected calls
            assert ed.ed_distance_noalloc(ctx, p, 100) == ed.ed_distance(ctx, p)
        finally:
            ed.ed_release(p)
    finally:
        ed.ed_shutdown(ctx)
