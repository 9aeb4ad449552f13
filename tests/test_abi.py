"""C-ABI checks that need no GPU: the library loads, exports every function
that include/ed.h declares, and its host-side helpers agree with the oracle."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "ed.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = set(re.findall(r"\b(ed_[a-z_0-9]+)\s*\(", src))
    return sorted(names)


def test_header_lists_match_binding():
    import paper_2306_17461_amd as ed
    assert sorted(ed.EXPORTS) == _declared_functions()


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2306_17461_amd", "libed.so"))
    for name in _declared_functions():
        assert hasattr(lib, name), name


def test_hash_base_matches_oracle(orc):
    import paper_2306_17461_amd as ed
    for seed in [0, 1, 0x5EED, 2 ** 63 + 5, 2 ** 64 - 1]:
        assert ed.ed_hash_base(seed) == orc.hash_base(seed)


def test_default_options_and_strerror():
    import paper_2306_17461_amd as ed
    o = ed.options()
    assert o.engine == ed.ENGINE_DIRECT and o.block == 32 and o.pack_bits == 0
    for s in [ed.ED_OK, ed.ED_EINVAL, ed.ED_ENOMEM, ed.ED_EDEVICE, ed.ED_EBUSY, ed.ED_EINTERNAL, 7]:
        assert isinstance(ed.ed_strerror(s), str) and ed.ed_strerror(s)


def test_init_rejects_bad_options_without_device():
    import paper_2306_17461_amd as ed
    for kw in [dict(engine=5), dict(pack_bits=3), dict(block=48), dict(block=8192),
               dict(lds_rounds=10 ** 6)]:
        with pytest.raises(ed.EdError) as ei:
            ed.ed_init(0, **kw)
        assert ei.value.status == ed.ED_EINVAL


def test_null_arguments_rejected():
    import paper_2306_17461_amd as ed
    assert ed.lib.ed_shutdown(None) == ed.ED_EINVAL
    assert ed.lib.ed_release(None) == ed.ED_EINVAL
    assert ed.lib.ed_distance(None, None, -1, None, None) == ed.ED_EINVAL
    assert ed.lib.ed_prepare(None, None, 0, None, 0, 1, None, None) == ed.ED_EINVAL


def test_binding_constants_match_the_header():
    import re
    import paper_2306_17461_amd as ed
    src = open(os.path.join(ROOT, "include", "ed.h")).read()
    consts = {m.group(1): m.group(2) for m in re.finditer(r"#define (ED_\w+) \(?\(?(?:uint64_t\))?(-?\d+)u?\)?", src)}
    assert int(consts["ED_MAX_LEN"]) == ed.ED_MAX_LEN
    for name, py in [("ED_FLAG_DEBUG_DUMP", "FLAG_DEBUG_DUMP"), ("ED_FLAG_NO_PHASE_A", "FLAG_NO_PHASE_A"),
                     ("ED_FLAG_SHUFFLE", "FLAG_SHUFFLE"), ("ED_FLAG_TIMING", "FLAG_TIMING"),
                     ("ED_FLAG_CERTIFY", "FLAG_CERTIFY"), ("ED_FLAG_WEAK_HASH", "FLAG_WEAK_HASH"),
                     ("ED_OP_MATCH", "OP_MATCH"), ("ED_OP_SUB", "OP_SUB"), ("ED_OP_DEL", "OP_DEL"),
                     ("ED_OP_INS", "OP_INS"), ("ED_ECOLLISION", "ED_ECOLLISION"), ("ED_EINVAL", "ED_EINVAL"),
                     ("ED_FLAG_NO_GRID_ROUNDS", "FLAG_NO_GRID_ROUNDS"), ("ED_FLAG_HASH_FIRST", "FLAG_HASH_FIRST"),
                     ("ED_BUF_PACKED2", "BUF_PACKED2"), ("ED_BUF_BYTES", "BUF_BYTES"), ("ED_BUF_TABLE", "BUF_TABLE"),
                     ("ED_BUF_PACKED4", "BUF_PACKED4"), ("ED_FLAG_ALIGN_SEGMENTS", "FLAG_ALIGN_SEGMENTS")]:
        assert int(consts[name]) == getattr(ed, py), name
