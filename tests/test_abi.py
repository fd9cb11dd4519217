"""CPU-side checks of the C ABI: the library loads, exports every function
include/stablemerge.h declares, and rejects bad arguments before launching
anything (no GPU is touched: every call here fails host-side validation)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "include")


def declared_functions():
    names = set()
    for fn in os.listdir(HEADER_DIR):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(HEADER_DIR, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for mt in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            if not mt.group(0).lstrip().startswith(("typedef", "#", "return")):
                names.add(mt.group(1))
    return names


@pytest.fixture(scope="module")
def sm():
    import paper_1202_6575_amd as m
    return m


def test_exports_every_declared_symbol(sm):
    lib = ctypes.CDLL(sm.LIB_PATH)
    names = declared_functions()
    assert {"stable_merge", "stable_merge_partition", "stable_merge_workspace_bytes",
            "sm_last_error"} <= names
    for name in sorted(names):
        assert hasattr(lib, name), f"{name} declared in include/ but not exported"


def call_merge(sm, keys=0x10000, pay=None, n=10, m=10, out=0x20000, opay=None, dtype=1,
               ws=0x30000, ws_bytes=1 << 20, opts=None):
    o = opts if opts is not None else sm.Options()
    return sm._lib.stable_merge(keys, pay, n, m, out, opay, dtype, ws, ws_bytes,
                                ctypes.byref(o), None)


def test_error_paths(sm):
    assert call_merge(sm, dtype=7) == -2
    assert call_merge(sm, n=-1) == -1
    assert call_merge(sm, pay=0x40000) == -1                      # payload without out_payloads
    assert call_merge(sm, keys=None) == -1
    assert call_merge(sm, keys=0x10004) == -1                     # not 16-byte aligned
    assert call_merge(sm, out=0x10000 + 16) == -3                 # out overlaps keys
    assert call_merge(sm, ws_bytes=8) == -4
    assert call_merge(sm, ws=None) == -4
    assert b"workspace" in sm._lib.sm_last_error()
    o = sm.Options()
    o.p_a = -3
    assert call_merge(sm, opts=o) == -1
    o = sm.Options()
    o.tile = 1 << 15                                               # subproblem too big for LDS
    assert call_merge(sm, opts=o) == -1
    o = sm.Options()
    o.tile = -5
    assert call_merge(sm, opts=o) == -1
    assert call_merge(sm, n=0, m=0) == 0                           # nothing to do


def test_partition_error_paths(sm):
    f = sm._lib.stable_merge_partition
    assert f(0x10000, 10, 10, 0, 1, 1, 0x20000, 0x30000, None) == -1
    assert f(0x10000, 10, 10, 1, 1, 9, 0x20000, 0x30000, None) == -2
    assert f(0x10000, 10, 10, 1, 1, 1, None, 0x30000, None) == -1


def test_workspace_bytes(sm):
    import torch
    w = sm.workspace_bytes(1 << 20, 1 << 19, torch.uint32)
    assert w >= ((1 << 20) // 2048 + (1 << 19) // 2048 + 2) * 8
    assert sm.workspace_bytes(-1, 3, torch.uint32) == 0
    assert sm.workspace_bytes(100, 100, torch.uint32, p_a=5, p_b=5) == 256 + 256 + 512
    # forced p with subproblems beyond one workgroup: the second-level state is added
    big = sm.workspace_bytes(1 << 20, 1 << 20, torch.uint32, p_a=2, p_b=2)
    assert big > 256 + 256 + 256 + ((1 << 21) // 2048) * 32
    assert sm.pieces_workspace_bytes(100, 100, 5, 5, torch.uint32) == 512
    assert sm.pieces_workspace_bytes(100, 100, 0, 5, torch.uint32) == 0
    assert sm.batched_workspace_bytes(10, 1000, torch.uint32) > 10 * 32
    assert sm.batched_workspace_bytes(-1, 1000, torch.uint32) == 0


def test_batched_error_paths(sm):
    f = sm._lib.stable_merge_batched
    o = sm.Options()
    args = dict(keys=0x10000, pay=None, offs=0x50000, na=0x60000, count=4, total=100,
                out=0x20000, opay=None, dtype=1, ws=0x30000, ws_bytes=1 << 20)

    def call(**kw):
        a = dict(args, **kw)
        return f(a["keys"], a["pay"], a["offs"], a["na"], a["count"], a["total"], a["out"],
                 a["opay"], a["dtype"], a["ws"], a["ws_bytes"], ctypes.byref(o), None)
    assert call(dtype=6) == -2
    assert call(count=-1) == -1
    assert call(offs=None) == -1
    assert call(out=0x10000) == -3
    assert call(ws_bytes=16) == -4
    assert call(count=0) == 0
    assert call(total=0) == 0


def test_version(sm):
    assert sm._lib.sm_version() >= 100


def test_learned_merge_error_paths(sm):
    from paper_1202_6575_amd import learned  # noqa: F401  (sets the argument types)
    f = sm._lib.stable_merge_learned

    def call(keys=0x10000, pay=None, n=100, m=100, out=0x20000, opay=None, dtype=1, block=16,
             ws=0x30000, ws_bytes=1 << 20):
        return f(keys, pay, n, m, out, opay, dtype, 0x40000, 0x50000, 1, 1, block, 256, 0x60000,
                 0x70000, ws, ws_bytes, None)

    assert call(dtype=9) == -2
    assert call(n=-1) == -1
    assert call(block=0) == -1
    assert call(block=(1 << 20) + 1) == -1
    assert call(out=0x10000 + 64) == -3                            # out overlaps keys
    assert call(ws_bytes=16) == -4
    assert call(n=0, m=0) == 0                                      # nothing to do
    q = sm._lib.stable_merge_learned_workspace_bytes
    assert q(100, 100, 0, 1, 0) == 0
    assert q(100, 100, 16, 1, 0) > 0 and q(100, 100, 16, 1, 1) >= q(100, 100, 16, 1, 0)


def test_segmented_sort_error_paths(sm):
    f = sm._lib.stable_merge_segmented_sort
    o = sm.Options()

    def call(keys=0x10000, pay=None, offs=0x50000, count=4, N=100, max_len=50, out=0x20000,
             opay=None, dtype=1, ws=0x30000, ws_bytes=1 << 24):
        return f(keys, pay, offs, count, N, max_len, out, opay, dtype, ws, ws_bytes,
                 ctypes.byref(o), None)

    assert call(dtype=6) == -2
    assert call(count=0) == -1
    assert call(max_len=101) == -1
    assert call(max_len=-1) == -1
    assert call(offs=None) == -1
    assert call(pay=0x40000) == -1                                  # payload without out_payloads
    assert call(out=0x10000 + 64) == -3                             # partial overlap
    assert call(ws_bytes=8) == -4
    assert call(N=0, max_len=0) == 0                                # nothing to do
    q = sm._lib.stable_merge_segmented_sort_workspace_bytes
    assert q(0, 100, 50, 1, 0, ctypes.byref(o)) == 0
    assert q(4, 100, 50, 1, 0, ctypes.byref(o)) > 0


def test_descending_workspace_and_errors(sm):
    """Descending order needs no more workspace than ascending; bad
    arguments are rejected host-side as in ascending order."""
    import torch
    for dt in (torch.uint32, torch.float64):
        assert sm.workspace_bytes(1000, 3000, dt, descending=True) == sm.workspace_bytes(1000, 3000, dt)
        assert sm.batched_workspace_bytes(10, 5000, dt, descending=True) == \
            sm.batched_workspace_bytes(10, 5000, dt)
        o = sm._opts(descending=True)
        assert sm._lib.stable_merge_sort_workspace_bytes(5000, sm.DTYPES[dt], 1, ctypes.byref(o)) \
            == sm.sort_workspace_bytes(5000, dt, True)
    o = sm._opts(descending=True)
    assert call_merge(sm, ws_bytes=8, opts=o) == -4
    assert call_merge(sm, dtype=7, opts=o) == -2
    assert call_merge(sm, dtype=8, opts=o) == -2      # kernel-only codes are not public
    assert call_merge(sm, dtype=9) == -2
    assert call_merge(sm, n=0, m=0, opts=o) == 0


def test_sort_learned_error_paths(sm):
    f = sm._lib.stable_merge_sort_learned
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_float,
                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                  ctypes.c_void_p]

    def call(model=0x50000, step=0.01, dtype=1, N=100, opts=None, ws_bytes=1 << 24):
        o = opts if opts is not None else sm.Options()
        return f(0x10000, None, N, 0x20000, None, dtype, model, step, None, 0x30000, ws_bytes,
                 ctypes.byref(o), None)

    assert call(model=None) == -1
    assert call(dtype=7) == -2
    assert call(step=-1.0) == -1
    assert call(step=float("nan")) == -1
    assert call(opts=sm._opts(descending=True)) == -1
    assert call(ws_bytes=8) == -4
    assert call(N=0) == 0


def test_reserved_options_rejected(sm):
    import torch
    o = sm.Options()
    o.reserved[2] = 1
    assert call_merge(sm, opts=o) == -1
    assert sm._lib.stable_merge_workspace_bytes(10, 10, 1, 0, ctypes.byref(o)) == 0
    assert sm._lib.stable_merge_batched_workspace_bytes(2, 10, 1, 0, ctypes.byref(o)) == 0
    assert sm._lib.stable_merge_sort_workspace_bytes(100, 1, 0, ctypes.byref(o)) == 0
    assert sm._lib.stable_merge_segmented_sort_workspace_bytes(2, 100, 60, 1, 0,
                                                                ctypes.byref(o)) == 0
    assert sm._lib.stable_merge_sort(0x10000, None, 100, 0x20000, None, 1, 0x30000, 1 << 20,
                                     ctypes.byref(o), None) == -1
    assert sm.workspace_bytes(10, 10, torch.uint32) > 0


def test_workspace_alias_rejected(sm):
    """A workspace that shares bytes with keys, payloads, outputs, the pair
    descriptors or the cross ranks is rejected before any launch."""
    # stable_merge: 20 uint32 keys at 0x10000, outputs at 0x20000
    assert call_merge(sm, ws=0x10000) == -3                       # on the keys
    assert call_merge(sm, ws=0x20000 - 256) == -3                 # runs into the outputs
    assert call_merge(sm, pay=0x40000, opay=0x50000, ws=0x40000) == -3
    assert call_merge(sm, pay=0x40000, opay=0x50000, ws=0x50000) == -3
    assert call_merge(sm, ws=0x30000) != -3                       # separate: not an alias error
    f = sm._lib.stable_merge_batched
    o = sm.Options()

    def batched(ws, offs=0x50000, na=0x60000):
        return f(0x10000, None, offs, na, 4, 100, 0x20000, None, 1, ws, 1 << 20,
                 ctypes.byref(o), None)
    assert batched(0x10000) == -3
    assert batched(0x30000, offs=0x30000 + 64) == -3              # offsets inside the workspace
    assert batched(0x30000, na=0x30000 + 64) == -3
    p = sm._lib.stable_merge_pieces
    # xbar / ybar inside the workspace
    assert p(0x10000, None, 10, 10, 2, 2, 0x30000, 0x31000, 0x20000, None, 1, 0x30000,
             1 << 20, None) == -3
    assert b"workspace overlaps" in sm._lib.sm_last_error()


def _fnv1a(b: bytes) -> int:
    """FNV-1a, 32 bits (offset basis 2166136261, prime 16777619)."""
    h = 2166136261
    for x in b:
        h = ((h ^ x) * 16777619) & 0xFFFFFFFF
    return h


def _blob(magic=0x4D524D53, version=1, dtype=1, is_high=0, feature=1, hidden=32, nparam=97,
          loss=0.25, length=1000, params=None, checksum=None) -> bytes:
    import struct
    params = params if params is not None else [0.5] * 97
    head = struct.pack("<IIiiiiifq", magic, version, dtype, is_high, feature, hidden, nparam,
                       loss, length) + struct.pack("<97f", *params)
    assert len(head) == 428
    return head + struct.pack("<I", _fnv1a(head) if checksum is None else checksum)


def test_predictor_blob_checks(sm):
    """Loading rejects every malformed blob host-side, before touching the
    GPU; the handle calls reject NULL handles."""
    from paper_1202_6575_amd import learned  # noqa: F401  (sets the argument types)
    lib = sm._lib
    h = ctypes.c_void_p()

    def load(b, size=None):
        buf = ctypes.create_string_buffer(b, len(b))
        return lib.sm_predictor_load(ctypes.byref(h), buf, len(b) if size is None else size)

    assert lib.sm_predictor_load(None, None, 0) == -1
    assert load(_blob(), size=431) == -1                  # short
    assert load(_blob(magic=0x12345678)) == -1
    assert load(_blob(version=2)) == -1
    assert load(_blob(checksum=1)) == -1                  # corrupted
    assert b"checksum" in lib.sm_last_error()
    bad = bytearray(_blob())
    bad[100] ^= 1                                          # a flipped parameter bit
    assert load(bytes(bad)) == -1
    assert load(_blob(dtype=6)) == -2
    assert load(_blob(hidden=16)) == -1
    assert load(_blob(nparam=49)) == -1
    assert load(_blob(feature=2)) == -1
    assert load(_blob(is_high=2)) == -1
    assert load(_blob(length=-1)) == -1
    assert h.value is None                                 # nothing was created
    assert lib.sm_predictor_create(ctypes.byref(h), 9, 0) == -2
    assert lib.sm_predictor_destroy(None) == 0
    assert lib.sm_predictor_params(None) is None
    assert lib.sm_predictor_save(None, ctypes.create_string_buffer(432), 432) == -1
    assert lib.sm_predictor_info(None, None, None, None, None) == -1


def test_noalloc_error_paths(sm):
    """stable_merge_noalloc rejects bad arguments, validate, and plans above
    its scratch limit before it looks up the scratch array (no GPU call)."""
    def call(keys=0x10000, pay=None, n=10, m=10, out=0x20000, opay=None, dtype=1, opts=None):
        o = opts if opts is not None else sm.Options()
        return sm._lib.stable_merge_noalloc(keys, pay, n, m, out, opay, dtype, ctypes.byref(o),
                                            None)
    assert call(dtype=9) == -2
    assert call(n=-1) == -1
    assert call(pay=0x40000) == -1
    assert call(out=0x10000 + 16) == -3
    assert call(n=0, m=0) == 0
    o = sm.Options()
    o.validate = 1
    assert call(opts=o) == -1
    o = sm.Options()
    o.reserved[0] = 1
    assert call(opts=o) == -1
    # 2^21 + 2^21 blocks need 32 MiB of cross ranks alone
    n = m = 1 << 21
    o = sm.Options()
    o.p_a, o.p_b = n, m
    assert call(n=n, m=m, out=0x10000 + 64 * n, opts=o) == -4
    assert b"scratch" in sm._lib.sm_last_error()
    hdr = open(os.path.join(HEADER_DIR, "stablemerge.h")).read()
    mt = re.search(r"#define SM_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", hdr)
    assert mt and sm.NOALLOC_SCRATCH_BYTES == int(mt.group(1)) << int(mt.group(2))


def test_sort_runs_error_paths(sm):
    """stable_merge_sort_runs checks its arguments before any launch."""
    def call(keys=0x10000, pay=None, N=1000, out=0x20000, opay=None, dtype=1, run=512):
        return sm._lib.stable_merge_sort_runs(keys, pay, N, out, opay, dtype, run, None)
    assert call(dtype=6) == -2
    assert call(N=-1) == -1
    assert call(run=300) == -1
    assert call(run=4096, dtype=2) == -1          # 4096 only for 32-bit keys
    assert call(pay=0x40000) == -1
    assert call(keys=0x10008) == -1
    assert call(out=0x10000 + 16) == -3           # partial overlap
    assert call(N=0) == 0
