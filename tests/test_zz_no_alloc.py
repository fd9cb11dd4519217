"""stable_merge_noalloc (the entry point for callers that cannot allocate)
against stable_merge with a workspace, bit for bit, through the C ABI.

Two calls in a row share the device's scratch array; the second merges a
smaller input over what the first left there.  Sizes span several workgroup
blocks with ragged tails, with and without payloads, ascending and
descending, 32- and 64-bit keys.  A plan above the scratch limit must be
rejected before any launch.
"""
import numpy as np
import pytest
import torch

import datagen
from helpers import dev, flush, host, rand_sorted

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402


def both(A, B, pay, **kw):
    keys = dev(np.concatenate([A, B]))
    p = None if pay is None else dev(np.concatenate(pay).astype(np.uint32))
    rk, rp = sm.merge(keys, len(A), len(B), p, **kw)
    ok = torch.empty_like(keys)
    op = None if p is None else torch.empty_like(p)
    sm.merge_noalloc(keys, len(A), len(B), p, ok, op, **kw)
    torch.cuda.synchronize()
    return host(rk), (None if rp is None else host(rp)), host(ok), (None if op is None else host(op))


@pytest.mark.parametrize("dtype,with_pay,desc", [
    (np.uint32, False, False), (np.int32, True, False), (np.uint64, True, False),
    (np.float32, False, True), (np.int64, False, False)])
def test_noalloc_matches_workspace_merge_twice(dtype, with_pay, desc):
    g = np.random.default_rng(20260 + int(with_pay) + 2 * int(desc))
    # second call smaller than the first, both with ragged block tails
    for (n, m, alphabet) in [(700_001, 400_003, 1 << 12), (5_003, 9_001, 37)]:
        flush(f"noalloc {np.dtype(dtype).name} pay={with_pay} desc={desc} n={n} m={m}")
        A = rand_sorted(g, n, alphabet, dtype)
        B = rand_sorted(g, m, alphabet, dtype)
        if desc:
            A, B = A[::-1].copy(), B[::-1].copy()
        pay = datagen.source_tag_payloads(n, m) if with_pay else None
        rk, rp, ok, op = both(A, B, pay, descending=desc)
        assert np.array_equal(ok.view(np.uint8), rk.view(np.uint8)), \
            f"keys differ at {np.flatnonzero(ok != rk)[:10]}"
        if with_pay:
            assert np.array_equal(op, rp), f"payloads differ at {np.flatnonzero(op != rp)[:10]}"


def test_noalloc_forced_blocks_and_edges():
    g = np.random.default_rng(7)
    cases = [(3_000, 0, {}), (0, 2_500, {}), (1, 1, {}), (50_000, 30_000, dict(p_a=256, p_b=256)),
             (40_000, 41_000, dict(tile=512))]
    for n, m, kw in cases:
        flush(f"noalloc edge n={n} m={m} {kw}")
        A = rand_sorted(g, n, 100, np.int32)
        B = rand_sorted(g, m, 100, np.int32)
        pay = datagen.source_tag_payloads(n, m)
        rk, rp, ok, op = both(A, B, pay, **kw)
        assert np.array_equal(ok, rk) and np.array_equal(op, rp)


def test_noalloc_rejects_plans_above_the_scratch_limit():
    n = m = 1 << 20
    keys = torch.zeros(n + m, dtype=torch.int32, device="cuda:0")
    out = torch.empty_like(keys)
    need = sm.workspace_bytes(n, m, torch.int32, p_a=n, p_b=m)
    assert need > sm.NOALLOC_SCRATCH_BYTES
    sentinel = out.fill_(-7).clone()
    with pytest.raises(sm.SMError) as e:
        sm.merge_noalloc(keys, n, m, None, out, p_a=n, p_b=m)
    assert e.value.code == -4
    # validate needs a host read-back, which this entry point does not do
    with pytest.raises(sm.SMError) as e:
        o = sm._opts(validate=True)
        sm._check(sm._lib.stable_merge_noalloc(sm._ptr(keys), None, n, m, sm._ptr(out), None,
                                               sm.SM_INT32, sm.ctypes.byref(o), sm._stream_ptr()))
    assert e.value.code == -1
    torch.cuda.synchronize()
    assert torch.equal(out, sentinel), "a rejected call wrote its output"
