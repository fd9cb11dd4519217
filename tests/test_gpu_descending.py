"""Descending order: merges and sorts from largest to smallest key.

The expected result comes from the CPU oracle run on the reversed order
(``descending=True``): its merge and sort are pinned on the CPU against
Python's stable sorted(..., reverse=True), so ties put A first and keep each
source's order.  Payloads are the element indices, so the payload output is
the permutation itself."""
import numpy as np
import pytest
import torch

import oracle
from helpers import total_order_sequence, dev, flush, host, rand_sorted

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402

DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def oracle_merge_desc(keys: np.ndarray, n: int):
    """(keys, index permutation) of the oracle's descending merge of
    keys[:n] and keys[n:], payload = index."""
    idx = np.arange(len(keys), dtype=np.uint32)
    c, pc = oracle.merge(keys[:n], keys[n:], idx[:n], idx[n:], descending=True)
    return c, pc


def oracle_sort_desc(keys: np.ndarray):
    """(keys, index permutation) of the oracle's descending stable sort."""
    c, pc = oracle.sort(keys, np.arange(len(keys), dtype=np.uint32), descending=True)
    return c, pc


def same_bits(a: np.ndarray, b: np.ndarray) -> bool:
    return a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def desc_sorted(g, n, alphabet, dt):
    return rand_sorted(g, n, alphabet, dt)[::-1].copy()


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_merge_descending(dtype, with_pay):
    g = np.random.default_rng(51)
    for n, m in [(0, 0), (0, 7), (9, 0), (1, 1), (1000, 3), (4099, 4097), (60_001, 39_999)]:
        for alpha in (4, 1 << 30):
            A, B = desc_sorted(g, n, alpha, dtype), desc_sorted(g, m, alpha, dtype)
            keys = np.concatenate([A, B])
            pay = np.arange(n + m, dtype=np.uint32) if with_pay else None
            flush(f"merge descending {np.dtype(dtype).name} n={n} m={m} alpha={alpha}")
            ck, cp = sm.merge(dev(keys), n, m, None if pay is None else dev(pay),
                              descending=True, validate=True)
            torch.cuda.synchronize()
            rk, rp = oracle_merge_desc(keys, n)
            assert same_bits(host(ck), rk)
            if with_pay:
                assert np.array_equal(host(cp), rp)


def test_merge_descending_inputs_untouched_and_tiles():
    """The caller's keys stay as they were; small tiles and an explicit p
    give the same bytes; ascending input is rejected by validate."""
    g = np.random.default_rng(52)
    A, B = desc_sorted(g, 30_000, 100, np.int32), desc_sorted(g, 20_011, 100, np.int32)
    keys = np.concatenate([A, B])
    dk = dev(keys)
    rk, rp = oracle_merge_desc(keys, len(A))
    for kw in ({}, {"tile": 64}, {"p_a": 7, "p_b": 3}):
        flush(f"merge descending options {kw}")
        ck, cp = sm.merge(dk, len(A), len(B), dev(np.arange(len(keys), dtype=np.uint32)),
                          descending=True, **kw)
        torch.cuda.synchronize()
        assert np.array_equal(host(ck), rk)
        assert np.array_equal(host(cp), rp)
        assert np.array_equal(host(dk), keys)
    asc = np.concatenate([A[::-1], B[::-1]])
    with pytest.raises(sm.SMError):
        sm.merge(dev(asc), len(A), len(B), descending=True, validate=True)


@pytest.mark.parametrize("dtype", [np.int32, np.uint64, np.float32])
def test_merge_descending_small_blocks(dtype):
    """Blocks of a few elements: ascending merges take the small-block
    kernel there, descending ones the general merge kernel."""
    g = np.random.default_rng(58)
    for n, m, p in [(10_000, 10_000, 2000), (3001, 7, 1000), (64, 640, 64)]:
        A, B = desc_sorted(g, n, 30, dtype), desc_sorted(g, m, 30, dtype)
        keys = np.concatenate([A, B])
        flush(f"merge descending small blocks {np.dtype(dtype).name} n={n} m={m} p={p}")
        ck, cp = sm.merge(dev(keys), n, m, dev(np.arange(n + m, dtype=np.uint32)),
                          p_a=p, p_b=p, descending=True)
        torch.cuda.synchronize()
        rk, rp = oracle_merge_desc(keys, n)
        assert same_bits(host(ck), rk)
        assert np.array_equal(host(cp), rp)


@pytest.mark.parametrize("dtype", DTYPES)
def test_batched_descending(dtype):
    g = np.random.default_rng(53)
    sizes = [(0, 0), (5, 0), (0, 3), (700, 1300), (4096, 4097), (1, 1), (20_000, 9)]
    parts, n_a, offs = [], [], [0]
    for n, m in sizes:
        parts += [desc_sorted(g, n, 50, dtype), desc_sorted(g, m, 50, dtype)]
        n_a.append(n)
        offs.append(offs[-1] + n + m)
    keys = np.concatenate(parts)
    pay = np.arange(len(keys), dtype=np.uint32)
    flush(f"batched descending {np.dtype(dtype).name}")
    ck, cp = sm.merge_batched(dev(keys), dev(np.array(offs, np.int64)),
                              dev(np.array(n_a, np.int64)), dev(pay), descending=True)
    torch.cuda.synchronize()
    ck, cp = host(ck), host(cp)
    for k in range(len(sizes)):
        lo, hi = offs[k], offs[k + 1]
        rk, rp = oracle_merge_desc(keys[lo:hi], n_a[k])
        assert same_bits(ck[lo:hi], rk)
        assert np.array_equal(cp[lo:hi], rp + np.uint32(lo))


def rand_keys(g, N, alphabet, dtype):
    return g.permutation(rand_sorted(g, N, alphabet, dtype))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_sort_descending(dtype, with_pay):
    g = np.random.default_rng(54)
    for N in [0, 1, 2, 513, 4096, 50_001]:
        for alpha in (3, 1 << 30):
            keys = rand_keys(g, N, alpha, dtype)
            pay = np.arange(N, dtype=np.uint32) if with_pay else None
            flush(f"sort descending {np.dtype(dtype).name} pay={with_pay} N={N} alpha={alpha}")
            ck, cp = sm.sort(dev(keys), None if pay is None else dev(pay), descending=True)
            torch.cuda.synchronize()
            rk, rp = oracle_sort_desc(keys)
            assert same_bits(host(ck), rk)
            if with_pay:
                assert np.array_equal(host(cp), rp)


def test_sort_descending_in_place_and_runs():
    g = np.random.default_rng(55)
    keys = rand_keys(g, 100_003, 200, np.uint64)
    rk, rp = oracle_sort_desc(keys)
    for run in (256, 2048):
        flush(f"sort descending in place run={run}")
        dk, dp = dev(keys), dev(np.arange(len(keys), dtype=np.uint32))
        sm.sort(dk, dp, out_keys=dk, out_payloads=dp, run=run, descending=True)
        torch.cuda.synchronize()
        assert np.array_equal(host(dk), rk)
        assert np.array_equal(host(dp), rp)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_float_specials_descending(dt):
    """NaNs of both signs, infinities, -0 and +0 and subnormals: the
    descending sort and merge are the reverse totalOrder, bit for bit."""
    seq = total_order_sequence(dt)
    g = np.random.default_rng(56)
    keys = seq[g.integers(0, len(seq), size=30_000)]
    flush(f"float specials descending {np.dtype(dt).name}")
    ck, cp = sm.sort(dev(keys), dev(np.arange(len(keys), dtype=np.uint32)), descending=True)
    torch.cuda.synchronize()
    rk, rp = oracle_sort_desc(keys)
    assert same_bits(host(ck), rk)
    assert np.array_equal(host(cp), rp)
    A, B = oracle_sort_desc(keys[:12_000])[0], oracle_sort_desc(keys[12_000:])[0]
    both = np.concatenate([A, B])
    mk, _ = sm.merge(dev(both), len(A), len(B), descending=True, validate=True)
    torch.cuda.synchronize()
    assert same_bits(host(mk), oracle_merge_desc(both, len(A))[0])


def test_segmented_descending():
    g = np.random.default_rng(57)
    lengths = np.concatenate([[0, 1, 512, 513, 5000], g.integers(0, 900, size=60), [0]])
    offs = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    for dt in (np.int32, np.float64):
        keys = rand_keys(g, int(offs[-1]), 40, dt)
        pay = np.arange(len(keys), dtype=np.uint32)
        flush(f"segmented descending {np.dtype(dt).name}")
        ck, cp = sm.segmented_sort(dev(keys), dev(offs), int(lengths.max()), dev(pay),
                                   descending=True, validate=True)
        torch.cuda.synchronize()
        ck, cp = host(ck), host(cp)
        for s in range(len(lengths)):
            lo, hi = int(offs[s]), int(offs[s + 1])
            rk, rp = oracle_sort_desc(keys[lo:hi])
            assert same_bits(ck[lo:hi], rk)
            assert np.array_equal(cp[lo:hi], rp + np.uint32(lo))
