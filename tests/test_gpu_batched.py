"""GPU parity of the batched stable merge (many independent pairs in one
launch sequence) against the CPU oracle, pair by pair, bit-exact."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from helpers import dev, flush, host, rand_sorted

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402

DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def make_batch(g, lengths, alpha, dtype, gap=0):
    """Pairs A_k || B_k laid out contiguously (after `gap` unused leading
    elements); lengths is a list of (n_k, m_k)."""
    parts, offsets, n_a = [np.zeros(gap, dtype=dtype)], [gap], []
    for n, m in lengths:
        parts += [rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)]
        offsets.append(offsets[-1] + n + m)
        n_a.append(n)
    return np.concatenate(parts), np.array(offsets, np.int64), np.array(n_a, np.int64)


def check_batched(keys, offsets, n_a, with_pay=True, **kw):
    pay = np.arange(len(keys), dtype=np.uint32) if with_pay else None
    ck, cp = sm.merge_batched(dev(keys), dev(offsets), dev(n_a),
                              None if pay is None else dev(pay), **kw)
    torch.cuda.synchronize()
    ck = host(ck)
    cp = None if cp is None else host(cp)
    rk, rp = oracle.merge_batched(keys, offsets, n_a, pay)
    for k in range(len(n_a)):
        lo, hi = offsets[k], offsets[k + 1]
        assert np.array_equal(ck[lo:hi], rk[lo:hi]), f"pair {k} keys differ"
        if with_pay:
            assert np.array_equal(cp[lo:hi], rp[lo:hi]), f"pair {k} payloads differ"


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_batched_mixed_sizes(dtype, with_pay):
    """Log-uniform pair lengths from 1 to 2^14: whole-workgroup pairs and
    pairs split by the method, m_k > n_k included."""
    n_k, m_k = datagen.batch_lengths(300, 0, 14, seed=11)
    g = np.random.default_rng(5)
    keys, offsets, n_a = make_batch(g, list(zip(n_k, m_k)), 1 << 10, dtype)
    flush(f"batched mixed dtype={np.dtype(dtype).name} pay={with_pay} total={len(keys)}")
    check_batched(keys, offsets, n_a, with_pay)


@pytest.mark.parametrize("tile", [1, 7, 64, 1000, 1536, 3072, 4096])
def test_batched_tiles(tile):
    """Tiny tiles split nearly every pair into many subproblems."""
    n_k, m_k = datagen.batch_lengths(120, 0, 12, seed=tile)
    g = np.random.default_rng(tile)
    keys, offsets, n_a = make_batch(g, list(zip(n_k, m_k)), 50, np.int32)
    flush(f"batched tile={tile} total={len(keys)}")
    check_batched(keys, offsets, n_a, True, tile=tile)


def test_batched_edges():
    """Empty pairs, one-sided pairs, single elements, all-equal keys, a pair
    bigger than many tiles, and unused elements before the first pair."""
    g = np.random.default_rng(9)
    lengths = [(0, 0), (5, 0), (0, 5), (1, 1), (0, 0), (4097, 4095), (10000, 1), (1, 10000),
               (3, 0), (0, 70000), (123, 456)]
    keys, offsets, n_a = make_batch(g, lengths, 3, np.uint32, gap=8)
    flush("batched edges")
    check_batched(keys, offsets, n_a, True)
    check_batched(keys, offsets, n_a, False, tile=16)
    # a single pair equals the plain merge
    A, B = rand_sorted(g, 30000, 7, np.uint64), rand_sorted(g, 20000, 7, np.uint64)
    keys = np.concatenate([A, B])
    check_batched(keys, np.array([0, 50000], np.int64), np.array([30000], np.int64), True)


def test_batched_validate():
    keys = np.array([1, 2, 3, 0, 4, 9, 9, 1], dtype=np.uint32)
    offsets = dev(np.array([0, 4, 8], np.int64))
    # pair 0: A = [1,2,3], B = [0]; pair 1: A = [4,9,9], B = [1] -- both valid
    check_batched(keys, np.array([0, 4, 8], np.int64), np.array([3, 3], np.int64), True,
                  validate=True)
    with pytest.raises(sm.SMError) as e:                        # pair 1: A = [4,9,9,1] unsorted
        sm.merge_batched(dev(keys), offsets, dev(np.array([3, 4], np.int64)), validate=True)
    assert e.value.code == -6
    with pytest.raises(sm.SMError) as e:                        # n_a beyond the pair
        sm.merge_batched(dev(keys), offsets, dev(np.array([5, 1], np.int64)), validate=True)
    assert e.value.code == -1
    with pytest.raises(sm.SMError) as e:                        # offsets past total
        sm.merge_batched(dev(keys), dev(np.array([0, 4, 9], np.int64)),
                         dev(np.array([3, 1], np.int64)), validate=True)
    assert e.value.code == -1


def test_batched_invalid_pair_skipped():
    """Without validate an invalid pair is skipped: the others are merged."""
    g = np.random.default_rng(2)
    keys, offsets, n_a = make_batch(g, [(100, 50), (30, 30), (7, 9)], 20, np.int32)
    bad = n_a.copy()
    bad[1] = 1000
    out = torch.full((len(keys),), -1, dtype=torch.int32, device="cuda:0")
    sm.merge_batched(dev(keys), dev(offsets), dev(bad), out_keys=out)
    torch.cuda.synchronize()
    got = host(out)
    rk, _ = oracle.merge_batched(keys, offsets, n_a)
    assert np.array_equal(got[offsets[0]:offsets[1]], rk[offsets[0]:offsets[1]])
    assert np.array_equal(got[offsets[2]:offsets[3]], rk[offsets[2]:offsets[3]])
    assert (got[offsets[1]:offsets[2]] == -1).all()


@pytest.mark.slow
def test_batched_65536_pairs_to_2e15_sampled():
    """65,536 pairs with log-uniform totals in [16, 2^15] (about 2^28 int32
    keys in [0, 2^20)), default launch configuration: 1024 sampled pairs
    against the oracle, and every pair's output a sorted permutation of its
    input (checked on the GPU with torch)."""
    count = 65536
    n_k, m_k = datagen.batch_lengths(count, 4, 15, seed=datagen.BASE_SEED + 4)
    flush("65,536 pairs up to 2^15 generate")
    keys, offsets, n_a = datagen.batched_pairs(n_k, m_k, 0, 1 << 20, np.int32,
                                               seed=datagen.BASE_SEED + 4)
    flush(f"65,536 pairs up to 2^15 gpu total={len(keys)}")
    dk = dev(keys)
    ck, _ = sm.merge_batched(dk, dev(offsets), dev(n_a))
    torch.cuda.synchronize()
    got = host(ck)
    g = np.random.default_rng(1)
    for k in g.choice(count, 1024, replace=False):
        lo, hi, na = offsets[k], offsets[k + 1], n_a[k]
        rk, _ = oracle.merge(keys[lo:lo + na], keys[lo + na:hi])
        assert np.array_equal(got[lo:hi], rk), f"pair {k}"
    # properties at full size: per-pair non-decreasing and same multiset
    pair_id = np.repeat(np.arange(count, dtype=np.int64), np.diff(offsets))
    comp_in = torch.from_numpy(pair_id << 21 | keys.astype(np.int64)).to("cuda:0")
    comp_out = torch.from_numpy(pair_id << 21 | got.astype(np.int64)).to("cuda:0")
    assert bool((comp_out[1:] >= comp_out[:-1]).all())
    assert torch.equal(torch.sort(comp_in).values, comp_out)


@pytest.mark.slow
def test_batched_65536_pairs_to_2e20_sampled():
    """The literal batch recipe: 65,536 pairs with totals log-uniform in
    [16, 2^20] (about 6.2e9 int32 keys in [0, 2^20), generated on the GPU),
    merged in the default launch configuration; 256 sampled pairs against
    the oracle."""
    import datagen.torch_gen as tg
    count = 65536
    n_k, m_k = datagen.batch_lengths(count, 4, 20, seed=datagen.BASE_SEED + 4)
    flush("65,536 pairs up to 2^20 generate")
    keys, offsets, n_a = tg.batched_pairs(n_k, m_k, 0, 1 << 20, seed=datagen.BASE_SEED + 4)
    flush(f"65,536 pairs up to 2^20 gpu total={keys.numel()}")
    ck, _ = sm.merge_batched(keys, offsets, n_a)
    torch.cuda.synchronize()
    off, na = host(offsets), host(n_a)
    g = np.random.default_rng(2)
    for k in g.choice(count, 256, replace=False):
        lo, hi = int(off[k]), int(off[k + 1])
        inp = host(keys[lo:hi])
        rk, _ = oracle.merge(inp[:na[k]], inp[na[k]:])
        assert np.array_equal(host(ck[lo:hi]), rk), f"pair {k}"
    # every pair at full size, on the GPU in groups of pairs: each output
    # range non-decreasing and holding the same multiset as its input
    k0 = 0
    while k0 < count:
        k1 = int(np.searchsorted(off, off[k0] + (1 << 28), side="right")) - 1
        k1 = max(k0 + 1, min(k1, count))
        lo, hi = int(off[k0]), int(off[k1])
        flush(f"literal batch properties pairs [{k0}, {k1})")
        pid = torch.repeat_interleave(torch.arange(k0, k1, device=keys.device),
                                      offsets[k0 + 1:k1 + 1] - offsets[k0:k1])
        comp_in = (pid << 21) | keys[lo:hi].to(torch.int64)
        comp_out = (pid << 21) | ck[lo:hi].to(torch.int64)
        assert bool((comp_out[1:] >= comp_out[:-1]).all()), f"pairs [{k0}, {k1}) unsorted"
        assert torch.equal(torch.sort(comp_in).values, comp_out), f"pairs [{k0}, {k1}) multiset"
        del pid, comp_in, comp_out
        k0 = k1
