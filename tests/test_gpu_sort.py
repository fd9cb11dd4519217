"""GPU parity of the stable merge sort against the CPU oracle (bit-exact),
and at full size against the definition of a stable sort."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from helpers import total_order_sequence, dev, flush, host

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402

DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def rand_keys(g, N, alphabet, dtype):
    """Unsorted keys over an alphabet spread so that signed / unsigned order
    matters (negative int32, values above 2^31 / 2^63)."""
    if dtype == np.int32:
        return g.integers(-alphabet // 2, alphabet - alphabet // 2, size=N).astype(np.int32)
    if dtype == np.uint32:
        return (g.integers(0, alphabet, size=N) * ((2 ** 32 - 1) // alphabet)).astype(np.uint32)
    if dtype == np.int64:
        return g.integers(-alphabet // 2, alphabet - alphabet // 2, size=N) * ((2 ** 63 - 1) // alphabet)
    if dtype in (np.float32, np.float64):
        return (g.integers(-alphabet // 2, alphabet - alphabet // 2, size=N) * 0.375).astype(dtype)
    return g.integers(0, alphabet, size=N).astype(np.uint64) * np.uint64((2 ** 64 - 1) // alphabet)


def check_sort(keys, with_pay=True, run=0, in_place=False, **kw):
    N = len(keys)
    pay = np.arange(N, dtype=np.uint32)[::-1].copy() if with_pay else None
    rk, rp = oracle.sort(keys, pay, run or 512)
    dk = dev(keys)
    dp = None if pay is None else dev(pay)
    if in_place:
        ck, cp = sm.sort(dk, dp, out_keys=dk, out_payloads=dp, run=run, **kw)
    else:
        ck, cp = sm.sort(dk, dp, run=run, **kw)
    torch.cuda.synchronize()
    # compare bits: float keys may be NaN
    assert np.array_equal(host(ck).view(np.uint8), rk.view(np.uint8)), "keys differ"
    if with_pay:
        assert np.array_equal(host(cp), rp), "payloads differ"


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_sort_sizes(dtype, with_pay):
    """Ragged sizes around the run length and across several passes."""
    g = np.random.default_rng(21)
    for N in [0, 1, 2, 511, 512, 513, 1024, 1500, 4096, 20_001, 131_073]:
        for alpha in (3, 1 << 30):
            flush(f"sort dtype={np.dtype(dtype).name} pay={with_pay} N={N} alpha={alpha}")
            check_sort(rand_keys(g, N, alpha, dtype), with_pay)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("run", [256, 512, 2048])
def test_sort_runs_alone(dtype, run):
    """The sort's first phase alone: every run sorted on its own, equal to
    the oracle's stable sort of that run; a ragged last run; in place too."""
    if run == 4096 and np.dtype(dtype).itemsize == 8:
        pytest.skip("4096-element runs are for 32-bit keys")
    g = np.random.default_rng(run)
    N = 7 * run + run // 3
    keys = rand_keys(g, N, 5, dtype)
    pay = np.arange(N, dtype=np.uint32)
    flush(f"sort runs dtype={np.dtype(dtype).name} run={run} N={N}")
    ck, cp = sm.sort_runs(dev(keys), run, dev(pay))
    dk, dp = dev(keys), dev(pay)
    sm.sort_runs(dk, run, dp, out_keys=dk, out_payloads=dp)
    torch.cuda.synchronize()
    ck, cp, ik, ip = host(ck), host(cp), host(dk), host(dp)
    for r0 in range(0, N, run):
        rk, rp = oracle.sort(keys[r0:r0 + run], pay[r0:r0 + run], run)
        assert np.array_equal(ck[r0:r0 + run].view(np.uint8), rk.view(np.uint8)), f"run {r0}"
        assert np.array_equal(cp[r0:r0 + run], rp), f"run {r0} payloads"
    assert np.array_equal(ik.view(np.uint8), ck.view(np.uint8)) and np.array_equal(ip, cp)


@pytest.mark.parametrize("run", [256, 512, 1024, 2048, 4096])
def test_sort_run_lengths(run):
    """Every run length and a tiny merge tile give the same bytes."""
    g = np.random.default_rng(run)
    keys = rand_keys(g, 300_007, 100, np.uint32)
    flush(f"sort run={run}")
    check_sort(keys, True, run=run)
    check_sort(keys, True, run=run, tile=64)


def test_sort_special_inputs():
    ar = np.arange(100_000)
    for keys in [ar.astype(np.int32), ar[::-1].astype(np.int32), np.full(70_000, 5, np.int32),
                 (ar % 7).astype(np.int32), np.array([np.iinfo(np.int32).max] * 600 +
                                                      [np.iinfo(np.int32).min] * 600, np.int32)]:
        flush(f"sort special N={len(keys)}")
        check_sort(keys, True)


def test_sort_in_place():
    g = np.random.default_rng(4)
    for N in [700, 5000, 100_000]:      # odd and even numbers of passes
        flush(f"sort in place N={N}")
        check_sort(rand_keys(g, N, 50, np.uint64), True, in_place=True)
        check_sort(rand_keys(g, N, 50, np.int32), False, in_place=True)


def test_sort_alias_rejected():
    k = dev(np.arange(1000, dtype=np.uint32))
    with pytest.raises(sm.SMError) as e:
        sm.sort(k[:996], out_keys=k[4:])
    assert e.value.code in (-1, -3)
    with pytest.raises(sm.SMError) as e:
        sm.sort(k, run=300)
    assert e.value.code == -1


@pytest.mark.slow
def test_sort_u32_2e28_full():
    """N = 2^28 uint32 keys uniform in [0, 2^24), payload = index, runs of
    512 and 19 merge passes.  With distinct payloads in input order the
    stable sort is the unique order by (key, payload): the output must be a
    permutation of the input pairs that is strictly increasing in that order."""
    N = 1 << 28
    flush("sort 2^28 generate")
    keys, pay = datagen.sort_input(N, 1 << 24, seed=datagen.BASE_SEED + 5)
    dk, dp = dev(keys), dev(pay)
    flush("sort 2^28 gpu sort")
    ck, cp = sm.sort(dk, dp)
    torch.cuda.synchronize()
    comp = ck.to(torch.int64) << 32 | cp.to(torch.int64)
    assert bool((comp[1:] > comp[:-1]).all())
    # the payloads are a permutation of 0..N-1 and carry their own keys
    assert bool((torch.sort(cp.to(torch.int64)).values ==
                 torch.arange(N, device=cp.device)).all())
    assert torch.equal(dk.to(torch.int64)[cp.to(torch.int64)], ck.to(torch.int64))
    # sampled windows against the oracle's merge sort of the same input
    flush("sort 2^28 oracle check on a prefix")
    M = 1 << 20
    rk, rp = oracle.sort(keys[:M], pay[:M], 512)
    sub, _ = sm.sort(dev(keys[:M]), dev(pay[:M]))
    torch.cuda.synchronize()
    assert np.array_equal(host(sub), rk)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_sort_float_total_order(dt):
    """NaNs of both signs and several payloads, infinities, -0 and +0,
    subnormals and ordinary values, repeated and shuffled: the GPU sort
    equals the oracle's sort bit for bit, payloads included."""
    seq = total_order_sequence(dt)
    g = np.random.default_rng(31)
    keys = seq[g.integers(0, len(seq), size=50_000)]
    flush(f"sort float specials {np.dtype(dt).name}")
    for run in (0, 2048):
        check_sort(keys, True, run=run)
        check_sort(keys, False, run=run)


def oracle_segmented(keys, pay, offsets, run=512):
    outk, outp = np.empty_like(keys), (None if pay is None else np.empty_like(pay))
    for s in range(len(offsets) - 1):
        lo, hi = int(offsets[s]), int(offsets[s + 1])
        if hi > lo:
            k, p = oracle.sort(keys[lo:hi], None if pay is None else pay[lo:hi], run)
            outk[lo:hi] = k
            if pay is not None:
                outp[lo:hi] = p
    return outk, outp


def check_segmented(keys, lengths, with_pay=True, run=0, max_len=None, **kw):
    offsets = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    N = int(offsets[-1])
    assert N == len(keys)
    pay = np.arange(N, dtype=np.uint32)[::-1].copy() if with_pay else None
    rk, rp = oracle_segmented(keys, pay, offsets)
    ml = max_len if max_len is not None else int(max(lengths) if len(lengths) else 0)
    ck, cp = sm.segmented_sort(dev(keys), dev(offsets), ml, None if pay is None else dev(pay),
                               run=run, **kw)
    torch.cuda.synchronize()
    assert np.array_equal(host(ck).view(np.uint8), rk.view(np.uint8)), "keys differ"
    if with_pay:
        assert np.array_equal(host(cp), rp), "payloads differ"


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_segmented_sort_mixed(dtype, with_pay):
    """Segments of every size class at once: empty, one element, below,
    at and above the run length, and long ones needing several passes."""
    g = np.random.default_rng(41)
    lengths = np.concatenate([[0, 1, 511, 512, 513, 0, 3000, 70_001, 2, 1024, 4097],
                              g.integers(0, 2000, size=300), [0]])
    keys = rand_keys(g, int(lengths.sum()), 97, dtype)
    flush(f"segmented mixed dtype={np.dtype(dtype).name} pay={with_pay} count={len(lengths)}")
    check_segmented(keys, lengths, with_pay)


@pytest.mark.parametrize("run", [256, 2048])
def test_segmented_sort_shapes(run):
    """One segment (the plain sort); many tiny segments; a loose max_len
    bound (extra passes that only copy); validation in the call; in place."""
    g = np.random.default_rng(42)
    N = 200_003
    keys = rand_keys(g, N, 1000, np.uint32)
    flush(f"segmented shapes run={run}")
    check_segmented(keys, [N], True, run=run)
    tiny = g.integers(0, 9, size=40_000)
    check_segmented(rand_keys(g, int(tiny.sum()), 5, np.int32), tiny, True, run=run)
    lens = g.integers(0, 5000, size=100)
    k2 = rand_keys(g, int(lens.sum()), 50, np.uint64)
    check_segmented(k2, lens, True, run=run, max_len=int(lens.sum()), validate=True)
    offsets = dev(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64))
    dk = dev(k2)
    sm.segmented_sort(dk, offsets, int(lens.max()), out_keys=dk, run=run)
    torch.cuda.synchronize()
    rk, _ = oracle_segmented(k2, None, host(offsets))
    assert np.array_equal(host(dk), rk)


def test_segmented_sort_validation():
    keys = dev(np.arange(100, dtype=np.uint32)[::-1].copy())
    bad = [np.array([0, 60, 40, 100]), np.array([0, 50, 99]), np.array([5, 50, 100])]
    for offs in bad:
        with pytest.raises(sm.SMError) as e:
            sm.segmented_sort(keys, dev(offs.astype(np.int64)), 100, validate=True)
        assert e.value.code == -1
    with pytest.raises(sm.SMError):   # a segment longer than max_len
        sm.segmented_sort(keys, dev(np.array([0, 70, 100], dtype=np.int64)), 50, validate=True)
