"""GPU parity of the plain stable merge against the CPU oracle (bit-exact).

Every case runs the HIP path through the C ABI (paper_1202_6575_amd) and
compares keys and payloads element by element with the oracle on the same
seeded inputs.
"""
import json
import os

import numpy as np
import pytest
import torch

import datagen
import oracle
from helpers import total_order_sequence, dev, flush, host, rand_sorted

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "figure1.json")
DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def run_merge(A, B, pa=None, pb=None, **kw):
    keys = dev(np.concatenate([A, B]))
    pay = None if pa is None else dev(np.concatenate([pa, pb]).astype(np.uint32))
    ck, cp = sm.merge(keys, len(A), len(B), pay, **kw)
    torch.cuda.synchronize()
    return host(ck), (None if cp is None else host(cp))


def check(A, B, with_pay=True, **kw):
    n, m = len(A), len(B)
    pa = pb = None
    if with_pay:
        pa, pb = datagen.source_tag_payloads(n, m)
    rk, rp = oracle.merge(A, B, pa, pb)
    ck, cp = run_merge(A, B, pa, pb, **kw)
    assert np.array_equal(ck, rk), f"keys differ at {np.flatnonzero(ck != rk)[:10]}"
    if with_pay:
        assert np.array_equal(cp, rp), f"payloads differ at {np.flatnonzero(cp != rp)[:10]}"


def test_figure1_partition_and_merge():
    flush("figure1")
    with open(GOLD) as f:
        g = json.load(f)
    A = np.array(g["A"], dtype=np.int32)
    B = np.array(g["B"], dtype=np.int32)
    xbar, ybar = sm.partition(dev(np.concatenate([A, B])), len(A), len(B), g["p"])
    assert host(xbar).tolist() == g["xbar"]
    assert host(ybar).tolist() == g["ybar"]
    check(A, B, p_a=5, p_b=5)
    check(A, B)


@pytest.mark.parametrize("dtype", DTYPES)
def test_partition_matches_oracle(dtype):
    g = np.random.default_rng(21)
    for trial in range(20):
        n, m = int(g.integers(0, 5000)), int(g.integers(0, 5000))
        p_a, p_b = int(g.integers(1, 300)), int(g.integers(1, 300))
        A, B = rand_sorted(g, n, int(g.integers(1, 500)), dtype), rand_sorted(g, m, 300, dtype)
        flush(f"partition dtype={np.dtype(dtype).name} n={n} m={m} p_a={p_a} p_b={p_b}")
        xb, yb = sm.partition(dev(np.concatenate([A, B])), n, m, p_a, p_b)
        rx, ry = oracle.cross_ranks(A, B, p_a, p_b)
        assert np.array_equal(host(xb), rx) and np.array_equal(host(yb), ry)


@pytest.mark.parametrize("dtype", DTYPES)
def test_partition_both_search_forms(dtype):
    """Block counts on both sides of the switch between group searches (up
    to 2048 block starts, 16 lanes per search) and one lane per search,
    over empty, tiny, all-equal and long arrays."""
    g = np.random.default_rng(83)
    for n, m, alpha in [(0, 5000, 10), (5000, 0, 10), (3, 4, 2), (200_000, 150_000, 1 << 20),
                        (100_000, 90_000, 1), (1_000_003, 7, 1000)]:
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        keys = dev(np.concatenate([A, B]))
        for p_a, p_b in [(1, 1), (1023, 1023), (1024, 1023), (2000, 100), (5, 3000)]:
            flush(f"partition forms dtype={np.dtype(dtype).name} n={n} m={m} p_a={p_a} p_b={p_b}")
            xb, yb = sm.partition(keys, n, m, p_a, p_b)
            rx, ry = oracle.cross_ranks(A, B, p_a, p_b)
            assert np.array_equal(host(xb), rx) and np.array_equal(host(yb), ry)


def test_int32_1m_600k_partition_p256():
    """The config-1 arrays (int32 uniform in [0, 65536), n = 1e6, m = 6e5), p = 256."""
    A, B = datagen.uniform_pair(1_000_000, 600_000, 0, 65536, np.int32, seed=datagen.BASE_SEED)
    flush("int32 1,000,000 + 600,000 partition p=256")
    xb, yb = sm.partition(dev(np.concatenate([A, B])), len(A), len(B), 256)
    rx, ry = oracle.cross_ranks(A, B, 256)
    assert np.array_equal(host(xb), rx) and np.array_equal(host(yb), ry)


def test_int32_1m_600k_merge_p256():
    A, B = datagen.uniform_pair(1_000_000, 600_000, 0, 65536, np.int32, seed=datagen.BASE_SEED)
    flush("int32 1,000,000 + 600,000 merge p=256 and auto")
    check(A, B, p_a=256, p_b=256)
    check(A, B)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_random_small(dtype, with_pay):
    g = np.random.default_rng(1000 + DTYPES.index(dtype) + 10 * with_pay)
    for trial in range(25):
        n, m = int(g.integers(0, 3000)), int(g.integers(0, 3000))
        alpha = int(g.integers(1, 2000))
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        tile = int(g.choice([1, 2, 7, 64, 300, 2048]))
        flush(f"small dtype={np.dtype(dtype).name} pay={with_pay} n={n} m={m} tile={tile}")
        check(A, B, with_pay, tile=tile)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_several_tiles_ragged(dtype, with_pay):
    """Sizes spanning many top-level blocks with ragged ends."""
    g = np.random.default_rng(77)
    for n, m, alpha in [(100_003, 77_777, 1 << 30), (65_537, 1, 10), (1, 65_537, 10),
                        (250_001, 249_999, 50), (3, 200_000, 5)]:
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        flush(f"tiles dtype={np.dtype(dtype).name} pay={with_pay} n={n} m={m}")
        check(A, B, with_pay)


@pytest.mark.parametrize("p", [1, 2, 5, 17, 256])
def test_forced_p(p):
    g = np.random.default_rng(p)
    A, B = rand_sorted(g, 20_000, 100, np.uint32), rand_sorted(g, 9_000, 100, np.uint32)
    flush(f"forced p={p}")
    check(A, B, True, p_a=p, p_b=p)
    check(A, B, False, p_a=p, p_b=max(1, p // 2))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_subproblem_sizes_across_kernels(dtype, with_pay):
    """Forced block counts whose subproblems span every merge kernel: the
    register-pipelined one, the nine-chunk one, the
    one-workgroup-per-subproblem one and the second-level split."""
    g = np.random.default_rng(44)
    A, B = rand_sorted(g, 60_001, 500, dtype), rand_sorted(g, 59_999, 500, dtype)
    for blk in (1000, 2600, 3000, 4100, 6000, 8200, 12_000, 30_000):
        p = max(1, -(-len(A) // blk))
        flush(f"subproblem sizes dtype={np.dtype(dtype).name} pay={with_pay} block={blk} p={p}")
        check(A, B, with_pay, p_a=p, p_b=p)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_large_subproblems_few_and_many(dtype, with_pay):
    """Subproblems too large for the register-pipelined merge: up to four
    per compute unit they take the workgroups that select their own cases
    (1024 lanes), past that the descriptor kernels (nine-chunk pipelined or
    one workgroup per subproblem)."""
    g = np.random.default_rng(90 + DTYPES.index(dtype) + 10 * with_pay)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    side_max = 2 * cus + 200
    A0 = rand_sorted(g, 4700 * side_max, 5000, dtype)
    B0 = rand_sorted(g, 4700 * side_max, 5000, dtype)
    for blk in (3000, 4700):
        for side in (1, 100, 2 * cus, side_max):
            n = blk * side
            A, B = A0[:n], B0[:n - 1]
            flush(f"large subproblems dtype={np.dtype(dtype).name} pay={with_pay} block={blk} "
                  f"p={side}")
            check(A, B, with_pay, p_a=side, p_b=side)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_few_blocks_merge_and_pieces(dtype, with_pay):
    """Few block starts over large subproblems (group searches, then the
    workgroups that take their cases from the cross ranks): merge() and
    partition() + merge_pieces() both give the oracle's bytes, and the
    partition agrees with the oracle's cross ranks.  Heavy ties, ragged
    ends, p_a != p_b and an empty side included."""
    g = np.random.default_rng(120 + DTYPES.index(dtype) + 10 * with_pay)
    for n, m, p_a, p_b, alpha in [(100_003, 60_001, 40, 25, 50), (30_000, 1, 7, 1, 3),
                                   (1, 30_000, 1, 9, 3), (0, 20_000, 3, 5, 10),
                                   (50_000, 50_000, 16, 16, 1), (200_001, 100_000, 100, 60, 1 << 20)]:
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        pa = pb = None
        if with_pay:
            pa, pb = datagen.source_tag_payloads(n, m)
        rk, rp = oracle.merge(A, B, pa, pb)
        keys = dev(np.concatenate([A, B]))
        pay = None if pa is None else dev(np.concatenate([pa, pb]).astype(np.uint32))
        flush(f"few blocks dtype={np.dtype(dtype).name} pay={with_pay} n={n} m={m} "
              f"p_a={p_a} p_b={p_b}")
        ck, cp = sm.merge(keys, n, m, pay, p_a=p_a, p_b=p_b)
        xb, yb = sm.partition(keys, n, m, p_a, p_b)
        ck2, cp2 = sm.merge_pieces(keys, n, m, p_a, p_b, xb, yb, pay)
        torch.cuda.synchronize()
        rx, ry = oracle.cross_ranks(A, B, p_a, p_b)
        assert np.array_equal(host(xb), rx) and np.array_equal(host(yb), ry)
        for k, pp in ((ck, cp), (ck2, cp2)):
            assert np.array_equal(host(k), rk)
            if with_pay:
                assert np.array_equal(host(pp), rp)


@pytest.mark.parametrize("dtype", DTYPES)
def test_forced_few_blocks_large(dtype):
    """Few forced blocks over large arrays: subproblems far beyond one
    workgroup are split again by the method (two levels)."""
    g = np.random.default_rng(41)
    A, B = rand_sorted(g, 300_001, 1000, dtype), rand_sorted(g, 200_003, 1000, dtype)
    for pa, pb in [(1, 1), (2, 3), (7, 1)]:
        flush(f"forced large dtype={np.dtype(dtype).name} p_a={pa} p_b={pb}")
        check(A, B, True, p_a=pa, p_b=pb)
        check(A, B, False, p_a=pa, p_b=pb, tile=100)


def test_tiling_independence():
    """A stable merge is unique: every tiling gives the same bytes."""
    g = np.random.default_rng(3)
    A, B = rand_sorted(g, 50_000, 64, np.int32), rand_sorted(g, 30_000, 64, np.int32)
    pa, pb = datagen.source_tag_payloads(len(A), len(B))
    ref = run_merge(A, B, pa, pb)
    # 1526 and 1528 sit on either side of the largest payload block length
    # that three register chunks per thread can stage
    for kw in [dict(tile=1), dict(tile=16), dict(tile=1000), dict(tile=1526), dict(tile=1528),
               dict(tile=3072), dict(tile=4096),
               dict(p_a=3, p_b=7),
               dict(p_a=1000, p_b=1)]:
        flush(f"tiling {kw}")
        got = run_merge(A, B, pa, pb, **kw)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


@pytest.mark.parametrize("dtype", DTYPES)
def test_special_cases(dtype):
    z = np.zeros(0, dtype=dtype)
    k = lambda *v: np.array(v, dtype=dtype)
    ar = lambda lo, hi, st=1: np.arange(lo, hi, st).astype(dtype)
    cases = [(z, z), (ar(0, 10), z), (z, ar(0, 10)), (k(5, 5, 5, 5), k(5, 5, 5)),
             (ar(0, 5000), ar(4999, 9000)), (ar(5000, 9000), ar(0, 5000)),
             (ar(0, 20000, 2), ar(1, 20001, 2)), (k(3), k(3)),
             (np.full(10000, 7, dtype), np.full(9000, 7, dtype))]
    for A, B in cases:
        flush(f"special dtype={np.dtype(dtype).name} n={len(A)} m={len(B)}")
        check(A, B, True)
        check(A, B, False)
        check(A, B, True, tile=1)


@pytest.mark.parametrize("dtype", DTYPES)
def test_small_blocks_keys_only(dtype):
    """Blocks of at most 16 elements without payloads: the one-lane-per-
    subproblem merge that loads each part into registers."""
    g = np.random.default_rng(8)
    for n, m, alpha in [(5000, 3001, 7), (1, 999, 3), (999, 1, 3), (40_000, 40_000, 1 << 30),
                        (17, 0, 5), (0, 33, 5)]:
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        for kw in (dict(tile=1), dict(tile=7), dict(tile=16),
                   dict(p_a=max(1, n // 16), p_b=max(1, m // 16))):
            flush(f"small blocks dtype={np.dtype(dtype).name} n={n} m={m} {kw}")
            check(A, B, False, **kw)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("with_pay", [False, True])
def test_small_blocks_staging_limits(dtype, with_pay):
    """Small blocks where one workgroup's 64 A blocks enclose far more B
    elements than it stages (it merges from global memory), mixed with
    workgroups that stage; empty sides; blocks of one element."""
    g = np.random.default_rng(9)
    for n, m, alpha, kw in [(100, 100_000, 1 << 20, dict(tile=1)),
                            (100_000, 100, 1 << 20, dict(tile=1)),
                            (5000, 300_000, 1 << 16, dict(p_a=5000 // 16, p_b=300_000 // 16)),
                            (0, 5000, 100, dict(tile=1)), (5000, 0, 100, dict(tile=1)),
                            (70_001, 70_003, 3, dict(tile=16)),
                            (1 << 16, 1 << 16, 1 << 30, dict(tile=32))]:
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        # clustered keys: many B elements between neighbouring A block starts
        if n and m and alpha == 1 << 16:
            B = np.sort(np.concatenate([B[: m // 2], np.full(m - m // 2, A[n // 2], dtype)]))
        flush(f"staging limits dtype={np.dtype(dtype).name} pay={with_pay} n={n} m={m} {kw}")
        check(A, B, with_pay, **kw)


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_float_total_order_merge(dt):
    """Float keys merge in IEEE 754 totalOrder: specials (NaNs of both signs,
    infinities, -0 before +0, subnormals) sorted by the oracle, then merged
    on the GPU with payloads at several block lengths, against the oracle."""
    seq = total_order_sequence(dt)
    g = np.random.default_rng(17)
    for n, m in [(3000, 2000), (100_003, 7), (1, 40_000)]:
        A, _ = oracle.sort(seq[g.integers(0, len(seq), size=n)], None, 512)
        B, _ = oracle.sort(seq[g.integers(0, len(seq), size=m)], None, 512)
        for kw in (dict(), dict(tile=1), dict(tile=16), dict(p_a=3, p_b=5)):
            flush(f"float total order {np.dtype(dt).name} n={n} m={m} {kw}")
            ck, cp = run_merge(A, B, *datagen.source_tag_payloads(n, m), **kw)
            rk, rp = oracle.merge(A, B, *datagen.source_tag_payloads(n, m))
            ut = np.uint32 if dt == np.float32 else np.uint64
            assert np.array_equal(ck.view(ut), rk.view(ut)) and np.array_equal(cp, rp)


def test_validate_detects_unsorted():
    A = np.array([1, 2, 3, 2], dtype=np.uint32)
    B = np.array([1, 5], dtype=np.uint32)
    with pytest.raises(sm.SMError) as e:
        sm.merge(dev(np.concatenate([A, B])), 4, 2, validate=True)
    assert e.value.code == -6
    check(np.sort(A), B, True, validate=True)


def test_alias_rejected():
    keys = dev(np.arange(10, dtype=np.uint32))
    with pytest.raises(sm.SMError) as e:
        sm.merge(keys, 5, 5, out_keys=keys)
    assert e.value.code == -3


def test_unaligned_view():
    """A view that starts 1 element into a buffer is rejected, not misread."""
    keys = dev(np.arange(11, dtype=np.uint32))[1:]
    with pytest.raises(sm.SMError) as e:
        sm.merge(keys, 5, 5)
    assert e.value.code == -1


@pytest.mark.slow
def test_uniform_u32_2x2e28_full():
    """n = m = 2^28 uint32 uniform over the full range, keys only: the whole
    output against the oracle, in the default launch configuration."""
    n = m = 1 << 28
    flush("uniform uint32 2^28 + 2^28 generate")
    A, B = datagen.uniform_pair(n, m, 0, 2 ** 32, np.uint32, seed=datagen.BASE_SEED + 1)
    keys = dev(np.concatenate([A, B]))
    flush("uniform uint32 2^28 + 2^28 gpu merge")
    ck, _ = sm.merge(keys, n, m)
    torch.cuda.synchronize()
    got = host(ck)
    del keys, ck
    flush("uniform uint32 2^28 + 2^28 oracle merge")
    ref, _ = oracle.merge(A, B)
    assert np.array_equal(got, ref)


@pytest.mark.slow
def test_zipf_u64_2e27_2e23_full():
    """n = 2^27, m = 2^23 uint64 Zipf(1.1) keys, payload = concatenated index."""
    n, m = 1 << 27, 1 << 23
    flush("zipf uint64 2^27 + 2^23 generate")
    A, B = datagen.zipf_pair(n, m, 1.1, 10 ** 6, seed=datagen.BASE_SEED + 2)
    pa, pb = datagen.index_payloads(n, m)
    keys = dev(np.concatenate([A, B]))
    pay = dev(np.concatenate([pa, pb]))
    flush("zipf uint64 2^27 + 2^23 gpu merge")
    ck, cp = sm.merge(keys, n, m, pay)
    torch.cuda.synchronize()
    gk, gp = host(ck), host(cp)
    del keys, pay, ck, cp
    flush("zipf uint64 2^27 + 2^23 oracle merge")
    rk, rp = oracle.merge(A, B, pa, pb)
    assert np.array_equal(gk, rk) and np.array_equal(gp, rp)


@pytest.mark.slow
def test_beyond_32bit_indices():
    """n = m = 2^31 uint32 keys (2^32 elements, 16 GiB per array): indices
    and byte offsets past 32 bits, and windows far apart in one buffer.
    Keys are built sorted on the GPU as prefix sums of 0/1 steps (heavy
    ties).  Checks: the output is non-decreasing, and for sampled elements
    of A and of B the oracle's cross rank gives the output slot holding
    exactly that key (a stable merge puts A[i] at i + rank_low(A[i], B) and
    B[j] at j + rank_high(B[j], A))."""
    n = m = 1 << 31
    dev_ = torch.device("cuda:0")
    gen = torch.Generator(device=dev_)
    gen.manual_seed(datagen.BASE_SEED + 9)
    flush("2^31 + 2^31 generate")
    keys = torch.empty(n + m, dtype=torch.int32, device=dev_)
    for lo in (0, n):
        steps = torch.randint(0, 2, (n,), generator=gen, device=dev_, dtype=torch.int32)
        keys[lo:lo + n] = torch.cumsum(steps, 0, dtype=torch.int32)
        del steps
    keys = keys.view(torch.uint32)
    flush("2^31 + 2^31 gpu merge")
    out, _ = sm.merge(keys, n, m)
    torch.cuda.synchronize()
    o32 = out.view(torch.int32)
    for lo in range(0, n + m, 1 << 30):
        hi = min(lo + (1 << 30) + 1, n + m)
        assert bool((o32[lo + 1:hi] >= o32[lo:hi - 1]).all()), f"not sorted near {lo}"
    flush("2^31 + 2^31 sampled ranks")
    A = host(keys[:n])
    B = host(keys[n:])
    g = np.random.default_rng(3)
    ia = g.integers(0, n, 3000)
    jb = g.integers(0, m, 3000)
    pos = np.concatenate([ia + np.array([oracle.rank_low(A[i], B) for i in ia]),
                          jb + np.array([oracle.rank_high(B[j], A) for j in jb])])
    want = np.concatenate([A[ia], B[jb]])
    got = host(o32[torch.as_tensor(pos, device=dev_)]).view(np.uint32)
    assert np.array_equal(got, want)


@pytest.mark.slow
def test_payloads_beyond_4gib():
    """n = m = 2^30 uint32 keys with uint32 payloads (each array 4 GiB, so
    neither keys nor payloads fit one 32-bit buffer resource): the output
    keys are non-decreasing, and for sampled elements of A and of B the
    slot the oracle's cross rank gives holds that key and its payload (the
    element's index in A||B), which a stable merge fixes exactly."""
    n = m = 1 << 30
    dev_ = torch.device("cuda:0")
    gen = torch.Generator(device=dev_)
    gen.manual_seed(datagen.BASE_SEED + 10)
    flush("2^30 + 2^30 with payloads: generate")
    keys = torch.empty(n + m, dtype=torch.int32, device=dev_)
    for lo in (0, n):
        steps = torch.randint(0, 2, (n,), generator=gen, device=dev_, dtype=torch.int32)
        keys[lo:lo + n] = torch.cumsum(steps, 0, dtype=torch.int32)
        del steps
    keys = keys.view(torch.uint32)
    pay = torch.arange(n + m, dtype=torch.int64, device=dev_).to(torch.int32).view(torch.uint32)
    flush("2^30 + 2^30 with payloads: gpu merge")
    out, out_pay = sm.merge(keys, n, m, pay)
    torch.cuda.synchronize()
    del pay
    o32 = out.view(torch.int32)
    for lo in range(0, n + m, 1 << 29):
        hi = min(lo + (1 << 29) + 1, n + m)
        assert bool((o32[lo + 1:hi] >= o32[lo:hi - 1]).all()), f"not sorted near {lo}"
    flush("2^30 + 2^30 with payloads: sampled ranks")
    A = host(keys[:n])
    B = host(keys[n:])
    g = np.random.default_rng(4)
    ia = g.integers(0, n, 3000)
    jb = g.integers(0, m, 3000)
    pos = np.concatenate([ia + np.array([oracle.rank_low(A[i], B) for i in ia]),
                          jb + np.array([oracle.rank_high(B[j], A) for j in jb])])
    idx = torch.as_tensor(pos, device=dev_)
    got_k = host(o32[idx]).view(np.uint32)
    got_p = host(out_pay.view(torch.int32)[idx]).view(np.uint32)
    assert np.array_equal(got_k, np.concatenate([A[ia], B[jb]]))
    assert np.array_equal(got_p, np.concatenate([ia, n + jb]).astype(np.uint32))
