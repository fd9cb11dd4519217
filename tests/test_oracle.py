"""Pins of the CPU oracle against facts the paper and mathematics fix.

Nothing here compares the oracle with itself.  The pins are:
  * Figure 1 of the paper (block starts, cross ranks, the ten subproblems and
    their case letters), stored in tests/golden/figure1.json;
  * the counting definitions of rank_low / rank_high (Section 2);
  * brute force: Python's sort of (key, source, index)-tagged elements, and
    numpy's stable argsort of the concatenation A || B;
  * the closed-form output positions (Section 2, after Observation 1);
  * invariants: the 2p subproblems tile A, B and C, each holds at most
    ceil(n/p_a) + ceil(m/p_b) elements (Section 2, Theorem 1 discussion),
    Observation 1;
  * special cases (empty inputs, all-equal keys, disjoint ranges, p >= n+m).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle import mlp
from helpers import total_order_sequence

GOLD = os.path.join(os.path.dirname(__file__), "golden", "figure1.json")
DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def fig1():
    with open(GOLD) as f:
        g = json.load(f)
    return g, np.array(g["A"], dtype=np.int32), np.array(g["B"], dtype=np.int32)


def brute_merge(A, B, pa=None, pb=None):
    """Stable merge by sorting (key, source, index) tags with Python's sort."""
    tags = [(a.item(), 0, i) for i, a in enumerate(A)] + [(b.item(), 1, j) for j, b in enumerate(B)]
    tags.sort()
    keys = np.array([t[0] for t in tags], dtype=A.dtype) if tags else np.zeros(0, A.dtype)
    if pa is None:
        return keys, None
    pay = np.array([(pa if s == 0 else pb)[i] for _, s, i in tags], dtype=np.uint32)
    return keys, pay


def argsort_merge(A, B, pa, pb):
    """numpy stable argsort of A || B: equal keys keep A first, then index order."""
    cat = np.concatenate([A, B])
    order = np.argsort(cat, kind="stable")
    return cat[order], np.concatenate([pa, pb])[order]


def rand_sorted(g, n, alphabet, dtype):
    if dtype == np.int32:
        x = g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n).astype(np.int32)
    elif dtype == np.uint32:
        x = (g.integers(0, alphabet, size=n) + (2 ** 32 - alphabet) * g.integers(0, 2)).astype(np.uint32)
    elif dtype == np.int64:
        # both signs, magnitudes beyond 32 bits
        x = (g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n).astype(np.int64)
             * np.int64(0x0100000001))
    elif dtype in (np.float32, np.float64):
        # no NaN and no -0: numeric order is the totalOrder here
        x = (g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n) * 0.375).astype(dtype)
    else:
        x = (g.integers(0, alphabet, size=n).astype(np.uint64) * np.uint64(0x0100000000000001))
    x.sort()
    return x


# --------------------------------------------------------------------------
# Figure 1 (Section 2): the worked example, n = 18, m = 15, p = 5
# --------------------------------------------------------------------------

def test_figure1_block_starts():
    g, A, B = fig1()
    p = g["p"]
    assert [oracle.block_start(len(A), p, i) for i in range(p + 1)] == g["x"]
    assert [oracle.block_start(len(B), p, j) for j in range(p + 1)] == g["y"]


def test_figure1_cross_ranks():
    g, A, B = fig1()
    xbar, ybar = oracle.cross_ranks(A, B, g["p"])
    assert xbar.tolist() == g["xbar"]
    assert ybar.tolist() == g["ybar"]


def test_figure1_subproblems_and_cases():
    g, A, B = fig1()
    p = g["p"]
    xbar, ybar = oracle.cross_ranks(A, B, p)
    pcs = oracle.pieces(len(A), len(B), p, p, xbar, ybar)
    got = {}
    for s, (alo, ahi, blo, bhi, coff, kase) in enumerate(pcs):
        name = ("A%d" % s) if s < p else ("B%d" % (s - p))
        got[name] = dict(A=[alo, ahi - 1] if ahi > alo else None,
                         B=[blo, bhi - 1] if bhi > blo else None,
                         C=[coff, coff + (ahi - alo) + (bhi - blo) - 1], case=chr(kase))
    for ref in g["subproblems_caption"]:
        mine = got[ref["block"]]
        assert mine["A"] == ref["A"], ref
        assert mine["B"] == ref["B"], ref
        assert mine["C"] == ref["C"], ref
    for i, letter in g["a_side_cases"].items():
        assert got["A" + i]["case"] == letter
    for j, letter in g["b_side_cases_named_in_caption"].items():
        assert got["B" + j]["case"] == letter.upper()


def test_figure1_merge():
    g, A, B = fig1()
    pa, pb = np.arange(len(A), dtype=np.uint32), np.arange(100, 100 + len(B), dtype=np.uint32)
    ref_k, ref_p = brute_merge(A, B, pa, pb)
    for f in (lambda: oracle.merge(A, B, pa, pb),
              lambda: oracle.merge_by_pieces(A, B, g["p"], g["p"], pa, pb)):
        c, pc = f()
        assert c.tolist() == ref_k.tolist()
        assert pc.tolist() == ref_p.tolist()


# --------------------------------------------------------------------------
# Ranks: counting definitions (Section 2, low and high rank)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
def test_rank_counting_definition(dtype):
    g = np.random.default_rng(7)
    for _ in range(300):
        n = int(g.integers(0, 30))
        X = rand_sorted(g, n, int(g.integers(1, 12)), dtype)
        probe = rand_sorted(g, 5, 14, dtype)
        for x in probe:
            lo, hi = oracle.rank_low(x, X), oracle.rank_high(x, X)
            assert lo == int(np.sum(X < x))
            assert hi == int(np.sum(X <= x))
            # the defining inequalities with sentinels X[-1] = -inf, X[n] = +inf
            assert (lo == 0 or X[lo - 1] < x) and (lo == n or x <= X[lo])
            assert (hi == 0 or X[hi - 1] <= x) and (hi == n or x < X[hi])


# --------------------------------------------------------------------------
# O1 / O2 against brute force
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", DTYPES)
def test_merge_brute_force(dtype):
    g = np.random.default_rng(11)
    for _ in range(400):
        n, m = int(g.integers(0, 41)), int(g.integers(0, 41))
        alpha = int(g.integers(1, 51))
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        pa = g.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        pb = g.integers(0, 2 ** 32, size=m, dtype=np.uint64).astype(np.uint32)
        rk, rp = brute_merge(A, B, pa, pb)
        c, pc = oracle.merge(A, B, pa, pb)
        assert np.array_equal(c, rk) and np.array_equal(pc, rp)
        c2, pc2, ok = oracle.merge_scatter(A, B, pa, pb)
        assert ok
        assert np.array_equal(c2, rk) and np.array_equal(pc2, rp)
        ak, ap = argsort_merge(A, B, pa, pb)
        assert np.array_equal(ak, rk) and np.array_equal(ap, rp)


@pytest.mark.parametrize("dtype", [np.int32, np.uint64, np.float32])
def test_merge_batched_brute_force(dtype):
    """O5 (every pair merged on its own) against the brute-force stable sort
    of each pair's tagged elements; empty pairs, empty sides and m > n
    included, and a pair range merged alone leaves the rest untouched."""
    g = np.random.default_rng(29)
    lengths = [(0, 0), (5, 0), (0, 7), (1, 1)] + [(int(g.integers(0, 30)), int(g.integers(0, 30)))
                                                  for _ in range(60)]
    parts, offsets, n_a = [], [0], []
    for n, m in lengths:
        parts += [rand_sorted(g, n, 9, dtype), rand_sorted(g, m, 9, dtype)]
        offsets.append(offsets[-1] + n + m)
        n_a.append(n)
    keys = np.concatenate(parts).astype(dtype)
    offsets, n_a = np.array(offsets, np.int64), np.array(n_a, np.int64)
    pay = g.integers(0, 2 ** 32, size=len(keys), dtype=np.uint64).astype(np.uint32)
    ck, cp = oracle.merge_batched(keys, offsets, n_a, pay)
    for k, (n, m) in enumerate(lengths):
        lo = offsets[k]
        rk, rp = brute_merge(keys[lo:lo + n], keys[lo + n:lo + n + m], pay[lo:lo + n],
                             pay[lo + n:lo + n + m])
        assert np.array_equal(ck[lo:lo + n + m], rk) and np.array_equal(cp[lo:lo + n + m], rp)
    out = np.full(len(keys), 7, dtype=dtype)
    oracle.merge_batched(keys, offsets, n_a, pairs=(10, 20), out=out)
    assert np.all(out[:offsets[10]] == 7) and np.all(out[offsets[20]:] == 7)
    assert np.array_equal(out[offsets[10]:offsets[20]], ck[offsets[10]:offsets[20]])


def test_merge_keys_only():
    g = np.random.default_rng(3)
    A, B = rand_sorted(g, 100, 20, np.uint32), rand_sorted(g, 70, 20, np.uint32)
    c, pc = oracle.merge(A, B)
    assert pc is None
    assert np.array_equal(c, brute_merge(A, B)[0])


# --------------------------------------------------------------------------
# Steps 1-4: the method against brute force, exhaustively on tiny inputs
# --------------------------------------------------------------------------

def nondecreasing(length, alphabet):
    return [np.array(c, dtype=np.int32)
            for c in itertools.combinations_with_replacement(range(alphabet), length)]


def check_tiling(n, m, p_a, p_b, pcs):
    """The 2p subproblems tile A, B and C exactly once, and each holds at most
    ceil(n/p_a) + ceil(m/p_b) elements."""
    ca, cb, cc = np.zeros(n, int), np.zeros(m, int), np.zeros(n + m, int)
    bound = -(-n // p_a) + -(-m // p_b)
    for alo, ahi, blo, bhi, coff, _ in pcs:
        assert 0 <= alo <= ahi <= n and 0 <= blo <= bhi <= m
        ca[alo:ahi] += 1
        cb[blo:bhi] += 1
        cc[coff:coff + (ahi - alo) + (bhi - blo)] += 1
        assert (ahi - alo) + (bhi - blo) <= bound
    assert (ca == 1).all() and (cb == 1).all() and (cc == 1).all()


def test_method_exhaustive_tiny():
    seqs = [s for L in range(0, 5) for s in nondecreasing(L, 3)]
    hit = set()
    for A in seqs:
        for B in seqs:
            ref = brute_merge(A, B)[0]
            n, m = len(A), len(B)
            pa_src = np.arange(n, dtype=np.uint32)
            pb_src = np.arange(n, n + m, dtype=np.uint32)
            ref_p = brute_merge(A, B, pa_src, pb_src)[1]
            for p_a in range(1, 7):
                for p_b in range(1, 7):
                    c, pc = oracle.merge_by_pieces(A, B, p_a, p_b, pa_src, pb_src)
                    assert np.array_equal(c, ref) and np.array_equal(pc, ref_p), (A, B, p_a, p_b)
                    xbar, ybar = oracle.cross_ranks(A, B, p_a, p_b)
                    pcs = oracle.pieces(n, m, p_a, p_b, xbar, ybar)
                    two = oracle.pieces(n, m, p_a, p_b, xbar, ybar, two_select=True)
                    assert np.array_equal(pcs[:, :5], two[:, :5]), (A, B, p_a, p_b)
                    check_tiling(n, m, p_a, p_b, pcs)
                    hit.update(chr(k) for k in pcs[:, 5])
    assert hit == set("abcdeABCDE"), hit


@pytest.mark.parametrize("dtype", DTYPES)
def test_method_random(dtype):
    g = np.random.default_rng(5)
    hit = set()
    for _ in range(1500):
        n, m = int(g.integers(0, 65)), int(g.integers(0, 65))
        alpha = int(g.integers(1, 65))
        A, B = rand_sorted(g, n, alpha, dtype), rand_sorted(g, m, alpha, dtype)
        p_a, p_b = int(g.integers(1, 13)), int(g.integers(1, 13))
        pa = np.arange(n, dtype=np.uint32)
        pb = np.arange(n, n + m, dtype=np.uint32)
        rk, rp = brute_merge(A, B, pa, pb)
        c, pc = oracle.merge_by_pieces(A, B, p_a, p_b, pa, pb)
        assert np.array_equal(c, rk) and np.array_equal(pc, rp)
        xbar, ybar = oracle.cross_ranks(A, B, p_a, p_b)
        pcs = oracle.pieces(n, m, p_a, p_b, xbar, ybar)
        check_tiling(n, m, p_a, p_b, pcs)
        two = oracle.pieces(n, m, p_a, p_b, xbar, ybar, two_select=True)
        assert np.array_equal(pcs[:, :5], two[:, :5])
        hit.update(chr(k) for k in pcs[:, 5])
    assert hit == set("abcdeABCDE")


def test_observation1():
    """Cross ranks do not cross (Section 2, Observation 1): with a = A[i] and
    j = rank_low(a, B), every B[j'] with j' < j has rank_high(B[j'], A) <= i,
    and every B[j''] with j'' >= j has rank_high(B[j''], A) > i."""
    g = np.random.default_rng(9)
    for _ in range(300):
        n, m = int(g.integers(1, 30)), int(g.integers(1, 30))
        alpha = int(g.integers(1, 10))
        A, B = rand_sorted(g, n, alpha, np.int32), rand_sorted(g, m, alpha, np.int32)
        for i in range(n):
            j = oracle.rank_low(A[i], B)
            for jj in range(m):
                r = oracle.rank_high(B[jj], A)
                assert (r <= i) if jj < j else (r > i)


def test_cross_ranks_monotone_large():
    g = np.random.default_rng(1)
    A = np.sort(g.integers(0, 65536, size=100_000).astype(np.int32))
    B = np.sort(g.integers(0, 65536, size=60_000).astype(np.int32))
    xbar, ybar = oracle.cross_ranks(A, B, 256)
    assert (np.diff(xbar) >= 0).all() and (np.diff(ybar) >= 0).all()
    xs = np.array([oracle.block_start(len(A), 256, i) for i in range(256)])
    assert np.array_equal(xbar[:-1], np.searchsorted(B, A[xs], side="left"))
    ys = np.array([oracle.block_start(len(B), 256, j) for j in range(256)])
    assert np.array_equal(ybar[:-1], np.searchsorted(A, B[ys], side="right"))


# --------------------------------------------------------------------------
# Blocks (Section 2): sizes and membership against the definition
# --------------------------------------------------------------------------

def test_block_math():
    for L in range(0, 45):
        for p in range(1, 14):
            starts = [oracle.block_start(L, p, i) for i in range(p + 1)]
            sizes = np.diff(starts)
            assert starts[0] == 0 and starts[-1] == L
            c, r = -(-L // p), L % p
            assert (sizes[:r] == c).all() and (sizes[r:] == L // p).all()
            for k in range(L):
                owners = [i for i in range(p) if starts[i] <= k < starts[i + 1]]
                assert oracle.block_of(L, p, k) == owners[0]
            assert oracle.block_of(L, p, L) == p


# --------------------------------------------------------------------------
# Special cases
# --------------------------------------------------------------------------

@pytest.mark.parametrize("p", [1, 2, 5, 64])
def test_special_cases(p):
    def both(A, B):
        pa = np.arange(len(A), dtype=np.uint32)
        pb = np.arange(len(A), len(A) + len(B), dtype=np.uint32)
        c1, p1 = oracle.merge(A, B, pa, pb)
        c2, p2 = oracle.merge_by_pieces(A, B, p, p, pa, pb)
        assert np.array_equal(c1, c2) and np.array_equal(p1, p2)
        return c1, p1
    u = np.uint32
    A = np.arange(10, dtype=u)
    e = np.zeros(0, dtype=u)
    assert np.array_equal(both(A, e)[0], A)                       # m = 0
    assert np.array_equal(both(e, A)[0], A)                       # n = 0
    eq = np.full(7, 5, dtype=u)
    c, pc = both(eq, np.full(4, 5, dtype=u))                      # all equal: A || B
    assert pc.tolist() == list(range(11))
    c, pc = both(np.arange(5, dtype=u), np.arange(4, 9, dtype=u))  # max A == min B
    assert pc.tolist() == list(range(10))
    c, pc = both(np.arange(10, 15, dtype=u), np.arange(5, dtype=u))  # max B < min A: B || A
    assert pc.tolist() == list(range(5, 10)) + list(range(5))
    c, pc = both(np.array([3], u), np.array([3], u))
    assert pc.tolist() == [0, 1]
    c, pc = both(np.arange(0, 20, 2, dtype=u), np.arange(1, 21, 2, dtype=u))  # interleaved
    assert c.tolist() == list(range(20))
    assert pc.tolist() == [k // 2 + (k % 2) * 10 for k in range(20)]


def test_many_blocks_small_subproblems():
    """p >= n + m: every subproblem holds at most 2 elements."""
    g = np.random.default_rng(2)
    A, B = rand_sorted(g, 9, 4, np.int32), rand_sorted(g, 7, 4, np.int32)
    xbar, ybar = oracle.cross_ranks(A, B, 20, 20)
    pcs = oracle.pieces(9, 7, 20, 20, xbar, ybar)
    assert ((pcs[:, 1] - pcs[:, 0]) + (pcs[:, 3] - pcs[:, 2]) <= 2).all()
    check_tiling(9, 7, 20, 20, pcs)


# --------------------------------------------------------------------------
# O4: stable merge sort (Section 3)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,run_len", [(0, 4), (1, 4), (17, 1), (1000, 3), (5000, 512), (4096, 512),
                                       (4097, 512), (3 * 512 + 5, 512)])
def test_sort_against_stable_argsort(N, run_len):
    g = np.random.default_rng(N + run_len)
    keys = g.integers(0, max(1, N // 8), size=N).astype(np.uint32)
    pay = np.arange(N, dtype=np.uint32)
    k, p = oracle.sort(keys, pay, run_len)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(k, keys[order]) and np.array_equal(p, pay[order])


@pytest.mark.parametrize("dtype", DTYPES)
def test_sort_dtypes(dtype):
    g = np.random.default_rng(4)
    keys = rand_sorted(g, 3000, 50, dtype)
    keys = keys[g.permutation(3000)]
    pay = g.integers(0, 2 ** 32, size=3000, dtype=np.uint64).astype(np.uint32)
    k, p = oracle.sort(keys, pay, 64)
    order = np.argsort(keys, kind="stable")
    assert np.array_equal(k, keys[order]) and np.array_equal(p, pay[order])


# --------------------------------------------------------------------------
# O6: bounded exponential search
# --------------------------------------------------------------------------

# --------------------------------------------------------------------------
# Descending order: the same routines on the reversed order relation
# --------------------------------------------------------------------------

def _desc_index(keys: np.ndarray) -> np.ndarray:
    """Indices of a stable descending sort, by Python's sorted(reverse=True),
    which keeps equal keys in input order; keys compared in their type's
    order (floats here are finite and nonzero-signed, so numeric order)."""
    vals = keys.tolist()
    return np.array(sorted(range(len(vals)), key=vals.__getitem__, reverse=True), dtype=np.int64)


@pytest.mark.parametrize("dtype", DTYPES)
def test_descending_merge_and_sort_brute_force(dtype):
    """With descending=True the merge of two non-increasing arrays is the
    stable descending sort of A || B (ties: A first, each source in order),
    and the sort is the stable descending sort of its input."""
    g = np.random.default_rng(71)
    for _ in range(150):
        n, m = int(g.integers(0, 60)), int(g.integers(0, 60))
        alpha = int(g.integers(1, 12))
        A = rand_sorted(g, n, alpha, dtype)[::-1].copy()
        B = rand_sorted(g, m, alpha, dtype)[::-1].copy()
        cat = np.concatenate([A, B])
        idx = _desc_index(cat)
        pa = np.arange(n, dtype=np.uint32)
        pb = np.arange(n, n + m, dtype=np.uint32)
        c, pc = oracle.merge(A, B, pa, pb, descending=True)
        assert np.array_equal(c, cat[idx]) and np.array_equal(pc, idx.astype(np.uint32))
        p_a, p_b = int(g.integers(1, 9)), int(g.integers(1, 9))
        c2, pc2 = oracle.merge_by_pieces(A, B, p_a, p_b, pa, pb, descending=True)
        assert np.array_equal(c2, c) and np.array_equal(pc2, pc)
        shuffled = g.permutation(cat)
        run = int(g.integers(1, 9))
        sk, sp = oracle.sort(shuffled, np.arange(len(cat), dtype=np.uint32), run, descending=True)
        sidx = _desc_index(shuffled)
        assert np.array_equal(sk, shuffled[sidx]) and np.array_equal(sp, sidx.astype(np.uint32))


def test_descending_ranks_counting_definition():
    """In non-increasing order, rank_low(x, X) counts the elements strictly
    greater than x and rank_high(x, X) those greater than or equal to x."""
    g = np.random.default_rng(72)
    for _ in range(300):
        X = np.sort(g.integers(-20, 20, size=int(g.integers(0, 40))).astype(np.int32))[::-1].copy()
        x = int(g.integers(-25, 25))
        assert oracle.rank_low(x, X, descending=True) == int((X > x).sum())
        assert oracle.rank_high(x, X, descending=True) == int((X >= x).sum())
    A = np.array([9, 7, 7, 3], dtype=np.int32)
    B = np.array([8, 7, 1], dtype=np.int32)
    xbar, ybar = oracle.cross_ranks(A, B, 2, 3, descending=True)
    # A blocks start at 9 and 7: 0 and 1 elements of B come strictly before;
    # B blocks start at 8, 7, 1: 1, 3 and 4 elements of A come at or before
    assert list(xbar) == [0, 1, 3] and list(ybar) == [1, 3, 4, 4]


@pytest.mark.parametrize("is_high", [False, True])
def test_gallop_exact(is_high):
    g = np.random.default_rng(12)
    for _ in range(600):
        n = int(g.integers(0, 300))
        X = rand_sorted(g, n, int(g.integers(1, 60)), np.uint32)
        x = rand_sorted(g, 1, 64, np.uint32)[0]
        r = int(np.sum(X <= x)) if is_high else int(np.sum(X < x))
        for e in (0, 1, -1, 2, -3, 7, -40, 1000, -1000):
            for W in (0, 1, 4, 64, 1 << 20):
                got, probes, fb = oracle.gallop(x, X, is_high, r + e, W)
                assert got == r
                g_cl = min(max(r + e, 0), n)
                dist = abs(g_cl - r)
                if W >= 2 * max(dist, 1):
                    assert not fb
                    # probe at g, gallop to at most 2*dist, bisect the bracket
                    assert probes <= 2 + 2 * (dist.bit_length() + 1)
                if fb:
                    # probe g, the steps up to the window, then the whole of
                    # [0, n] with aligned splits (at most bitlen(n) + 1 reads)
                    assert probes <= 1 + (W.bit_length() + 1) + n.bit_length() + 1


def _trailing_zeros(t: int) -> int:
    return (t & -t).bit_length() - 1


def _aligned_probe_count(lo: int, hi: int, r: int) -> int:
    """Reads of the aligned bisection of [lo, hi] for the answer r, from its
    definition: each read splits at the number in (lo, hi] with the most
    trailing zero bits (found here by scanning the whole interval)."""
    count = 0
    while lo < hi:
        m = max(range(lo + 1, hi + 1), key=_trailing_zeros)
        count += 1
        if r >= m:
            lo = m
        else:
            hi = m - 1
    return count


@pytest.mark.parametrize("is_high", [False, True])
def test_gallop_aligned_bisection(is_high):
    """With window 0 every search gives up at once: after the probe of g it
    bisects [0, n] at the points of most trailing zeros.  Its read count
    equals the count of that definition, and is at most bitlen(n) + 1."""
    g = np.random.default_rng(14)
    for _ in range(300):
        n = int(g.integers(0, 700))
        X = rand_sorted(g, n, int(g.integers(1, 200)), np.uint32)
        x = rand_sorted(g, 1, 256, np.uint32)[0]
        r = int(np.sum(X <= x)) if is_high else int(np.sum(X < x))
        for e in (0, 3, -5, 10_000):
            gs = min(max(r + e, 0), n)
            got, probes, fb = oracle.gallop(x, X, is_high, r + e, 0)
            assert got == r and fb
            assert probes == int(gs < n) + _aligned_probe_count(0, n, r)
            assert probes <= int(gs < n) + n.bit_length() + 1


@pytest.mark.parametrize("is_high", [False, True])
def test_gallop_initial_step(is_high):
    """Any initial step gives the exact rank; with the step at or above the
    guess error, the bracket is found by the first move (at most two probes
    before the bisection of a bracket no wider than the step)."""
    g = np.random.default_rng(13)
    for _ in range(400):
        n = int(g.integers(1, 2000))
        X = rand_sorted(g, n, int(g.integers(1, 400)), np.uint32)
        x = rand_sorted(g, 1, 512, np.uint32)[0]
        r = int(np.sum(X <= x)) if is_high else int(np.sum(X < x))
        for e in (0, 1, -1, 5, -9, 33, -100, 700):
            gs = min(max(r + e, 0), n)
            dist = abs(gs - r)
            for s0 in (1, 2, 8, 64, 512):
                for W in (0, 16, 1024, 1 << 20):
                    got, probes, fb = oracle.gallop(x, X, is_high, r + e, W, step0=s0)
                    assert got == r
                    if s0 > W:
                        # every search moves at least once, and the first move is too far
                        assert fb
                    elif s0 >= dist:
                        # probe g, one step, bisect a bracket of at most s0 elements
                        assert not fb and probes <= 2 + (s0.bit_length() + 1)


# --------------------------------------------------------------------------
# O7: the predictor network
# --------------------------------------------------------------------------

def test_mlp_gradient_finite_differences():
    g = np.random.default_rng(0)
    phi = g.random(200)
    target = np.sort(g.random(200))
    params = g.normal(size=mlp.NPARAM)
    L, grad = mlp.loss_and_grad(params, phi, target)
    assert abs(L - mlp.loss(params, phi, target)) < 1e-15
    h = 1e-6
    for k in range(mlp.NPARAM):
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss(params + e, phi, target) - mlp.loss(params - e, phi, target)) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad[k])), k


def test_adam_first_step_closed_form():
    """With zero moments, the first bias-corrected step is lr * g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    p1, m, v = mlp.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, 0.01)
    assert np.allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_three_steps_from_nonzero_moments():
    """Three Adam updates (Kingma and Ba, 2015: m_t = b1 m_{t-1} + (1 - b1) g_t,
    v_t = b2 v_{t-1} + (1 - b2) g_t^2, p_t = p_{t-1} - lr mhat_t / (sqrt(vhat_t)
    + eps) with mhat_t = m_t / (1 - b1^t), vhat_t = v_t / (1 - b2^t)) from
    m_0 = 2, v_0 = 8, p_0 = 0 with b1 = 3/4, b2 = 7/8, lr = 1, eps = 0 and
    gradients 4, 0, -4 at t = 1, 2, 3.  Worked by hand in fractions:
      t=1: m = 3/2 + 1 = 5/2,  v = 7 + 2 = 9,         mhat = 10,    vhat = 72
      t=2: m = 15/8,           v = 63/8,              mhat = 30/7,  vhat = 168/5
      t=3: m = 45/32 - 1 = 13/32, v = 441/64 + 2 = 569/64,
           mhat = (13/32) / (37/64) = 26/37,  vhat = (569/64) / (169/512) = 4552/169
    Neither b1 nor b2 is 1/2, so exchanging b and 1 - b in either moment, a
    missing bias correction or a power t - 1 in it changes the result."""
    p3_expected = -(10 / math.sqrt(72)) - (30 / 7) / math.sqrt(168 / 5) \
        - (26 / 37) / math.sqrt(4552 / 169)
    p = np.array([0.0])
    m = np.array([2.0])
    v = np.array([8.0])
    seen = []
    for t, g in ((1, 4.0), (2, 0.0), (3, -4.0)):
        p, m, v = mlp.adam_step(p, np.array([g]), m, v, t, 1.0, beta1=0.75, beta2=0.875, eps=0.0)
        seen.append((float(p[0]), float(m[0]), float(v[0])))
    assert seen[0][1] == 2.5 and seen[0][2] == 9.0
    assert abs(seen[0][0] - (-10 / math.sqrt(72))) < 1e-14
    assert seen[1][1] == 15 / 8 and seen[1][2] == 63 / 8
    assert seen[2][1] == 13 / 32 and seen[2][2] == 569 / 64
    assert abs(seen[2][0] - p3_expected) < 1e-13
    # eps is added to the square root, not under it: with vhat = 72 and
    # eps = 1, the first step is 10 / (sqrt(72) + 1)
    p1, _, _ = mlp.adam_step(np.array([0.0]), np.array([4.0]), np.array([2.0]), np.array([8.0]),
                             1, 1.0, beta1=0.75, beta2=0.875, eps=1.0)
    assert abs(float(p1[0]) + 10 / (math.sqrt(72) + 1)) < 1e-14


def _constant_net(b2: float) -> np.ndarray:
    """A network whose output is b2 for every key (first layer and output
    weights zero)."""
    p = np.zeros(mlp.NPARAM)
    p[96] = b2
    return p


def test_predict_rank_rounding_and_clamps():
    """predict_rank = y * len rounded half to even, clamped to [0, len], NaN
    -> 0 (the GPU predictor returns 0 for a non-number as well).  len = 8:
    y = 5/16 -> 2.5 -> 2, 7/16 -> 3.5 -> 4, 3/16 -> 1.5 -> 2, 9/16 -> 4.5 -> 4;
    y < 0 -> 0; y * len > len -> len; +inf -> len, -inf and NaN -> 0."""
    keys = np.array([0, 7, 2 ** 32 - 1], dtype=np.uint32)
    cases = [(5 / 16, 2), (7 / 16, 4), (3 / 16, 2), (9 / 16, 4), (0.0, 0), (1.0, 8),
             (-0.25, 0), (1.25, 8), (math.inf, 8), (-math.inf, 0), (math.nan, 0)]
    for b2, want in cases:
        with np.errstate(invalid="ignore"):
            got = mlp.predict_rank(_constant_net(b2), keys, 8)
        assert got.dtype == np.int64
        assert list(got) == [want] * 3, (b2, got)
    # an empty target array: every prediction is 0
    assert list(mlp.predict_rank(_constant_net(0.7), keys, 0)) == [0, 0, 0]


def test_predict_rank_through_hidden_unit():
    """One hidden unit h = ReLU(phi - 1/2) with output 1/4 + 2 h.  uint32 keys:
    phi(0) = 0 -> y = 1/4; phi(2^24 - 1) = log2(2^24) / 32 = 3/4 -> y = 3/4;
    phi(2^32 - 1) = 1 -> y = 5/4.  With len = 8: 2, 6 and 8 (clamped)."""
    p = np.zeros(mlp.NPARAM)
    p[0] = 1.0       # W1[0]
    p[32] = -0.5     # b1[0]
    p[64] = 2.0      # w2[0]
    p[96] = 0.25     # b2
    keys = np.array([0, 2 ** 24 - 1, 2 ** 32 - 1], dtype=np.uint32)
    assert list(mlp.predict_rank(p, keys, 8)) == [2, 6, 8]
    # a negative W1 turns the unit off above the knot: h = ReLU(1/2 - phi)
    # gives y = 5/4 (clamped to 8), 1/4 and 1/4
    p[0], p[32] = -1.0, 0.5
    assert list(mlp.predict_rank(p, keys, 8)) == [8, 2, 2]


def test_mlp_init_interpolates_knots():
    """The initial network passes through every knot (c_k, t_k), is flat at
    t_0 below the first knot and linear between neighbouring knots."""
    g = np.random.default_rng(5)
    phi = np.sort(g.random(5000))
    target = np.sort(g.random(5000))
    p = mlp.init_params(phi, target)
    idx = ((np.arange(32) + 0.5) * 5000 / 32).astype(np.int64)
    c, t = phi[idx], target[idx]
    y, _, _ = mlp.forward(p, c)
    assert np.allclose(y, t, rtol=0, atol=1e-9)
    below, _, _ = mlp.forward(p, np.array([0.0, c[0] * 0.5]))
    assert np.allclose(below, t[0], atol=1e-12)
    mid = (c[:-1] + c[1:]) / 2
    ym, _, _ = mlp.forward(p, mid)
    assert np.allclose(ym, (t[:-1] + t[1:]) / 2, atol=1e-9)
    # tied knots (a run of equal features) give a zero slope, not a division by zero
    phi2 = np.concatenate([np.zeros(3000), np.linspace(0.5, 1.0, 2000)])
    p2 = mlp.init_params(phi2, np.linspace(0, 1, 5000))
    assert np.isfinite(p2).all()


def test_mlp_features_order_preserving():
    k32 = np.array([-2 ** 31, -1, 0, 1, 2 ** 31 - 1], dtype=np.int32)
    f = mlp.features(k32)
    assert (np.diff(f) > 0).all() and f[0] == 0.0
    ku = np.array([0, 1, 2 ** 32 - 1], dtype=np.uint32)
    assert np.isclose(mlp.features(ku)[-1], 1.0)
    k64 = np.array([-2 ** 63, -1, 0, 1, 2 ** 63 - 1], dtype=np.int64)
    u64 = [int(v) for v in mlp.unsigned_order(k64)]
    assert u64 == [0, 2 ** 63 - 1, 2 ** 63, 2 ** 63 + 1, 2 ** 64 - 1]
    for dt in (np.float32, np.float64):
        seq = total_order_sequence(dt)
        u = mlp.unsigned_order(seq)
        assert all(int(u[i]) < int(u[i + 1]) for i in range(len(u) - 1))
        assert int(u[0]) == 0 and int(u[-1]) == 2 ** (8 * seq.itemsize) - 1


# --------------------------------------------------------------------------
# Float keys: IEEE 754 totalOrder
# --------------------------------------------------------------------------

@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_float_total_order(dt):
    """The oracle's sort of shuffled specials gives back the totalOrder
    sequence bit for bit (-0 strictly before +0, NaNs by sign and payload);
    finite non-zero values follow numeric order; a merge of two sorted
    subsets equals the sorted union."""
    seq = total_order_sequence(dt)
    ut = np.uint32 if dt == np.float32 else np.uint64
    g = np.random.default_rng(21)
    for _ in range(20):
        perm = g.permutation(len(seq))
        k, _ = oracle.sort(seq[perm], np.arange(len(seq), dtype=np.uint32), 4)
        assert np.array_equal(k.view(ut), seq.view(ut))
        take = np.sort(g.choice(len(seq), size=len(seq) // 2, replace=False))
        rest = np.setdiff1d(np.arange(len(seq)), take)
        c, _ = oracle.merge(seq[take], seq[rest])
        assert np.array_equal(c.view(ut), seq.view(ut))
    vals = (g.standard_normal(500) * 10.0 ** g.integers(-30, 30, 500)).astype(dt)
    vals = vals[vals != 0]
    k, _ = oracle.sort(vals, np.arange(len(vals), dtype=np.uint32), 64)
    assert np.array_equal(k, np.sort(vals))


def test_error_bins():
    assert oracle.error_bin(0) == 32
    assert oracle.error_bin(1) == 33 and oracle.error_bin(-1) == 31
    assert oracle.error_bin(2) == 34 and oracle.error_bin(3) == 34 and oracle.error_bin(4) == 35
    assert oracle.error_bin(-7) == 29 and oracle.error_bin(-8) == 28
    assert oracle.error_bin(2 ** 40) == 64 and oracle.error_bin(-(2 ** 40)) == 0


# --------------------------------------------------------------------------
# A config-1 shaped case: heavy duplicates, p = 256
# --------------------------------------------------------------------------

def test_int32_heavy_ties_shape_small():
    g = np.random.default_rng(17)
    A = np.sort(g.integers(0, 65536, size=200_000).astype(np.int32))
    B = np.sort(g.integers(0, 65536, size=120_000).astype(np.int32))
    pa = np.arange(len(A), dtype=np.uint32)
    pb = np.arange(len(B), dtype=np.uint32) | np.uint32(1 << 31)
    ak, ap = argsort_merge(A, B, pa, pb)
    c, pc = oracle.merge(A, B, pa, pb)
    assert np.array_equal(c, ak) and np.array_equal(pc, ap)
    c, pc = oracle.merge_by_pieces(A, B, 256, 256, pa, pb)
    assert np.array_equal(c, ak) and np.array_equal(pc, ap)


def successor_property(A, B, pcs):
    """For each subproblem: the element after its A range is strictly greater
    than every element of its B range, and the element after its B range is
    greater than or equal to every element of its A range (when they exist).
    The GPU merge loop relies on this to run without bounds checks."""
    n, m = len(A), len(B)
    for alo, ahi, blo, bhi, _, _ in pcs:
        if ahi < n and bhi > blo:
            assert A[ahi] > B[blo:bhi].max()
        if bhi < m and ahi > alo:
            assert B[bhi] >= A[alo:ahi].max()


def test_successor_sentinels_exhaustive():
    seqs = [s for L in range(0, 5) for s in nondecreasing(L, 3)]
    for A in seqs:
        for B in seqs:
            for p_a in range(1, 6):
                for p_b in range(1, 6):
                    xbar, ybar = oracle.cross_ranks(A, B, p_a, p_b)
                    successor_property(A, B, oracle.pieces(len(A), len(B), p_a, p_b, xbar, ybar))


def test_successor_sentinels_random():
    g = np.random.default_rng(31)
    for _ in range(2000):
        n, m = int(g.integers(0, 80)), int(g.integers(0, 80))
        alpha = int(g.integers(1, 40))
        A, B = rand_sorted(g, n, alpha, np.int32), rand_sorted(g, m, alpha, np.int32)
        p_a, p_b = int(g.integers(1, 20)), int(g.integers(1, 20))
        xbar, ybar = oracle.cross_ranks(A, B, p_a, p_b)
        successor_property(A, B, oracle.pieces(n, m, p_a, p_b, xbar, ybar))
