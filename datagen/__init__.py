"""Seeded synthetic inputs for the stable merge tests and benchmarks.

This module only draws random numbers and sorts them with numpy; it holds none
of the merge method's arithmetic, so both the CPU oracle and the GPU library
can be fed from it.  Every generator takes an explicit seed and returns numpy
arrays that are already sorted where the method requires sorted input.

Workloads (the shapes of the stable-merge configurations):
  * ``uniform_pair``   - two sorted arrays of uniform integers in [lo, hi)
  * ``source_tag_payloads`` - payload (src << 31) | index_in_source
  * ``zipf_pair``      - sorted uint64 keys whose values follow Zipf(s) over
                          a fixed set of distinct random 64-bit values
  * ``lognormal_mixture`` - sorted uint32 keys from a 3-component log-normal
                          mixture (medians 2^10, 2^20, 2^28, sigma 0.5)
  * ``batch_lengths``  - per-pair (n_k, m_k) with log-uniform totals
  * ``batched_pairs``  - contiguous sorted A_k || B_k segments
  * ``sort_input``     - unsorted (key, index) pairs for the merge sort
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 0x12026575

_KEY_RANGE = {np.int32: (-(2 ** 31), 2 ** 31), np.uint32: (0, 2 ** 32),
              np.uint64: (0, 2 ** 64)}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_keys(count: int, lo: int, hi: int, dtype, seed: int, sort: bool = True):
    """count integers uniform in [lo, hi) of the given numpy dtype."""
    g = rng(seed)
    if dtype == np.uint64 and hi > 2 ** 63:
        x = g.integers(0, 2 ** 64, size=count, dtype=np.uint64, endpoint=False)
        if lo != 0 or hi != 2 ** 64:
            x = (x % np.uint64(hi - lo)) + np.uint64(lo)
    else:
        x = g.integers(lo, hi, size=count, dtype=dtype)
    if sort:
        x.sort()
    return x


def uniform_pair(n: int, m: int, lo: int, hi: int, dtype, seed: int):
    """Sorted A (n) and B (m), independent uniform draws in [lo, hi)."""
    A = uniform_keys(n, lo, hi, dtype, seed * 2 + 1)
    B = uniform_keys(m, lo, hi, dtype, seed * 2 + 2)
    return A, B


def concat(A, B):
    """The library's input layout: A followed by B in one buffer."""
    return np.concatenate([A, B])


def source_tag_payloads(n: int, m: int):
    """(src << 31) | index_in_source, src 0 for A and 1 for B."""
    pa = np.arange(n, dtype=np.uint32)
    pb = np.arange(m, dtype=np.uint32) | np.uint32(1 << 31)
    return pa, pb


def index_payloads(n: int, m: int):
    """Index in the concatenated A || B buffer."""
    return np.arange(n, dtype=np.uint32), np.arange(n, n + m, dtype=np.uint32)


def _splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014), vectorised in uint64."""
    x = x.astype(np.uint64)
    with np.errstate(over="ignore"):
        x = x + np.uint64(0x9E3779B97F4A7C15)
        x = (x ^ (x >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        x = (x ^ (x >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        x = x ^ (x >> np.uint64(31))
    return x


def zipf_values(distinct: int, seed: int) -> np.ndarray:
    """The distinct key values, value of Zipf rank r is splitmix64(seed ^ r)."""
    r = np.arange(1, distinct + 1, dtype=np.uint64)
    v = _splitmix64(r ^ np.uint64(seed))
    assert len(np.unique(v)) == distinct
    return v


def zipf_keys(count: int, s: float, distinct: int, seed: int, values=None):
    """count sorted uint64 keys; key rank r in [1, distinct] is drawn with
    probability proportional to r^-s by inverse CDF over the exact weights."""
    if values is None:
        values = zipf_values(distinct, BASE_SEED + 3)
    w = np.arange(1, distinct + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng(seed).random(count)
    r = np.minimum(np.searchsorted(cdf, u, side="right"), distinct - 1)
    k = values[r]
    k.sort()
    return k


def zipf_pair(n: int, m: int, s: float = 1.1, distinct: int = 10 ** 6, seed: int = 0):
    values = zipf_values(distinct, BASE_SEED + 3)
    return (zipf_keys(n, s, distinct, seed * 2 + 1, values),
            zipf_keys(m, s, distinct, seed * 2 + 2, values))


def lognormal_mixture(count: int, seed: int, medians_log2=(10, 20, 28), sigma=0.5):
    """Sorted uint32 keys: a component is picked uniformly, then
    key = floor(exp(ln(2^median) + sigma * N(0, 1))) clipped to [0, 2^32 - 1]."""
    g = rng(seed)
    comp = g.integers(0, len(medians_log2), size=count)
    mu = np.log(2.0) * np.asarray(medians_log2, dtype=np.float64)[comp]
    x = np.exp(mu + sigma * g.standard_normal(count))
    x = np.clip(np.floor(x), 0, 2 ** 32 - 1).astype(np.uint32)
    x.sort()
    return x


def batch_lengths(count: int, lo_log2: float, hi_log2: float, seed: int):
    """Per-pair totals L_k = floor(2^U), U ~ U[lo_log2, hi_log2], split as
    m_k = floor(f * L_k), f ~ U[0, 1), n_k = L_k - m_k (so m_k > n_k occurs)."""
    g = rng(seed)
    L = np.floor(2.0 ** g.uniform(lo_log2, hi_log2, size=count)).astype(np.int64)
    f = g.random(count)
    mk = np.floor(f * L).astype(np.int64)
    return L - mk, mk


def batched_pairs(n_k, m_k, lo: int, hi: int, dtype, seed: int):
    """Contiguous A_0 || B_0 || A_1 || B_1 ... with each array sorted.
    Returns (keys, offsets[count+1], n_a[count])."""
    n_k = np.asarray(n_k, dtype=np.int64)
    m_k = np.asarray(m_k, dtype=np.int64)
    tot = n_k + m_k
    offsets = np.zeros(len(tot) + 1, dtype=np.int64)
    np.cumsum(tot, out=offsets[1:])
    keys = uniform_keys(int(offsets[-1]), lo, hi, dtype, seed, sort=False)
    # sort every run at once: sort the composite run_id * (hi - lo) + (key - lo)
    run_len = np.empty(2 * len(tot), dtype=np.int64)
    run_len[0::2] = n_k
    run_len[1::2] = m_k
    span = hi - lo
    assert 2 * len(tot) * span < 2 ** 64
    run_id = np.repeat(np.arange(2 * len(tot), dtype=np.uint64), run_len)
    comp = run_id * np.uint64(span) + (keys.astype(np.int64) - lo).astype(np.uint64)
    comp.sort()
    keys = ((comp % np.uint64(span)).astype(np.int64) + lo).astype(dtype)
    return keys, offsets, n_k.copy()


def sort_input(N: int, key_hi: int, seed: int):
    """Unsorted uint32 keys uniform in [0, key_hi) and payload = index."""
    keys = uniform_keys(N, 0, key_hi, np.uint32, seed, sort=False)
    return keys, np.arange(N, dtype=np.uint32)
