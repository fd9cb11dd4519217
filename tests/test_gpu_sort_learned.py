"""The merge sort with learned cross ranks in every pass: byte for byte the
plain sort's output (and the oracle's) whatever the model, with fewer
probes per cross rank when the model is trained."""
import numpy as np
import pytest
import torch

import oracle
from helpers import dev, flush, host

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402
from paper_1202_6575_amd import learned  # noqa: E402

DTYPES = [np.int32, np.uint32, np.uint64, np.int64, np.float32, np.float64]


def rand_keys(g, N, alphabet, dtype):
    if dtype in (np.float32, np.float64):
        return (g.integers(-alphabet // 2, alphabet - alphabet // 2, size=N) * 0.375).astype(dtype)
    if dtype == np.int32:
        return g.integers(-alphabet // 2, alphabet - alphabet // 2, size=N).astype(np.int32)
    if dtype == np.int64:
        return (g.integers(0, alphabet, size=N).astype(np.uint64)
                * np.uint64((2 ** 64 - 1) // alphabet)).view(np.int64)
    if dtype == np.uint32:
        return (g.integers(0, alphabet, size=N) * ((2 ** 32 - 1) // alphabet)).astype(np.uint32)
    return g.integers(0, alphabet, size=N).astype(np.uint64) * np.uint64((2 ** 64 - 1) // alphabet)


def same_bits(a, b):
    return a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("dtype", DTYPES)
def test_sort_learned_equals_plain(dtype):
    g = np.random.default_rng(61)
    for N, alpha in [(1, 5), (513, 7), (70_001, 1 << 30), (300_007, 1000)]:
        keys = rand_keys(g, N, alpha, dtype)
        pay = np.arange(N, dtype=np.uint32)
        dk, dp = dev(keys), dev(pay)
        flush(f"sort learned {np.dtype(dtype).name} N={N} alpha={alpha}")
        if N >= 2:
            model, frac = learned.train_sort_model(dk, sample=1 << 16, samples=1 << 14, steps=200)
        else:
            model, frac = torch.zeros(learned.NPARAM, dtype=torch.float32, device=dk.device), 0.0
        lk, lp, cnt = learned.sort_learned(dk, model, frac, dp)
        pk, pp = sm.sort(dk, dp)
        torch.cuda.synchronize()
        assert same_bits(host(lk), host(pk))
        assert np.array_equal(host(lp), host(pp))
        if N <= 100_000:
            rk, rp = oracle.sort(keys, pay, 512)
            assert same_bits(host(lk), rk)
            assert np.array_equal(host(lp), rp)


def test_sort_learned_any_model():
    """A zero model, a random one and extreme step fractions: same bytes."""
    g = np.random.default_rng(62)
    keys = rand_keys(g, 200_003, 1 << 20, np.uint32)
    dk = dev(keys)
    pk, _ = sm.sort(dk)
    torch.cuda.synchronize()
    gen = torch.Generator(device="cpu").manual_seed(5)
    models = [torch.zeros(learned.NPARAM, dtype=torch.float32),
              torch.randn(learned.NPARAM, generator=gen, dtype=torch.float32),
              torch.full((learned.NPARAM,), 1e6, dtype=torch.float32)]
    for mi, mdl in enumerate(models):
        for frac in (0.0, 0.5, 1.0):
            flush(f"sort learned model={mi} frac={frac}")
            lk, _, _ = learned.sort_learned(dk, mdl.to(dk.device), frac, run=256)
            torch.cuda.synchronize()
            assert np.array_equal(host(lk), host(pk))


def test_sort_learned_fewer_probes():
    """Uniform keys at 2^22: a trained model's guesses need fewer probes per
    cross rank than searches that start from no information (a zero model
    with a step of the whole run, i.e. a bisection of the run)."""
    g = np.random.default_rng(63)
    keys = g.integers(0, 2 ** 32, size=1 << 22, dtype=np.uint64).astype(np.uint32)
    dk = dev(keys)
    flush("sort learned probes")
    model, frac = learned.train_sort_model(dk, sample=1 << 20, samples=1 << 18, steps=500)
    _, _, c_l = learned.sort_learned(dk, model, frac)
    zero = torch.zeros(learned.NPARAM, dtype=torch.float32, device=dk.device)
    _, _, c_z = learned.sort_learned(dk, zero, 1.0)
    torch.cuda.synchronize()
    sl, pl_ = (int(v) for v in host(c_l))
    sz, pz = (int(v) for v in host(c_z))
    assert sl == sz and sl > 0
    flush(f"probes per rank: learned {pl_ / sl:.2f}, uninformed {pz / sz:.2f}")
    assert pl_ / sl < 0.8 * (pz / sz)
