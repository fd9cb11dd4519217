"""The autotuner: every tile candidate gives the oracle's bytes, the tuned
choice round-trips through the cache file, and the package's batched merge
picks it up when it leaves the tile to the library."""
import json

import numpy as np
import pytest
import torch

import datagen
import oracle
from helpers import dev, flush, host, rand_sorted

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402
from paper_1202_6575_amd import autotune  # noqa: E402


def make_batch(g, count, log2max, dtype):
    n_k, m_k = datagen.batch_lengths(count, 0, log2max, seed=int(g.integers(1 << 30)))
    parts, offsets, n_a = [], [0], []
    for n, m in zip(n_k, m_k):
        parts += [rand_sorted(g, int(n), 300, dtype), rand_sorted(g, int(m), 300, dtype)]
        offsets.append(offsets[-1] + int(n) + int(m))
        n_a.append(int(n))
    return np.concatenate(parts), np.array(offsets, np.int64), np.array(n_a, np.int64)


def test_tuned_tile_round_trip(tmp_path, monkeypatch):
    g = np.random.default_rng(77)
    keys, offsets, n_a = make_batch(g, 400, 13, np.int32)
    total = len(keys)
    ref, _ = oracle.merge_batched(keys, offsets, n_a)
    dk, do, dn = dev(keys), dev(offsets), dev(n_a)
    out = torch.empty_like(dk)

    def run(tile):
        sm.merge_batched(dk, do, dn, out_keys=out, tile=tile)

    cands = (512, 1152, 2368, 4096)
    for tile in cands:
        flush(f"autotune candidate tile={tile}")
        out.fill_(-1)
        run(tile)
        torch.cuda.synchronize()
        assert np.array_equal(host(out), ref), f"tile={tile}"

    path = str(tmp_path / "tune.json")
    best, ms = autotune.tune("batched", run, torch.int32, False, total, cands=cands, reps=3,
                             path=path)
    assert best in cands and set(ms) == set(cands)
    with open(path) as f:
        stored = json.load(f)
    key = autotune.cache_key("batched", torch.int32, False, total)
    assert stored[key]["tile"] == best
    # a second tune reads the cache instead of timing again
    again, ms2 = autotune.tune("batched", lambda t: pytest.fail("timed again"), torch.int32,
                               False, total, path=path)
    assert again == best and set(ms2) == set(ms)
    assert autotune.lookup("batched", torch.int32, False, total, path=path) == best
    # the package's call leaves the tile to the library: the cached choice
    monkeypatch.setenv("SM_AUTOTUNE_CACHE", path)
    assert sm._tuned("batched", dk, False, total) == best
    assert sm._tuned("batched", dk, True, total) == 0          # another class: the default
    out.fill_(-1)
    ck, _ = sm.merge_batched(dk, do, dn, out_keys=out)
    torch.cuda.synchronize()
    assert np.array_equal(host(ck), ref)
