"""Seeded synthetic inputs generated on the GPU with torch (for benchmark
sizes where host generation would dominate).  Same recipes as the numpy
generators in this package; different random streams.  No merge arithmetic
here: sorting the inputs uses torch.sort."""
from __future__ import annotations

import math

import numpy as np
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed) & ((1 << 63) - 1))
    return g


def _sorted_runs(run_len, lo: int, hi: int, g, device):
    """Concatenated runs of the given lengths, each sorted, int32 keys
    uniform in [lo, hi)."""
    span = hi - lo
    bits = max(1, int(span - 1).bit_length())
    total = int(run_len.sum())
    keys = torch.randint(0, span, (total,), generator=g, device=device, dtype=torch.int64)
    run_id = torch.repeat_interleave(torch.arange(len(run_len), device=device), run_len)
    comp = torch.sort((run_id << bits) | keys).values
    return ((comp & ((1 << bits) - 1)) + lo).to(torch.int32)


def batched_pairs(n_k, m_k, lo: int, hi: int, seed: int, device="cuda:0",
                  chunk: int = 1 << 28):
    """int32 keys uniform in [lo, hi), laid out A_0 || B_0 || A_1 || B_1 ...
    with every A_k and B_k sorted.  Returns device tensors (keys, offsets[count+1],
    n_a[count]) (int32, int64, int64).  Pairs are generated in groups of about
    `chunk` elements, so totals far above 2^31 fit."""
    n_np = np.asarray(n_k, np.int64)
    m_np = np.asarray(m_k, np.int64)
    tot_np = n_np + m_np
    off_np = np.zeros(len(tot_np) + 1, dtype=np.int64)
    np.cumsum(tot_np, out=off_np[1:])
    total = int(off_np[-1])
    keys = torch.empty(total, dtype=torch.int32, device=device)
    g = _gen(seed, device)
    k0 = 0
    while k0 < len(tot_np):
        # pairs [k0, k1) with about `chunk` elements (at least one pair)
        k1 = int(np.searchsorted(off_np, off_np[k0] + chunk, side="right")) - 1
        k1 = min(max(k1, k0 + 1), len(tot_np))
        rl = np.stack([n_np[k0:k1], m_np[k0:k1]], 1).reshape(-1)
        keys[off_np[k0]:off_np[k1]] = _sorted_runs(torch.as_tensor(rl, device=device), lo, hi,
                                                   g, device)
        k0 = k1
    offsets = torch.as_tensor(off_np, device=device)
    return keys, offsets, torch.as_tensor(n_np, device=device)


def sort_input(N: int, key_hi: int, seed: int, device="cuda:0"):
    """Unsorted uint32 keys uniform in [0, key_hi) and payload = index."""
    k = torch.randint(0, key_hi, (N,), generator=_gen(seed, device), device=device,
                      dtype=torch.int64)
    keys = k.to(torch.int32).view(torch.uint32) if key_hi <= 2 ** 31 else \
        k.to(torch.uint32)
    pay = torch.arange(N, device=device, dtype=torch.int32).view(torch.uint32)
    return keys, pay


def lognormal_mixture(count: int, seed: int, medians_log2=(10, 20, 28), sigma=0.5,
                      device="cuda:0"):
    """Sorted uint32 keys: a component is picked uniformly, then
    key = floor(exp(ln(2^median) + sigma * N(0, 1))) clipped to [0, 2^32 - 1]
    (the recipe of the numpy generator, drawn on the GPU)."""
    g = _gen(seed, device)
    comp = torch.randint(0, len(medians_log2), (count,), generator=g, device=device)
    mu = torch.tensor([math.log(2.0) * v for v in medians_log2], dtype=torch.float64,
                      device=device)[comp]
    del comp
    x = torch.exp(mu + sigma * torch.randn(count, generator=g, device=device, dtype=torch.float64))
    del mu
    x = torch.clamp(torch.floor(x), 0, 2 ** 32 - 1).to(torch.int64)
    x = torch.sort(x).values
    # uint32 from the int64 values (two's complement wrap for values >= 2^31)
    return torch.where(x >= 2 ** 31, x - 2 ** 32, x).to(torch.int32).view(torch.uint32)
