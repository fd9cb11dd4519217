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


def batched_pairs(n_k, m_k, lo: int, hi: int, seed: int, device="cuda:0"):
    """int32 keys uniform in [lo, hi), laid out A_0 || B_0 || A_1 || B_1 ...
    with every A_k and B_k sorted.  Returns device tensors (keys, offsets[count+1],
    n_a[count]) (int32, int64, int64)."""
    n_k = torch.as_tensor(np.asarray(n_k, np.int64), device=device)
    m_k = torch.as_tensor(np.asarray(m_k, np.int64), device=device)
    tot = n_k + m_k
    offsets = torch.zeros(len(tot) + 1, dtype=torch.int64, device=device)
    torch.cumsum(tot, 0, out=offsets[1:])
    total = int(offsets[-1])
    span = hi - lo
    bits = max(1, int(span - 1).bit_length())
    keys = torch.randint(0, span, (total,), generator=_gen(seed, device), device=device,
                         dtype=torch.int64)
    run_len = torch.stack([n_k, m_k], 1).reshape(-1)
    run_id = torch.repeat_interleave(torch.arange(len(run_len), device=device), run_len)
    comp = torch.sort((run_id << bits) | keys).values
    keys = ((comp & ((1 << bits) - 1)) + lo).to(torch.int32)
    return keys, offsets, n_k.clone()


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
