"""The batched merge captured in a HIP graph: every replay, with other
eager work and synchronisations between replays, equals the eager result."""
import numpy as np
import pytest
import torch

import datagen
from helpers import dev, flush

pytestmark = pytest.mark.gpu

import paper_1202_6575_amd as sm  # noqa: E402


def test_batched_graph_replays():
    n_k, m_k = datagen.batch_lengths(500, 0, 14, seed=3)
    keys, offsets, n_a = datagen.batched_pairs(n_k, m_k, 0, 1 << 12, np.int32, seed=3)
    dk, do, dn = dev(keys), dev(offsets), dev(n_a)
    pay = dev(np.arange(len(keys), dtype=np.uint32))
    out = torch.empty_like(dk)
    opay = torch.empty_like(pay)
    ws = torch.empty(sm.batched_workspace_bytes(len(n_a), len(keys), torch.int32, True),
                     dtype=torch.uint8, device="cuda:0")
    sm.merge_batched(dk, do, dn, pay, out_keys=out, out_payloads=opay, workspace=ws)
    torch.cuda.synchronize()
    ref_k, ref_p = out.clone(), opay.clone()

    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            sm.merge_batched(dk, do, dn, pay, out_keys=out, out_payloads=opay, workspace=ws,
                             stream=side)
    torch.cuda.synchronize()
    other = dev(np.sort(np.random.default_rng(1).integers(0, 99, 30000)).astype(np.uint32))
    for r in range(4):
        flush(f"graph replay {r}")
        out.fill_(-1)
        opay.fill_(0)
        ws.fill_(0xAB)                   # the graph must not rely on leftover workspace
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref_k) and torch.equal(opay, ref_p), f"replay {r} differs"
        sm.merge(other, 10000, 20000)   # eager work between replays
        torch.cuda.synchronize()
