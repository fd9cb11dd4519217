"""Shared test helpers: numpy <-> torch device transfer and input recipes."""
import numpy as np
import torch

NP2T = {np.dtype(np.int32): torch.int32, np.dtype(np.uint32): torch.uint32,
        np.dtype(np.uint64): torch.uint64}


def dev(a: np.ndarray) -> torch.Tensor:
    """Copy a numpy array to cuda:0 (keeps uint32/uint64)."""
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def flush(msg: str):
    print(msg, flush=True)


def rand_sorted(g, n, alphabet, dtype):
    """Sorted keys with heavy duplicates over an alphabet placed so that the
    signed / unsigned order matters (negative int32, values above 2^31 / 2^63)."""
    if dtype == np.int32:
        x = g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n).astype(np.int32)
    elif dtype == np.uint32:
        x = (g.integers(0, alphabet, size=n) * ((2 ** 32 - 1) // max(alphabet, 1))).astype(np.uint32)
    else:
        x = g.integers(0, alphabet, size=n).astype(np.uint64) * np.uint64((2 ** 64 - 1) // max(alphabet, 1))
    x.sort()
    return x
