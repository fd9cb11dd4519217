"""Shared test helpers: numpy <-> torch device transfer and input recipes."""
import numpy as np
import torch

NP2T = {np.dtype(np.int32): torch.int32, np.dtype(np.uint32): torch.uint32,
        np.dtype(np.uint64): torch.uint64, np.dtype(np.int64): torch.int64,
        np.dtype(np.float32): torch.float32, np.dtype(np.float64): torch.float64}


def dev(a: np.ndarray) -> torch.Tensor:
    """Copy a numpy array to cuda:0 (keeps uint32/uint64)."""
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy()


def flush(msg: str):
    print(msg, flush=True)


def rand_sorted(g, n, alphabet, dtype):
    """Sorted keys with heavy duplicates over an alphabet placed so that the
    signed / unsigned order matters (negative int32 / int64, values above
    2^31 / 2^63); floats are negative and positive multiples of 0.75 (no NaN
    and no -0, so numpy's sort is the totalOrder sort)."""
    if dtype == np.int32:
        x = g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n).astype(np.int32)
    elif dtype == np.uint32:
        x = (g.integers(0, alphabet, size=n) * ((2 ** 32 - 1) // max(alphabet, 1))).astype(np.uint32)
    elif dtype == np.int64:
        # spread over the whole 64-bit range, read as signed: half the
        # alphabet is negative
        x = (g.integers(0, alphabet, size=n).astype(np.uint64)
             * np.uint64((2 ** 64 - 1) // max(alphabet, 1))).view(np.int64)
    elif dtype in (np.float32, np.float64):
        x = (g.integers(-alphabet // 2, alphabet - alphabet // 2, size=n) * 0.75).astype(dtype)
    else:
        x = g.integers(0, alphabet, size=n).astype(np.uint64) * np.uint64((2 ** 64 - 1) // max(alphabet, 1))
    x.sort()
    return x


def total_order_sequence(dt):
    """Bit patterns in ascending IEEE 754 totalOrder, built from the format's
    fields: -NaN (largest payload), -quiet NaN, -signaling NaN, -inf, -max,
    -1, -smallest normal, -largest and -smallest subnormal, -0, +0, then the
    same magnitudes ascending with a positive sign."""
    ut = np.uint32 if dt == np.float32 else np.uint64
    nb = 32 if dt == np.float32 else 64
    man = 23 if dt == np.float32 else 52
    sign = 1 << (nb - 1)
    exp_ones = ((1 << (nb - 1 - man)) - 1) << man
    quiet = 1 << (man - 1)
    one = int(np.array(1.0, dtype=dt).view(ut))
    mx = int(np.array(np.finfo(dt).max, dtype=dt).view(ut))
    tiny = int(np.array(np.finfo(dt).tiny, dtype=dt).view(ut))
    mags = [0, 1, (1 << man) - 1, tiny, one, mx, exp_ones, exp_ones | 1, exp_ones | quiet,
            exp_ones | ((1 << man) - 1)]
    neg = [sign | v for v in reversed(mags)]
    return np.array(neg + mags, dtype=ut).view(dt)
