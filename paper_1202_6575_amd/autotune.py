"""Autotuner for the merge launch parameters.

The one free launch parameter of the merge kernels is the block length
``tile``: a subproblem holds up to 2 * tile elements, so with 256 lanes per
workgroup each lane merges about 2 * tile / 256 items (items per lane 4 ..
32 for tile 512 .. 4096), and the LDS a workgroup stages (hence how many
workgroups share a compute unit) grows with it.  The output never depends on
the choice: a stable merge is unique.

``tune`` times every candidate on the caller's own data (HIP events on the
current stream, median of several runs), returns the fastest, and caches
the choice per (operation, key type, payload, size class, device) in a JSON
file (``SM_AUTOTUNE_CACHE``, default ``~/.cache/paper_1202_6575_amd/autotune.json``).
"""
from __future__ import annotations

import json
import math
import os
import statistics

import torch

TILES = (512, 1024, 1152, 1536, 2048, 2368, 3072, 4096)


def cache_path() -> str:
    return os.environ.get("SM_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1202_6575_amd",
                                       "autotune.json"))


def cache_key(op: str, dtype: torch.dtype, has_payload: bool, size: int) -> str:
    """Size class: the power of two of the element count."""
    cls = int(math.log2(max(size, 1)))
    dev = torch.cuda.get_device_name(0).replace(" ", "_")
    return f"{op}/{str(dtype).replace('torch.', '')}/{'pay' if has_payload else 'keys'}/2^{cls}/{dev}"


def _load(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def time_ms(fn, reps: int = 5, warmup: int = 1) -> float:
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        fn()
    ts = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return statistics.median(ts)


def tune(op: str, run, dtype: torch.dtype, has_payload: bool, size: int, candidates=None,
         valid=None, reps: int = 5, use_cache: bool = True, path: str | None = None):
    """Returns (best_tile, {tile: ms}).  run(tile) launches the operation once;
    valid(tile) filters candidates (e.g. by the library's workspace query,
    which returns 0 for a tile whose subproblems do not fit LDS)."""
    path = path or cache_path()
    key = cache_key(op, dtype, has_payload, size)
    cache = _load(path) if use_cache else {}
    if use_cache and key in cache:
        return int(cache[key]["tile"]), {int(k): v for k, v in cache[key]["ms"].items()}
    cands = [t for t in (candidates or TILES) if valid is None or valid(t)]
    if not cands:
        raise ValueError("no valid tile candidates")
    ms = {t: time_ms(lambda: run(t), reps=reps) for t in cands}
    best = min(ms, key=ms.get)
    if use_cache:
        cache = _load(path)
        cache[key] = {"tile": best, "ms": {str(k): v for k, v in ms.items()}}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, path)
    return best, ms
