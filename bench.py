#!/usr/bin/env python3
"""Benchmark: stable parallel merge on one MI355X (gfx950).

Workload (default): the large plain merge, n = m = 2^28 uint32 keys drawn
uniformly over the full 32-bit range and sorted, keys only.  One step is one
pass of the whole plain path over the resident input: Steps 1-2 (partition
kernel, cross ranks of the block starts) and Steps 3-4 (merge kernel: the
five cases, LDS staging, lane-level split, per-lane merges, write-back).

Prints ONE JSON line.  ``value`` is whole-job throughput in Gelem/s,
(n + m) / (wall time per step), with inputs resident in HBM.  ``roofline``
prices the merge kernel (the dominant kernel) against the 8 TB/s HBM peak:
algorithmic bytes per launch = (n + m) * 2 * (key bytes + payload bytes)
(every element read once and written once), divided by the kernel's mean
duration from HIP events recorded on the launch stream around it.
``cpu_baseline`` times the CPU oracle's sequential two-pointer merge on the
same arrays (one host thread).

``copy_reference`` is a plain elementwise stream over the same bytes
(bitwise NOT of the keys as int32: read 4 B, write 4 B per element), timed
the same way; it is the achievable-bandwidth context for the roofline, and
its rocprofv3 counters calibrate the merge kernel's FETCH_SIZE / WRITE_SIZE.

``python bench.py --summarize-pmc FETCH_DIR WRITE_DIR`` reads two
``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` output directories of
this benchmark (csv format) and writes the per-launch HBM traffic of the
merge kernel, scaled by the copy kernel's counters, to the profiles folder.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PMC_FILE = os.path.join(ROOT, "profiles", "merge_kernel_uniform2x2e28_u32_pmc.json")
KERNEL_SOURCES = ["paper_1202_6575_amd/csrc/sm_device.h", "paper_1202_6575_amd/csrc/sm_merge.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(launch_bytes_alg: float):
    """HBM bytes per launch from committed rocprofv3 --pmc counters, if they
    were taken on the current kernel source; else None."""
    if not os.path.exists(PMC_FILE):
        return None
    with open(PMC_FILE) as f:
        pmc = json.load(f)
    if pmc.get("source_hash") != kernel_source_hash():
        return None
    return pmc.get("hbm_bytes_per_launch")


MERGE_KERNEL_TAG = "merge_persistent_kernel"
COPY_KERNEL_TAG = "bitwise_not"


def _pmc_per_dispatch(run_dir: str, counter: str):
    """Mean counter value per dispatch for the merge and the copy kernel."""
    import csv
    import glob
    vals = {"merge": [], "copy": []}
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"]
            key = "merge" if MERGE_KERNEL_TAG in name else ("copy" if COPY_KERNEL_TAG in name else None)
            if key:
                vals[key].append(float(r["Counter_Value"]))
    return {k: (sum(v) / len(v) if v else None) for k, v in vals.items()}


def summarize_pmc(fetch_dir: str, write_dir: str, log2n: int, out_path: str = PMC_FILE):
    n = m = 1 << log2n
    stream_bytes = (n + m) * 4           # the copy reads this many bytes and writes as many
    f = _pmc_per_dispatch(fetch_dir, "FETCH_SIZE")
    w = _pmc_per_dispatch(write_dir, "WRITE_SIZE")
    if None in (f["merge"], f["copy"], w["merge"], w["copy"]):
        raise SystemExit(f"missing counters: fetch={f} write={w}")
    # counters are in KiB per dispatch; scale each by what it reads for the copy
    sf = stream_bytes / (f["copy"] * 1024.0)
    sw = stream_bytes / (w["copy"] * 1024.0)
    fetch_b = f["merge"] * 1024.0 * sf
    write_b = w["merge"] * 1024.0 * sw
    out = {"kernel": "merge_persistent_kernel<uint32, keys only>",
           "workload": f"n=m=2^{log2n} uint32 uniform, keys only",
           "source_hash": kernel_source_hash(),
           "fetch_kib_per_dispatch": f["merge"], "write_kib_per_dispatch": w["merge"],
           "copy_fetch_kib_per_dispatch": f["copy"], "copy_write_kib_per_dispatch": w["copy"],
           "copy_stream_bytes": stream_bytes, "fetch_scale": sf, "write_scale": sw,
           "hbm_bytes_per_launch": fetch_b + write_b,
           "algorithmic_bytes_per_launch": (n + m) * 2 * 4}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=28, help="n = m = 2^log2n")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true", help="compare one output with the oracle")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--pmc-out", default=PMC_FILE)
    args = ap.parse_args()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.log2n, args.pmc_out)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark measures one GPU only; the merge is not "
                                   "sharded across GPUs",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1202_6575_amd as sm

    n = m = 1 << args.log2n
    log(f"bench: generating n=m=2^{args.log2n} uint32 uniform keys")
    A, B = datagen.uniform_pair(n, m, 0, 2 ** 32, np.uint32, seed=datagen.BASE_SEED + 1)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(np.concatenate([A, B])).to(dev)
    out = torch.empty(n + m, dtype=torch.uint32, device=dev)
    tile = args.tile or 2048
    p_a = (n + tile - 1) // tile
    p_b = (m + tile - 1) // tile
    xbar = torch.empty(p_a + 1, dtype=torch.int64, device=dev)
    ybar = torch.empty(p_b + 1, dtype=torch.int64, device=dev)
    ws = torch.empty(sm.pieces_workspace_bytes(n, m, p_a, p_b, torch.uint32), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        sm.partition(keys, n, m, p_a, p_b, xbar=xbar, ybar=ybar, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        sm.merge_pieces(keys, n, m, p_a, p_b, xbar, ybar, out_keys=out, workspace=ws,
                        stream=stream)
        if ev is not None:
            ev[2].record(stream)

    log("bench: copy reference")
    src32, dst32 = keys.view(torch.int32), out.view(torch.int32)
    torch.bitwise_not(src32, out=dst32)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(3):
        torch.bitwise_not(src32, out=dst32)
    c1.record(stream)
    torch.cuda.synchronize()
    copy_ms = c0.elapsed_time(c1) / 3

    log("bench: warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    log(f"bench: timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    part_ms = [e[0].elapsed_time(e[1]) for e in evs]
    merge_ms = [e[1].elapsed_time(e[2]) for e in evs]
    ms_per_step = wall * 1e3 / args.steps
    gelems = (n + m) / (ms_per_step * 1e-3) / 1e9
    merge_avg_ms = float(np.mean(merge_ms))
    alg_bytes = (n + m) * 2 * 4
    achieved = alg_bytes / (merge_avg_ms * 1e-3) / 1e9

    if args.check:
        log("bench: checking against the oracle")
        import oracle
        ref, _ = oracle.merge(A, B)
        assert np.array_equal(out.cpu().numpy(), ref), "merge output differs from the oracle"

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        log("bench: timing the CPU oracle (sequential two-pointer merge, 1 thread)")
        t = time.perf_counter()
        oracle.merge(A, B)
        dt = time.perf_counter() - t
        cpu = {"value": round((n + m) / dt / 1e9, 4), "unit": "Gelem/s", "cores": 1,
               "kind": "oracle",
               "sample": f"the full workload once: oracle two-pointer merge of the same "
                         f"n=m=2^{args.log2n} uint32 arrays in host memory, {dt:.2f} s"}

    res = {
        "metric": "stable-merge Gelem/s (plain merge, n=m=2^28 uint32 keys)",
        "value": round(gelems, 2),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"large plain merge: n=m=2^{args.log2n} uint32 uniform over "
                               f"[0, 2^32), sorted, keys only",
                   "n": n, "m": m, "tile": tile, "p_a": p_a, "p_b": p_b,
                   "parallelism": "single GPU"},
        "phases_ms": {"partition (Steps 1-2)": round(float(np.mean(part_ms)), 4),
                      "cases + merge (Steps 3-4)": round(merge_avg_ms, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic_from_profile(alg_bytes),
                     "kernel": "merge_kernel<uint32, keys only>",
                     "algorithmic_bytes_per_launch": alg_bytes},
        "cpu_baseline": cpu,
        "copy_reference": {"GB/s": round(alg_bytes / (copy_ms * 1e-3) / 1e9, 1),
                           "ms": round(copy_ms, 4),
                           "kernel": "elementwise bitwise_not, reads and writes n+m uint32"},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
