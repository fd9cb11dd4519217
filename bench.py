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
TRACE_FILE = os.path.join(ROOT, "profiles", "merge_kernel_uniform2x2e28_u32_trace.json")
KERNEL_SOURCES = ["paper_1202_6575_amd/csrc/sm_device.h", "paper_1202_6575_amd/csrc/sm_merge.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_info() -> dict:
    """CPU model and core counts of the host the benchmark runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cores": usable}


def cpu_threads() -> int:
    """Worker threads for the multi-threaded oracle baselines: the cores this
    process may run on, at most 16 (one GPU's share of its host)."""
    return max(1, min(16, host_info()["usable_cores"]))


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


def trace_from_profile():
    """Steady-state merge-kernel duration from a committed rocprofv3 kernel
    trace of this benchmark, if it was taken on the current kernel source."""
    if not os.path.exists(TRACE_FILE):
        return None
    with open(TRACE_FILE) as f:
        tr = json.load(f)
    if tr.get("source_hash") != kernel_source_hash():
        return None
    return tr


def trace_summary(alg_bytes: float):
    tr = trace_from_profile()
    if tr is None:
        return None
    return {"source": os.path.relpath(TRACE_FILE, ROOT),
            "steady_mean_ms": tr["steady_mean_ms"], "steady_dispatches": tr["steady_dispatches"],
            "frac": round(alg_bytes / (tr["steady_mean_ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


MERGE_KERNEL_TAG = "merge_pipelined_kernel"
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


def _pmc_by_kernel(run_dir: str, counter: str):
    """{kernel name (template arguments kept, parameters dropped): (mean
    KiB per dispatch, dispatches)} for one counter."""
    import csv
    import glob
    acc = {}
    for f in glob.glob(os.path.join(run_dir, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            name = r["Kernel_Name"].replace("(anonymous namespace)::", "").split("(")[0]
            name = name.replace("void ", "")
            v = acc.setdefault(name, [0.0, 0])
            v[0] += float(r["Counter_Value"])
            v[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def summarize_trace(trace_dir: str, warmup: int, out_path: str = TRACE_FILE):
    """Per-dispatch durations of the merge kernel from a rocprofv3
    --kernel-trace (csv) of this benchmark: the first `warmup` dispatches
    (the untimed warm-up steps) are listed apart, the rest summarised."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            if MERGE_KERNEL_TAG in r["Kernel_Name"]:
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    rows.sort()
    if len(rows) <= warmup:
        raise SystemExit(f"{len(rows)} merge dispatches, warm-up {warmup}")
    ms = [d * 1e-6 for _, d in rows]
    steady = sorted(ms[warmup:])
    out = {"kernel": "merge_pipelined_kernel<uint32, keys only>",
           "source_hash": kernel_source_hash(),
           "warmup_dispatches_ms": [round(x, 4) for x in ms[:warmup]],
           "steady_dispatches": len(steady),
           "steady_mean_ms": round(sum(steady) / len(steady), 4),
           "steady_median_ms": round(steady[len(steady) // 2], 4),
           "steady_min_ms": round(steady[0], 4), "steady_max_ms": round(steady[-1], 4)}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out))


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
    out = {"kernel": "merge_pipelined_kernel<uint32, keys only>",
           "workload": f"n=m=2^{log2n} uint32 uniform, keys only",
           "source_hash": kernel_source_hash(),
           "fetch_kib_per_dispatch": f["merge"], "write_kib_per_dispatch": w["merge"],
           "copy_fetch_kib_per_dispatch": f["copy"], "copy_write_kib_per_dispatch": w["copy"],
           "copy_stream_bytes": stream_bytes, "fetch_scale": sf, "write_scale": sw,
           "hbm_bytes_per_launch": fetch_b + write_b,
           "algorithmic_bytes_per_launch": (n + m) * 2 * 4}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    # every kernel of the run: mean counters per dispatch, scaled alike
    fa = _pmc_by_kernel(fetch_dir, "FETCH_SIZE")
    wa = _pmc_by_kernel(write_dir, "WRITE_SIZE")
    table = {}
    for name in sorted(set(fa) | set(wa)):
        fk, fn = fa.get(name, (None, 0))
        wk, wn = wa.get(name, (None, 0))
        table[name] = {"dispatches": max(fn, wn),
                       "fetch_bytes_per_dispatch": None if fk is None else fk * 1024.0 * sf,
                       "write_bytes_per_dispatch": None if wk is None else wk * 1024.0 * sw}
    all_path = os.path.join(os.path.dirname(out_path), "library_kernels_pmc.json")
    with open(all_path, "w") as fh:
        json.dump({"source_hash": kernel_source_hash(), "fetch_scale": sf, "write_scale": sw,
                   "kernels": table}, fh, indent=1)
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--log2n", type=int, default=28, help="n = m = 2^log2n")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check", action="store_true", help="compare one output with the oracle")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched, sort and learned measurements")
    ap.add_argument("--extras",
                    default="heavy_ties,skewed,batched,batched_literal,sort,sort_learned,"
                            "learned,descending",
                    help="comma-separated subset of heavy_ties, skewed, batched, "
                         "batched_literal, sort, sort_learned (the sort with one learned "
                         "model; needs sort), learned, descending")
    ap.add_argument("--sort-run", type=int, default=512, help="run length of the merge sort")
    ap.add_argument("--batch-log2max", type=int, default=15,
                    help="batched pairs: totals log-uniform in [16, 2^this]")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--pmc-out", default=PMC_FILE)
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR")
    ap.add_argument("--trace-out", default=TRACE_FILE)
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.warmup, args.trace_out)
        return
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
    tile = args.tile or 2368      # the library's default block length for 32-bit keys
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
               "kind": "oracle", "host": host_info(),
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
                     "kernel": "merge_pipelined_kernel<uint32, keys only>",
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "timing": "HIP events on the launch stream around stable_merge_pieces "
                               "(the cases kernel, about 5 us, then the merge kernel), mean "
                               "over the timed steps",
                     "frac_whole_step": round(alg_bytes / (ms_per_step * 1e-3) / 1e9
                                              / HBM_PEAK_GBS, 4),
                     "trace": trace_summary(alg_bytes)},
        "cpu_baseline": cpu,
        "copy_reference": {"GB/s": round(alg_bytes / (copy_ms * 1e-3) / 1e9, 1),
                           "ms": round(copy_ms, 4),
                           "kernel": "elementwise bitwise_not, reads and writes n+m uint32"},
    }
    if not args.no_extras:
        del keys, out, ws, xbar, ybar, A, B
        torch.cuda.empty_cache()
        extras = set(args.extras.split(","))
        if "heavy_ties" in extras:
            res["heavy_ties"] = bench_heavy_ties(args)
            log(f"bench: heavy_ties {json.dumps(res['heavy_ties'])}")
            torch.cuda.empty_cache()
        if "skewed" in extras:
            res["skewed"] = bench_skewed(args)
            log(f"bench: skewed {json.dumps(res['skewed'])}")
            torch.cuda.empty_cache()
        if "batched" in extras:
            res["batched"] = bench_batched(args, gelems, args.batch_log2max)
            log(f"bench: batched {json.dumps(res['batched'])}")
            torch.cuda.empty_cache()
        if "batched_literal" in extras:
            # pair totals log-uniform up to 2^20: about 6.2e9 elements
            res["batched_literal"] = bench_batched(args, gelems, 20)
            log(f"bench: batched_literal {json.dumps(res['batched_literal'])}")
            torch.cuda.empty_cache()
        if "sort" in extras:
            res["sort"] = bench_sort(args, "sort_learned" in extras)
            log(f"bench: sort {json.dumps(res['sort'])}")
            torch.cuda.empty_cache()
        if "learned" in extras:
            res["learned"] = bench_learned(args)
            log(f"bench: learned {json.dumps(res['learned'])}")
            torch.cuda.empty_cache()
        if "descending" in extras:
            res["descending"] = bench_descending(args)
            log(f"bench: descending {json.dumps(res['descending'])}")
    print(json.dumps(res), flush=True)


def _events_ms(fn, steps, stream):
    """Mean ms of fn() over `steps` runs, HIP events on `stream`."""
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    for _ in range(steps):
        fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / steps


def bench_batched(args, plain_gelems, log2max):
    """65,536 independent pairs, totals L_k log-uniform in [16, 2^log2max]
    (2^15: about 2^28 int32 keys; 2^20, the literal recipe: about 6.2e9),
    keys uniform in [0, 2^20), keys only: the batched merge captured in one
    graph, the tile chosen by the autotuner, against one stable_merge call
    per pair on a sample of pairs."""
    import numpy as np
    import torch
    import datagen
    import datagen.torch_gen as tg
    import paper_1202_6575_amd as sm
    from paper_1202_6575_amd import autotune

    count = 65536
    log(f"bench: batched merge, {count} pairs, totals in [16, 2^{log2max}]")
    n_k, m_k = datagen.batch_lengths(count, 4, log2max, seed=datagen.BASE_SEED + 4)
    keys, offsets, n_a = tg.batched_pairs(n_k, m_k, 0, 1 << 20, seed=datagen.BASE_SEED + 4)
    total = keys.numel()
    out = torch.empty_like(keys)
    stream = torch.cuda.current_stream()

    def valid(t):
        return sm.batched_workspace_bytes(count, total, torch.int32, False, tile=t) > 0

    wss = {}

    def run(t):
        if t not in wss:
            wss[t] = torch.empty(sm.batched_workspace_bytes(count, total, torch.int32, False, tile=t),
                                 dtype=torch.uint8, device=keys.device)
        sm.merge_batched(keys, offsets, n_a, out_keys=out, tile=t, workspace=wss[t],
                         stream=stream)

    tile, tune_ms = autotune.tune("batched", run, torch.int32, False, total, valid=valid,
                                  use_cache=False)
    default_ms = tune_ms.get(2368)
    ws = wss[tile]
    for t in list(wss):
        if t != tile:
            del wss[t]
    run(tile)
    torch.cuda.synchronize()
    eager_out = out.clone()
    # one graph holds the whole launch sequence of the batched merge
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            sm.merge_batched(keys, offsets, n_a, out_keys=out, tile=tile, workspace=ws,
                             stream=side)
    torch.cuda.synchronize()
    out.zero_()
    g.replay()
    torch.cuda.synchronize()
    graph_ok = bool(torch.equal(out, eager_out))
    steps = max(5, args.steps)
    for _ in range(2):
        g.replay()
    graph_ms = _events_ms(g.replay, steps, stream)
    eager_ms = _events_ms(lambda: run(tile), steps, stream)
    gel = total / (graph_ms * 1e-3) / 1e9
    alg = total * 2 * 4

    # one stable_merge call per pair, on a sample of pairs copied to 16-byte
    # aligned slots (the library requires aligned arrays)
    g_np = np.random.default_rng(7)
    sample = np.sort(g_np.choice(count, 2048, replace=False))
    off_h = offsets.cpu().numpy()
    na_h = n_a.cpu().numpy()
    lens = off_h[sample + 1] - off_h[sample]
    slots = np.zeros(len(sample) + 1, np.int64)
    np.cumsum((lens + 3) // 4 * 4, out=slots[1:])
    packed = torch.empty(int(slots[-1]), dtype=torch.int32, device=keys.device)
    for i, k in enumerate(sample):
        packed[slots[i]:slots[i] + lens[i]] = keys[off_h[k]:off_h[k + 1]]
    pout = torch.empty_like(packed)
    pws = torch.empty(max(sm.workspace_bytes(int(na_h[k]), int(L - na_h[k]), torch.int32)
                          for k, L in zip(sample, lens)),
                      dtype=torch.uint8, device=keys.device)
    views = [(packed[slots[i]:slots[i] + lens[i]], int(na_h[k]), int(lens[i] - na_h[k]),
              pout[slots[i]:slots[i] + lens[i]]) for i, k in enumerate(sample)]

    def per_pair():
        for kv, na, mb, ov in views:
            sm.merge(kv, na, mb, out_keys=ov, workspace=pws, stream=stream)

    per_pair()
    pp_ms = _events_ms(per_pair, 2, stream)
    pp_gel = float(lens.sum()) / (pp_ms * 1e-3) / 1e9
    cpu = None if args.no_cpu_baseline else batched_cpu_baseline(keys, off_h, na_h)
    return {"workload": f"{count} pairs, L_k = floor(2^U), U ~ U[4, {log2max}], "
                        f"m_k = floor(f L_k), int32 keys uniform in [0, 2^20), keys only",
            "total_elements": total, "Gelem/s": round(gel, 2), "ms": round(graph_ms, 4),
            "eager_ms": round(eager_ms, 4), "graph_launches_per_step": 1,
            "graph_replay_matches_eager": graph_ok,
            "autotune": {"tile": tile, "items_per_lane": 2 * tile // 256,
                         "ms_tuned": round(tune_ms[tile], 4),
                         "ms_default_tile_2368": None if default_ms is None else round(default_ms, 4),
                         "ms_by_tile": {str(t): round(v, 4) for t, v in tune_ms.items()}},
            "roofline": {"bound": "hbm", "achieved": round(alg / (graph_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(alg / (graph_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)},
            "per_pair_calls": {"pairs_sampled": len(sample), "Gelem/s": round(pp_gel, 3),
                               "speedup_of_batched": round(gel / pp_gel, 1)},
            "cpu_baseline": cpu,
            "vs_plain_merge_Gelem/s": round(gel / plain_gelems, 3)}


def batched_cpu_baseline(keys, off_h, na_h, budget: int = 1 << 28):
    """The oracle's batched merge (its two-pointer merge applied pair by
    pair, in C) on the leading pairs of the batch (pairs are drawn
    independently, so a prefix is a sample of the whole), at most `budget`
    elements, split into contiguous ranges of pairs over host threads (the
    oracle's C routine runs without Python's lock)."""
    import concurrent.futures
    import numpy as np
    import oracle
    k = int(np.searchsorted(off_h, budget, side="right")) - 1
    k = max(1, min(k, len(na_h)))
    elems = int(off_h[k])
    host = keys[:elems].cpu().numpy()
    out = np.empty_like(host)
    offs = np.ascontiguousarray(off_h[:k + 1], dtype=np.int64)
    nas = np.ascontiguousarray(na_h[:k], dtype=np.int64)
    threads = cpu_threads()
    # contiguous pair ranges of about equal element counts
    cuts = np.searchsorted(offs, np.linspace(0, elems, threads + 1)).astype(np.int64)
    cuts[0], cuts[-1] = 0, k
    ranges = [(int(a), int(b)) for a, b in zip(cuts[:-1], cuts[1:]) if b > a]
    oracle.merge_batched(host, offs, nas, pairs=(0, min(k, 8)), out=out)
    t = time.perf_counter()
    with concurrent.futures.ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(lambda r: oracle.merge_batched(host, offs, nas, pairs=r, out=out), ranges))
    dt = time.perf_counter() - t
    return {"value": round(elems / dt / 1e9, 4), "unit": "Gelem/s", "cores": threads,
            "kind": "oracle", "host": host_info(),
            "sample": f"the first {k} pairs of the batch ({elems} elements): the oracle's "
                      f"batched two-pointer merge, contiguous pair ranges on {threads} host "
                      f"threads, {dt:.2f} s"}


def bench_heavy_ties(args):
    """A = 1,000,000 and B = 600,000 int32 keys uniform in [0, 65536) (about
    15 and 9 copies of every value), payload = source tag << 31 | index,
    p_a = p_b = 256 forced: the whole stable_merge call's latency.  The
    inputs (25.6 MB in and out) stay in the last-level cache, so latency,
    not HBM bandwidth, is the figure."""
    import numpy as np
    import torch
    import datagen
    import paper_1202_6575_amd as sm

    n, m = 1_000_000, 600_000
    log("bench: heavy ties, n=1e6, m=6e5 int32, p=256")
    A, B = datagen.uniform_pair(n, m, 0, 65536, np.int32, seed=datagen.BASE_SEED + 0)
    pa, pb = datagen.source_tag_payloads(n, m)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(np.concatenate([A, B])).to(dev)
    pay = torch.from_numpy(np.concatenate([pa, pb])).to(dev)
    ok, op = torch.empty_like(keys), torch.empty_like(pay)
    ws = torch.empty(sm.workspace_bytes(n, m, torch.int32, True, p_a=256, p_b=256),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def run():
        sm.merge(keys, n, m, pay, out_keys=ok, out_payloads=op, p_a=256, p_b=256,
                 workspace=ws, stream=stream)

    for _ in range(3):
        run()
    times = []
    for _ in range(max(args.steps, 20)):
        times.append(_events_ms(run, 1, stream))
    med = float(np.median(times))
    return {"workload": "A 1e6 and B 6e5 int32 uniform in [0, 65536), payload src<<31|index, "
                        "p_a = p_b = 256",
            "latency_us_median": round(med * 1e3, 1),
            "latency_us_min": round(min(times) * 1e3, 1),
            "Gelem/s": round((n + m) / (med * 1e-3) / 1e9, 2)}


def bench_skewed(args):
    """A = 2^27 and B = 2^23 uint64 keys, Zipf(1.1) over 10^6 distinct
    values, uint32 payload = index in A ‖ B: Gelem/s, the partition / merge
    split, the merge kernel's HBM roofline, and the sizes of the p_a + p_b
    subproblems (load balance under massive ties and m << n)."""
    import numpy as np
    import torch
    import datagen
    import paper_1202_6575_amd as sm

    n, m = 1 << 27, 1 << 23
    log("bench: skewed, n=2^27, m=2^23 uint64 Zipf(1.1) with payloads")
    A, B = datagen.zipf_pair(n, m, 1.1, 10 ** 6, seed=datagen.BASE_SEED + 2)
    dev = torch.device("cuda:0")
    keys = torch.from_numpy(np.concatenate([A, B]).view(np.int64)).to(dev).view(torch.uint64)
    del A, B
    pay = torch.arange(n + m, dtype=torch.int64, device=dev).to(torch.int32).view(torch.uint32)
    ok, op = torch.empty_like(keys), torch.empty_like(pay)
    tile = 1024                          # the library's default block length for uint64 + payload
    p_a, p_b = (n + tile - 1) // tile, (m + tile - 1) // tile
    xbar = torch.empty(p_a + 1, dtype=torch.int64, device=dev)
    ybar = torch.empty(p_b + 1, dtype=torch.int64, device=dev)
    ws = torch.empty(sm.pieces_workspace_bytes(n, m, p_a, p_b, torch.uint64, True),
                     dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    def part():
        sm.partition(keys, n, m, p_a, p_b, xbar=xbar, ybar=ybar, stream=stream)

    def pieces():
        sm.merge_pieces(keys, n, m, p_a, p_b, xbar, ybar, pay, out_keys=ok, out_payloads=op,
                        workspace=ws, stream=stream)

    part()
    pieces()
    torch.cuda.synchronize()
    steps = max(args.steps, 5)
    part_ms = _events_ms(part, steps, stream)
    merge_ms = _events_ms(pieces, steps, stream)
    alg = (n + m) * (8 + 4) * 2
    # subproblem sizes: the 2p pieces tile C in the order of their output
    # offsets x_i + xbar_i and y_j + ybar_j
    def starts(length, p):
        i = torch.arange(p, dtype=torch.int64, device=dev)
        q, r = length // p, length % p
        return i * q + torch.minimum(i, torch.tensor(r, device=dev))
    c = torch.cat([starts(n, p_a) + xbar[:p_a], starts(m, p_b) + ybar[:p_b],
                   torch.tensor([n + m], dtype=torch.int64, device=dev)])
    sizes = torch.diff(torch.sort(c).values)
    hist = torch.bincount(torch.floor(torch.log2(sizes.double() + 1)).long()).cpu().tolist()
    sz = sizes.double()
    return {"workload": "A 2^27 and B 2^23 uint64, Zipf(1.1) over 10^6 distinct values, "
                        "uint32 payload = index in A||B",
            "tile": tile, "p_a": p_a, "p_b": p_b,
            "Gelem/s": round((n + m) / ((part_ms + merge_ms) * 1e-3) / 1e9, 2),
            "phases_ms": {"partition (Steps 1-2)": round(part_ms, 4),
                          "cases + merge (Steps 3-4)": round(merge_ms, 4)},
            "roofline": {"bound": "hbm", "achieved": round(alg / (merge_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(alg / (merge_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes_per_launch": alg},
            "subproblem_sizes": {"count": int(sizes.numel()), "mean": round(float(sz.mean()), 1),
                                 "max": int(sizes.max()), "bound_2_blocks": 2 * tile,
                                 "p99": int(torch.quantile(sz, 0.99)),
                                 "log2_histogram": {f"[{(1 << k) - 1},{(1 << (k + 1)) - 1})": v
                                                    for k, v in enumerate(hist) if v}}}


def bench_descending(args):
    """The whole stable_merge call on the large plain merge's shape, ascending
    and descending (the same keys reversed): the cost of the two extra
    passes of the order transform."""
    import numpy as np
    import torch
    import datagen
    import paper_1202_6575_amd as sm

    n = m = 1 << args.log2n
    log(f"bench: descending, n=m=2^{args.log2n} uint32")
    A, B = datagen.uniform_pair(n, m, 0, 2 ** 32, np.uint32, seed=datagen.BASE_SEED + 1)
    dev = torch.device("cuda:0")
    asc = torch.from_numpy(np.concatenate([A, B])).to(dev)
    desc = torch.from_numpy(np.concatenate([A[::-1], B[::-1]])).to(dev)
    del A, B
    out = torch.empty_like(asc)
    ws = torch.empty(sm.workspace_bytes(n, m, torch.uint32, descending=True), dtype=torch.uint8,
                     device=dev)
    stream = torch.cuda.current_stream()
    res = {"workload": f"stable_merge of n=m=2^{args.log2n} uint32 uniform keys, keys only, "
                       f"default tile; descending input is the ascending one reversed"}
    for name, keys, flag in (("ascending", asc, False), ("descending", desc, True)):
        def run():
            sm.merge(keys, n, m, out_keys=out, descending=flag, workspace=ws, stream=stream)
        run()
        ms = _events_ms(run, max(args.steps // 2, 3), stream)
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_Gelem/s"] = round((n + m) / (ms * 1e-3) / 1e9, 2)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    res["output_non_increasing"] = bool((o[1:] <= o[:-1]).all())
    return res


def bench_sort(args, with_learned: bool = True):
    """Stable merge sort of 2^28 (uint32 key uniform in [0, 2^24), uint32
    index) pairs: runs of 512 formed in LDS, then 19 merge passes."""
    import numpy as np
    import torch
    import datagen
    import datagen.torch_gen as tg
    import paper_1202_6575_amd as sm

    N = 1 << 28
    log("bench: merge sort of 2^28 (key, index) pairs")
    keys, pay = tg.sort_input(N, 1 << 24, seed=datagen.BASE_SEED + 5)
    ok, op = torch.empty_like(keys), torch.empty_like(pay)
    run_len = args.sort_run
    ws = torch.empty(sm.sort_workspace_bytes(N, torch.uint32, True, run=run_len),
                     dtype=torch.uint8, device=keys.device)
    stream = torch.cuda.current_stream()

    def run():
        sm.sort(keys, pay, out_keys=ok, out_payloads=op, run=run_len, workspace=ws, stream=stream)

    run()
    torch.cuda.synchronize()
    ok64 = ok.to(torch.int64)
    sorted_ok = bool((ok64[1:] >= ok64[:-1]).all())
    del ok64
    ms = _events_ms(run, 3, stream)
    passes = 0
    while (run_len << passes) < N:
        passes += 1
    # run formation + every pass read and write 8 bytes per element
    alg = N * 8 * 2 * (passes + 1)
    # run formation alone (the sort's first phase)
    rk, rp = torch.empty_like(keys), torch.empty_like(pay)

    def runs_only():
        sm.sort_runs(keys, run_len, pay, out_keys=rk, out_payloads=rp, stream=stream)

    runs_only()
    runs_ms = _events_ms(runs_only, 3, stream)
    del rk, rp
    res = {"workload": f"N=2^28 uint32 keys uniform in [0, 2^24), uint32 payload = index, "
                       f"runs of {run_len}, {passes} merge passes",
           "Gelem/s": round(N / (ms * 1e-3) / 1e9, 3), "ms": round(ms, 3),
           "passes": passes, "output_sorted": sorted_ok,
           "avg_GB/s_over_passes": round(alg / (ms * 1e-3) / 1e9, 1),
           "run_formation_ms": round(runs_ms, 3),
           "cpu_baseline": None if args.no_cpu_baseline else sort_cpu_baseline(keys, pay)}
    if not with_learned:
        return res
    # the same sort with learned cross ranks in every pass: one model of the
    # keys' distribution, trained on the first 2^20 keys
    from paper_1202_6575_amd import learned
    log("bench: learned merge sort")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    model, frac = learned.train_sort_model(keys, sample=1 << 20, samples=1 << 18, steps=1000)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3
    lk, lp = torch.empty_like(keys), torch.empty_like(pay)
    cnt = torch.zeros(2, dtype=torch.uint64, device=keys.device)
    zero = torch.zeros(learned.NPARAM, dtype=torch.float32, device=keys.device)
    cz = torch.zeros(2, dtype=torch.uint64, device=keys.device)

    def run_learned():
        learned.sort_learned(keys, model, frac, pay, out_keys=lk, out_payloads=lp, run=run_len,
                             counters=cnt, workspace=ws, stream=stream)

    run_learned()
    learned.sort_learned(keys, zero, 1.0, pay, out_keys=lk, out_payloads=lp, run=run_len,
                         counters=cz, workspace=ws, stream=stream)
    run_learned()
    torch.cuda.synchronize()
    same = bool(torch.equal(lk, ok) and torch.equal(lp, op))
    c = cnt.cpu().numpy().astype(np.int64) // 2
    z = cz.cpu().numpy().astype(np.int64)
    lms = _events_ms(run_learned, 3, stream)
    res["learned"] = {"train_ms": round(train_ms, 1), "step_frac": float(frac),
                      "ms": round(lms, 3), "plain_ms": round(ms, 3),
                      "outputs_bit_equal": same,
                      "searches_per_sort": int(c[0]),
                      "probes_per_rank": round(float(c[1]) / max(int(c[0]), 1), 2),
                      "uninformed_probes_per_rank": round(float(z[1]) / max(int(z[0]), 1), 2)}
    return res


def sort_cpu_baseline(keys, pay, sample: int = 1 << 22):
    """The oracle's stable sort (runs of 512 sorted, then pairwise merge
    rounds, all on one host thread) on the first `sample` (key, index) pairs
    of the same input."""
    import oracle
    k = keys[:sample].cpu().numpy()
    p = pay[:sample].cpu().numpy()
    t = time.perf_counter()
    oracle.sort(k, p, run_len=512)
    dt = time.perf_counter() - t
    return {"value": round(sample / dt / 1e9, 4), "unit": "Gelem/s", "cores": 1,
            "kind": "oracle", "host": host_info(),
            "sample": f"the first {sample} (key, index) pairs of the 2^28 input, oracle stable "
                      f"sort (512-runs, then merge rounds), one thread, {dt:.2f} s; a 2^28 sort "
                      f"takes 28/22 times as many compares per element"}


def _bin_label(k: int) -> str:
    """Error bin k (predicted - exact): 0, or |e| in [2^(|k|-1), 2^|k|) with its sign."""
    if k == 0:
        return "0"
    lo, hi = 1 << (abs(k) - 1), (1 << abs(k)) - 1
    sign = "+" if k > 0 else "-"
    return f"{sign}{lo}" if lo == hi else f"{sign}[{lo},{hi}]"


def bench_learned(args):
    """n = m = 2^28 uint32 keys from a 3-component log-normal mixture, sorted;
    block starts every 16 elements (2^24 cross ranks per side).  Two rank
    models (B's CDF for A's block starts, A's CDF for B's) trained on 2^20
    sampled exact ranks; the learned partition against the plain binary
    search partition, both followed by the one-lane-per-subproblem merge."""
    import numpy as np
    import torch
    import datagen
    import datagen.torch_gen as tg
    import paper_1202_6575_amd as sm
    from paper_1202_6575_amd import learned

    n = m = 1 << 28
    log("bench: learned partition, n=m=2^28 log-normal mixture")
    A = tg.lognormal_mixture(n, seed=datagen.BASE_SEED + 6)
    B = tg.lognormal_mixture(m, seed=datagen.BASE_SEED + 7)
    keys = torch.cat([A, B])
    del A, B
    torch.cuda.empty_cache()
    dA, dB = keys[:n], keys[n:]
    stream = torch.cuda.current_stream()
    samples, steps = 1 << 20, 1000

    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    model_b, loss_b = learned.train_rank_model(dB, dA, False, samples, steps, seed=1)
    model_a, loss_a = learned.train_rank_model(dA, dB, True, samples, steps, seed=2)
    t1.record(stream)
    t1.synchronize()
    train_ms = t0.elapsed_time(t1)
    lb, la = float(loss_b.item()), float(loss_a.item())
    s0a, s0b = learned.step0_from_loss(lb, m), learned.step0_from_loss(la, n)

    p_a, p_b = n // 16, m // 16
    dev = keys.device
    xp = torch.empty(p_a + 1, dtype=torch.int64, device=dev)
    yp = torch.empty(p_b + 1, dtype=torch.int64, device=dev)
    xl, yl = torch.empty_like(xp), torch.empty_like(yp)
    hist = torch.zeros(learned.HIST_BINS, dtype=torch.uint64, device=dev)
    cnt = torch.zeros(4, dtype=torch.uint64, device=dev)
    reps = 5

    def plain():
        sm.partition(keys, n, m, p_a, p_b, xbar=xp, ybar=yp, stream=stream)

    plain()
    plain_ms = _events_ms(plain, reps, stream)
    windows = {}
    for mult in (4, 64):
        W = mult * max(s0a, s0b)

        def learned_run():
            learned.partition_learned(keys, n, m, p_a, p_b, model_b, model_a, s0a, s0b, W,
                                      xbar=xl, ybar=yl, hist=hist, counters=cnt, stream=stream)

        hist.zero_()
        cnt.zero_()
        learned_run()
        torch.cuda.synchronize()
        h = hist.cpu().numpy().astype(np.int64)
        c = cnt.cpu().numpy().astype(np.int64)
        same = bool(torch.equal(xl, xp) and torch.equal(yl, yp))
        ms = _events_ms(learned_run, reps, stream)
        windows[str(W)] = {"ms": round(ms, 4), "ranks_equal_plain": same,
                           "fallback_rate": round(c[1] / c[0], 5),
                           "probes_per_rank": round(c[2] / c[0], 3),
                           "histogram": {_bin_label(i - learned.HIST_CENTER): int(h[i])
                                         for i in range(len(h)) if h[i]}}
    best_w = min(windows, key=lambda w: windows[w]["ms"])

    out_p = torch.empty_like(keys)
    out_l = torch.empty_like(keys)
    ws = torch.empty(max(sm.pieces_workspace_bytes(n, m, p_a, p_b, torch.uint32), 16),
                     dtype=torch.uint8, device=dev)

    def merge_with(xb, yb, out):
        sm.merge_pieces(keys, n, m, p_a, p_b, xb, yb, out_keys=out, workspace=ws, stream=stream)

    merge_with(xp, yp, out_p)
    merge_with(xl, yl, out_l)
    torch.cuda.synchronize()
    outputs_equal = bool(torch.equal(out_p, out_l))
    fine_ms = _events_ms(lambda: merge_with(xl, yl, out_l), reps, stream)
    lw = windows[best_w]["ms"]
    del out_p, ws

    # the same models at the top-level split: blocks of 2368 (the tiled
    # merge's block length), learned against plain partition, then the
    # tiled merge
    tile = 2368
    tp_a, tp_b = (n + tile - 1) // tile, (m + tile - 1) // tile
    txp = torch.empty(tp_a + 1, dtype=torch.int64, device=dev)
    typ = torch.empty(tp_b + 1, dtype=torch.int64, device=dev)
    txl, tyl = torch.empty_like(txp), torch.empty_like(typ)
    tws = torch.empty(sm.pieces_workspace_bytes(n, m, tp_a, tp_b, torch.uint32),
                      dtype=torch.uint8, device=dev)
    W_top = int(best_w)

    def top_plain():
        sm.partition(keys, n, m, tp_a, tp_b, xbar=txp, ybar=typ, stream=stream)

    def top_learned():
        learned.partition_learned(keys, n, m, tp_a, tp_b, model_b, model_a, s0a, s0b, W_top,
                                  xbar=txl, ybar=tyl, hist=hist, counters=cnt, stream=stream)

    top_plain()
    hist.zero_()
    cnt.zero_()
    top_learned()
    torch.cuda.synchronize()
    tc = cnt.cpu().numpy().astype(np.int64)
    top_same = bool(torch.equal(txl, txp) and torch.equal(tyl, typ))
    top_plain_ms = _events_ms(top_plain, reps, stream)
    top_learned_ms = _events_ms(top_learned, reps, stream)
    top_merge_ms = _events_ms(lambda: sm.merge_pieces(keys, n, m, tp_a, tp_b, txl, tyl,
                                                      out_keys=out_l, workspace=tws,
                                                      stream=stream), reps, stream)
    top = {"block": tile, "splitters_per_side": tp_a, "ranks_equal_plain": top_same,
           "plain_partition_ms": round(top_plain_ms, 4),
           "learned_partition_ms": round(top_learned_ms, 4),
           "probes_per_rank": round(tc[2] / max(tc[0], 1), 3),
           "fallback_rate": round(tc[1] / max(tc[0], 1), 5),
           "merge_ms": round(top_merge_ms, 4),
           "end_to_end_Gelem/s": {
               "plain": round((n + m) / ((top_plain_ms + top_merge_ms) * 1e-3) / 1e9, 2),
               "learned": round((n + m) / ((top_learned_ms + top_merge_ms) * 1e-3) / 1e9, 2)}}
    return {"workload": "n=m=2^28 uint32, 3-component log-normal mixture (medians 2^10, 2^20, "
                        "2^28; sigma 0.5), sorted; block starts every 16 elements",
            "splitters_per_side": p_a, "train": {"samples": samples, "steps": steps,
                                                 "ms_both_models": round(train_ms, 2),
                                                 "rms_rank_error_elements":
                                                     [round(np.sqrt(lb) * m), round(np.sqrt(la) * n)],
                                                 "step0": [s0a, s0b]},
            "plain_partition_ms": round(plain_ms, 4),
            "plain_probes_per_rank": int(np.floor(np.log2(m))) + 1,
            "learned_partition": windows, "best_window": int(best_w),
            "partition_speedup_learned_vs_plain": round(plain_ms / lw, 3),
            "fine_merge_ms": round(fine_ms, 4), "outputs_bit_equal": outputs_equal,
            "end_to_end_Gelem/s": {"plain": round((n + m) / ((plain_ms + fine_ms) * 1e-3) / 1e9, 2),
                                   "learned": round((n + m) / ((lw + fine_ms) * 1e-3) / 1e9, 2)},
            "top_level_split": top}


if __name__ == "__main__":
    main()
