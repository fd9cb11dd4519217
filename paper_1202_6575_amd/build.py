"""Builds libstablemerge.so in-tree with hipcc for gfx950.

Every HIP source under csrc/ is compiled to an object of its own (in
parallel; each source holds its kernels and their launchers, so no
relocatable device code is needed), then the objects are linked into a
shared library next to this file.  Packed FP32 instructions are disabled
(``-packed-fp32-ops``) for all device code.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstablemerge.so")
ARCH = "gfx950"


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


COMPILE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
                 "-Wno-unused-function", "-fvisibility=hidden",
                 "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def compile_command(src: str, obj: str):
    return ["hipcc"] + COMPILE_FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", src, "-o", obj]


def link_command(objs, out: str):
    return ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out] + list(objs)


def _run(cmd, verbose: bool, what: str):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError(f"hipcc failed: {what}")
    if err.strip() and verbose:
        sys.stderr.write(err + "\n")


def build_library(verbose: bool = False, jobs: int = 0) -> str:
    import concurrent.futures
    import tempfile
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, (os.cpu_count() or 1)))
    with tempfile.TemporaryDirectory(prefix="sm_build_") as td:
        objs = [os.path.join(td, os.path.basename(s) + ".o") for s in srcs]
        with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
            futs = [ex.submit(_run, compile_command(s, o), verbose, os.path.basename(s))
                    for s, o in zip(srcs, objs)]
            for f in futs:
                f.result()
        tmp = LIB + f".tmp{os.getpid()}"
        _run(link_command(objs, tmp), verbose, "link")
    os.replace(tmp, LIB)
    return LIB


def kernel_resources(src_name: str = "sm_merge.hip"):
    """Compile one source with hipcc's resource-usage remarks and return
    {kernel: {"vgprs": int, "scratch": int, "occupancy": int}}."""
    import re
    import tempfile
    src = os.path.join(HERE, "csrc", src_name)
    with tempfile.TemporaryDirectory() as td:
        cmd = (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "--cuda-device-only",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Rpass-analysis=kernel-resource-usage", "-I", os.path.join(ROOT, "include"),
                "-c", src, "-o", os.path.join(td, "k.o")])
        res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(res.stderr)
    out, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            out[cur] = {}
            continue
        for key, pat in (("vgprs", r"\bVGPRs: (\d+)"), ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"),
                         ("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)")):
            m = re.search(pat, line)
            if m and cur:
                out[cur][key] = int(m.group(1))
    return out


if __name__ == "__main__":
    build_library(verbose=True)
