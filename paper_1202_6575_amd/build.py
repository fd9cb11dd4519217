"""Builds libstablemerge.so in-tree with hipcc for gfx950.

Every HIP source under csrc/ is compiled in one hipcc invocation into a
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


def hipcc_command(out: str):
    return (["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Wall", "-Wno-unused-function", "-fvisibility=hidden",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-o", out] + sources())


def build_library(verbose: bool = False) -> str:
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("hipcc failed to build libstablemerge.so")
    if err.strip() and verbose:
        sys.stderr.write(err + "\n")
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
