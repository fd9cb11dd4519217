"""Build-level checks (CPU only): every device kernel compiles for gfx950
without private (scratch) memory.  Scratch lives in HBM, so a spilled or
dynamically indexed private array silently adds memory traffic to kernels
whose whole budget is memory bandwidth."""
import os

import pytest

from paper_1202_6575_amd.build import kernel_resources, sources


@pytest.mark.parametrize("src", [os.path.basename(s) for s in sources() if "api" not in s])
def test_no_scratch(src):
    res = kernel_resources(src)
    assert res, "no kernels found"
    bad = {k: v for k, v in res.items() if v.get("scratch", 0) != 0}
    assert not bad, f"kernels using scratch memory: {bad}"
