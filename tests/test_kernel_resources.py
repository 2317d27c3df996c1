"""The HIP kernels compile for gfx950 without register spills in their loops.

A spill turns into per-lane scratch memory traffic on every loop trip of the
tile-block kernels, so the compiler's resource report (built here on the CPU)
must show zero scratch for every kernel but two. The nearest-higher and
density kernels are built for eight and seven waves per SIMD (64 and 72
VGPRs), and the compiler then keeps a few item-level values in scratch:
stored once per workgroup and reloaded a few times per work item, outside
the candidate loops. Nearest-higher may use up to 32 bytes and density up to
16."""
import os
import re
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, os.path.join(ROOT, "paper_2001_09761_amd"))


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_no_scratch_spills(tmp_path):
    import build as B
    flags = [f for f in B.FLAGS if f not in ("-shared", "-fPIC")]
    src = os.path.join(B.CSRC, "clue_kernels.hip")
    cmd = [B.HIPCC, *flags, "-I", os.path.join(ROOT, "include"), "-I", B.CSRC, "-c", src,
           "-o", str(tmp_path / "k.o"), "-Rpass-analysis=kernel-resource-usage"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    report = {}
    name = None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"ScratchSize \[bytes/lane\]: (\d+)", line)
        if m and name:
            report[name] = int(m.group(1))
    kernels = {k: v for k, v in report.items() if "k_" in k}
    assert len(kernels) >= 20, sorted(report)
    spills = {k: v for k, v in kernels.items()
              if v and not (("k_nearest_higher" in k and v <= 32) or ("k_density" in k and v <= 16))}
    assert not spills, spills
