"""Compile-time checks of the gfx950 kernels: no register spills, no scratch."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_02207_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="hipcc not available")
def test_kernels_use_no_scratch(tmp_path):
    from paper_2603_02207_amd.build import HIPCC_FLAGS, hipcc

    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip", "-c",
                                     os.path.join(CSRC, "kernels.hip"), "-o", str(tmp_path / "k.o"),
                                     "-Rpass-analysis=kernel-resource-usage"]
    out = subprocess.run(cmd, capture_output=True, text=True)
    assert out.returncode == 0, out.stderr[-2000:]
    names = re.findall(r"Function Name: (\S+)", out.stderr)
    scratch = [int(x) for x in re.findall(r"ScratchSize \[bytes/lane\]: (\d+)", out.stderr)]
    spills = [int(x) for x in re.findall(r"VGPRs Spill: (\d+)", out.stderr)]
    assert len(names) >= 20 and len(names) == len(scratch) == len(spills)
    bad = [(n, s, p) for n, s, p in zip(names, scratch, spills) if s or p]
    assert not bad, bad
