"""Compile-time checks of the HIP kernels (CPU only: hipcc cross-compiles for
gfx950).  The pivot kernel must keep every value in registers: builds of it
that spilled registers to scratch memory gave wrong factors at random clusters
of launches with hundreds of workgroups, while the same source without spills
gave the same factors on every run."""

import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1712_07297_amd", "csrc")


def _resource_usage(src):
    from paper_1712_07297_amd.build import COMMON, _hipcc

    flags = [f for f in COMMON if f != "-fPIC"]
    cmd = [_hipcc()] + flags + ["--cuda-device-only", "-c", os.path.join(CSRC, src), "-o", os.devnull,
                                "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    usage, cur = {}, None
    for line in res.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = m.group(1)
            usage[cur] = {}
            continue
        m = re.search(r"remark:\s+([A-Za-z \[\]/]+?): (\d+|True|False)\b", line)
        if m and cur:
            v = m.group(2)
            usage[cur][m.group(1).strip()] = int(v) if v.isdigit() else v == "True"
    return usage


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"), reason="no hipcc")
def test_pivot_kernel_spills_no_registers():
    usage = _resource_usage("k_factor.hip")
    pivots = {k: v for k, v in usage.items() if "k_pivot" in k}
    assert len(pivots) == 4, sorted(usage)
    for name, u in pivots.items():
        assert u.get("VGPRs Spill") == 0, (name, u)
        assert u.get("Dynamic Stack") is False, (name, u)
