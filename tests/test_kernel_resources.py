"""Register and scratch budgets of the trace kernels, read from the
compiler's resource report (a CPU-side compile of the two builds).

The 2-wave build must keep every Dormand-Prince kernel free of spills; the
3-wave build (kt_trace_w3.hip, compiled without machine loop-invariant code
motion) must fit every trace kernel in 168 VGPRs (3 waves per SIMD) without
spills.  A source edit that breaks either budget shows here before it shows
as a slower kernel."""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2202_00086_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

pytestmark = pytest.mark.slow


def _resources(src, extra, tmp_path):
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "--cuda-device-only", "-c", "-o", str(tmp_path / "k.o"),
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *extra, "-Rpass-analysis=kernel-resource-usage",
           os.path.join(CSRC, src)]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert p.returncode == 0, p.stderr[-3000:]
    out, name = {}, None
    for line in p.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            out[name] = {}
            continue
        m = re.search(r"(VGPRs|AGPRs|ScratchSize \[bytes/lane\]|Occupancy \[waves/SIMD\]): (\d+)", line)
        if m and name:
            out[name][m.group(1).split()[0]] = int(m.group(2))
    return {k: v for k, v in out.items() if "trace_kernel" in k}


def test_three_wave_build_fits_three_waves(tmp_path):
    res = _resources("kt_trace_w3.hip", ["-mllvm", "-disable-machine-licm"], tmp_path)
    assert len(res) >= 20
    for name, r in res.items():
        assert r["ScratchSize"] == 0, (name, r)
        assert r["VGPRs"] + r.get("AGPRs", 0) <= 168 and r["Occupancy"] >= 3, (name, r)


def test_two_wave_build_dp45_kernels_do_not_spill(tmp_path):
    res = _resources("kt_trace.hip", [], tmp_path)
    dp45 = {k: v for k, v in res.items() if "trace_kernelILi1E" in k}
    assert len(dp45) >= 10
    for name, r in dp45.items():
        assert r["ScratchSize"] == 0 and r["Occupancy"] >= 2, (name, r)
