"""Split backward sweeps on the host: the adjoint's step VJP
(kt_adjoint_math.h, compiled for the CPU) along a strong-field trajectory,
swept sequentially and as 64-step segments from basis cotangents whose
columns are then applied last segment first
(tests/sanitize/adjoint_split_check.cpp).  The phi cotangent stays exactly
zero in every basis sweep, the two results agree to 1e-13 of their scale,
and combining the segments first-to-last instead is off by far more (the
check sees the order).  Built plain and under ASan/UBSan."""
import os
import re
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2202_00086_amd", "csrc")
SRC = os.path.join(HERE, "sanitize", "adjoint_split_check.cpp")
HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.parametrize("flags", [[], ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]],
                         ids=["plain", "asan_ubsan"])
def test_split_sweep_equals_sequential_sweep(tmp_path, flags):
    exe = str(tmp_path / "split_check")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-g", "-O1", *flags, "-w",
                    "-I", CSRC, "-o", exe, SRC], check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0 and "runtime error" not in p.stderr and "Sanitizer" not in p.stderr, p.stderr[-3000:]
    out = p.stdout
    vals = dict(re.findall(r"(\w+) ([-+0-9.e]+)", out))
    assert float(vals["r_end"]) < 2.5                      # the trajectory reaches the strong field
    assert float(vals["phi_cotangent_sequential"]) == 0.0
    assert int(vals["phi_nonzero"]) == 0
    assert float(vals["split_err"]) < 1e-13, out
    assert float(vals["wrong_order_err"]) > 1e-3, out
