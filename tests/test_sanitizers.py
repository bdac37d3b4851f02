"""Sanitizer builds of the host code, run on the CPU.

- The oracle (plain C) under AddressSanitizer and UndefinedBehaviorSanitizer,
  driven over every kind of workload and entry point it serves
  (tests/sanitize/oracle_driver.c): no report, and the same checksum as an
  uninstrumented build.
- The library's host runtime (kt_api.cpp: argument checks, workspace
  layouts, parameter packing) under the same sanitizers, linked with host
  stand-ins of the kernel launchers that touch every byte their kernels
  would, on host buffers of exactly the sizes the library asks for
  (tests/sanitize/host_abi_driver.cpp, stub_launch.cpp).
- The adjoint's step vector-Jacobian product compiled for the host under
  ASan/UBSan, MemorySanitizer and with automatic variables initialised to a
  pattern and to zero, against central differences of the step map and
  against the variant that recomputes sin/cos of theta in its reverse loop
  (tests/sanitize/adjoint_vjp_check.cpp): every build prints the same line.
GPU code is never built with a sanitizer here: -Xarch_host keeps each
-fsanitize to the host side of a HIP compile."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
CSRC = os.path.join(ROOT, "paper_2202_00086_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.slow


def _run(exe, env=ENV):
    p = subprocess.run([exe], capture_output=True, text=True, timeout=900, env=env)
    assert p.returncode == 0, p.stdout[-2000:] + p.stderr[-4000:]
    assert "Sanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    return p.stdout.strip().splitlines()[-1]


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    src = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "kt_oracle.c")]
    inc = ["-I", os.path.join(ROOT, "oracle")]
    asan, plain = str(tmp_path / "oracle_asan"), str(tmp_path / "oracle_plain")
    subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *inc, "-o", asan, *src, "-lm"],
                   check=True)
    subprocess.run(["gcc", "-std=c99", "-O2", "-ffp-contract=off", "-fopenmp", *inc, "-o", plain, *src, "-lm"],
                   check=True)
    env = dict(ENV, ASAN_OPTIONS="detect_leaks=1")
    assert _run(asan, env) == _run(plain, env)


def test_host_runtime_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "host_abi_asan")
    subprocess.run([HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=all", "-w",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", exe,
                    os.path.join(SAN, "host_abi_driver.cpp"), os.path.join(SAN, "stub_launch.cpp"),
                    os.path.join(CSRC, "kt_api.cpp")], check=True, capture_output=True)
    line = _run(exe)
    assert line.startswith("ok ") and int(line.split()[1]) > 100


def test_adjoint_step_vjp_on_the_host(tmp_path):
    src = os.path.join(SAN, "adjoint_vjp_check.cpp")
    lines = {}
    for mode in ("plain", "asan_ubsan", "msan", "pattern", "zero"):
        exe = str(tmp_path / f"vjp_{mode}")
        if mode == "msan":
            # no HIP runtime linked: MemorySanitizer needs every linked library instrumented
            cmd = [CLANG, "-x", "hip", "--offload-host-only", "-nogpulib", "-no-hip-rt", "-std=c++17", "-g", "-O1",
                   "-Xarch_host", "-fsanitize=memory", "-I/opt/rocm/include", "-D__HIP_PLATFORM_AMD__"]
        else:
            flags = {"asan_ubsan": ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"],
                     "pattern": ["-ftrivial-auto-var-init=pattern"], "zero": ["-ftrivial-auto-var-init=zero"],
                     "plain": []}[mode]
            cmd = [HIPCC, "-x", "hip", "--offload-host-only", "-std=c++17", "-g", "-O1", *flags]
        subprocess.run(cmd + ["-w", "-I", CSRC, "-o", exe, src], check=True, capture_output=True)
        lines[mode] = _run(exe)
    assert "mismatches 0" in lines["plain"], lines["plain"]
    # every build computes the same numbers: no uninitialised read changes them
    assert len(set(lines.values())) == 1, lines
