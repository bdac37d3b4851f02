"""The plain-C demo (tests/c_abi_demo.c) renders the 64x64 Schwarzschild
shadow through the C ABI with hipMalloc'd buffers, no Python in the loop:
872 captured pixels, Synge's count for this grid."""
import subprocess
import sys

import pytest

from tests.c_abi import build_demo

pytestmark = pytest.mark.gpu


def test_plain_c_program_renders_the_shadow(tmp_path):
    exe = build_demo(str(tmp_path))
    print("[gpu-case] c_abi_demo schwarzschild 64", flush=True)
    sys.stdout.flush()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, (r.stdout, r.stderr)
    assert "captured 872 " in r.stdout
