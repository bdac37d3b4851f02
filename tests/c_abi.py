"""Build the plain-C demo of the C ABI (tests/c_abi_demo.c) with gcc: the
header and the HIP runtime API are all a C program needs."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
LIBDIR = os.path.join(ROOT, "paper_2202_00086_amd")


def build_demo(out_dir):
    exe = os.path.join(out_dir, "c_abi_demo")
    cmd = ["gcc", "-std=c99", "-Wall", "-Werror", "-O2", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"),
           os.path.join(HERE, "c_abi_demo.c"), "-L", LIBDIR, "-lkerrtrace",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           f"-Wl,-rpath,{LIBDIR}", f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}", "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe
