"""Build libkerrtrace.so for gfx950 with hipcc (in-tree).

    python -m paper_2202_00086_amd.build

Each source is compiled to an object of its own (in parallel), then linked.
kt_trace_w3.hip, the 3-wave form of the trace kernels, is compiled without
the backend's machine loop-invariant code motion (see that file).
"""
import os
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libkerrtrace.so")
# (source, flags of its own)
UNITS = [("kt_trace.hip", []),
         ("kt_trace_w3.hip", ["-mllvm", "-disable-machine-licm"]),
         ("kt_adjoint.hip", []),
         ("kt_noalloc.hip", []),
         ("kt_api.cpp", [])]
SOURCES = [os.path.join(CSRC, f) for f, _ in UNITS]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose=False, extra=(), out=LIB):
    tmp = tempfile.mkdtemp(prefix="kerrtrace_build_")
    try:
        cmds = []
        for f, own in UNITS:
            obj = os.path.join(tmp, os.path.splitext(f)[0] + ".o")
            cmds.append((obj, [HIPCC, *FLAGS, *own, *extra, "-c", "-o", obj, os.path.join(CSRC, f)]))
        if verbose:
            for _, cmd in cmds:
                print(" ".join(cmd), flush=True)
        with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
            for r in ex.map(lambda c: subprocess.run(c[1]), cmds):
                if r.returncode != 0:
                    raise subprocess.CalledProcessError(r.returncode, r.args)
        link = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", out + ".tmp", *[o for o, _ in cmds]]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
        os.replace(out + ".tmp", out)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
