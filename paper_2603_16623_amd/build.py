"""Build step: compile the gfx950 HIP library ``libwake.so`` in-tree.

Run ``python -m paper_2603_16623_amd.build``; ``__graft_entry__.build``
calls :func:`build`.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libwake.so")
SOURCES = [os.path.join(CSRC, "wake_march.hip"), os.path.join(CSRC, "wake_beam.hip"),
           os.path.join(CSRC, "wake_api.cpp"), os.path.join(CSRC, "wake_serve.cpp"),
           os.path.join(CSRC, "wake_tune.cpp"), os.path.join(CSRC, "wake_ions.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # keep loop-invariant constants (math-library coefficients) out of the
    # marcher's register file: measured faster than hoisting them
    "-mllvm", "-disable-machine-licm",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, *extra, *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libwake.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
