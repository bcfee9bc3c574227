"""Build the gfx950 shared library ``libdpml.so`` in-tree with hipcc.

    python -m paper_1804_01390_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdpml.so")
SOURCES = [os.path.join(HERE, "csrc", "dpml.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", "dpml_kernels.hpp"),
                  os.path.join(ROOT, "include", "dpml.h")]
ARCH = "gfx950"


def hipcc_command(out: str):
    return ["/opt/rocm/bin/hipcc", "--offload-arch=" + ARCH, "-O3", "-std=c++17",
            "-fPIC", "-shared",
            # no packed FP32 instructions in generated code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            # evaluate expressions exactly as written (no FMA contraction)
            "-ffp-contract=off",
            "-Wall", "-Wno-unused-result",
            "-I", os.path.join(ROOT, "include"),
            "-o", out] + SOURCES


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libdpml.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
