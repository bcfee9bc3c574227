"""Build the gfx950 shared library ``libdpml.so`` in-tree with hipcc.

Every source is compiled to an object in parallel, then linked.

    python -m paper_1804_01390_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdpml.so")
SOURCES = [os.path.join(HERE, "csrc", n)
           for n in ("dpml.hip", "dpml3d.hip", "dpml_hist.hip", "dpml_frame3d.hip", "probe.hip")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", "dpml_kernels.hpp"), os.path.join(HERE, "csrc", "dpml_host.hpp"),
                  os.path.join(HERE, "csrc", "dpml_kernels3d.hpp"),
                  os.path.join(ROOT, "include", "dpml.h")]
ARCH = "gfx950"

FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         # no packed FP32 instructions in generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # evaluate expressions exactly as written (no FMA contraction)
         "-ffp-contract=off",
         "-Wall", "-Wno-unused-result",
         "-I", os.path.join(ROOT, "include")]


def compile_command(src: str, obj: str):
    return ["/opt/rocm/bin/hipcc"] + FLAGS + ["-c", "-o", obj, src]


def link_command(objs, out: str):
    return ["/opt/rocm/bin/hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out] + list(objs)


def build(verbose: bool = False) -> str:
    tag = "%d" % os.getpid()
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(HERE, os.path.basename(src) + ".%s.o" % tag)
        cmd = compile_command(src, obj)
        if verbose:
            print(" ".join(cmd), flush=True)
        objs.append(obj)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    failed = False
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    try:
        if failed:
            raise RuntimeError("hipcc failed building libdpml.so")
        tmp = LIB + ".tmp" + tag
        cmd = link_command(objs, tmp)
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed linking libdpml.so")
        os.replace(tmp, LIB)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
