"""Build step: compile the C ABI library libdmc.so for gfx950 in the package directory.

The host compiler (diagram generation, code generation, runtime) is C++17; the graph-independent
kernels are HIP.  Graph kernels are compiled at run time by hiprtc for the same target.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmc.so")
ARCH = "gfx950"
# every HIP object is built without packed FP32 instructions
NOPK = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + cmd[-1])


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj = os.path.join(HERE, "_build")
    os.makedirs(obj, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    common = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
    objs = []
    for src, lang in [("graph.cpp", "c++"), ("blocks.cpp", "c++"), ("construct.cpp", "c++"), ("api.cpp", "c++"), ("renorm.cpp", "c++"), ("host.cpp", "c++"),
                      ("kernels.hip", "hip"),
                      ("flow.hip", "hip"), ("mcmc.hip", "hip"), ("nsf.hip", "hip"), ("probe.hip", "hip")]:
        o = os.path.join(obj, src + ".o")
        cmd = [hipcc, "-c", *common, *inc]
        if lang == "hip":
            cmd += [f"--offload-arch={ARCH}", *NOPK, "-x", "hip"]
        else:
            cmd += ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]
        cmd += ["-o", o, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(o)
    tmp = LIB + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lhiprtc"]
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
