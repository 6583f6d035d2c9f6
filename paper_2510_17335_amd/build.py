"""Builds libddmpm.so (HIP, gfx950) in-tree with hipcc.

hipcc flags: -O3, wave64 gfx950 code, hardware float atomics
(-munsafe-fp-atomics), and packed FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libddmpm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ddm_kernels.hip", "ddm_sort.hip", "ddm_treat.hip", "ddm_emd.hip", "ddm_diag.hip", "ddm_runtime.hip"]
HEADERS = ["ddm_device.hpp", "ddm_kernels.hpp", "ddm_state.hpp", os.path.join("..", "..", "include", "ddmpm.h")]

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-munsafe-fp-atomics",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build(verbose: bool = False) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for p in procs:
        _, err = p.communicate()
        lines = [ln for ln in err.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + "\n".join(lines))
        if lines and verbose:
            print("\n".join(lines), file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs, "-L/opt/rocm/lib",
           "-lrocprofiler-sdk-roctx"]
    subprocess.run(cmd, check=True, stderr=subprocess.PIPE)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
