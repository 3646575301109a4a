"""Builds the gfx950 shared library libbx.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbx.so")
# host C++ (g++) and HIP translation units (hipcc); the tiled UTIL kernel is
# split by cost type and staging variant so the units compile in parallel
SOURCES = ["bx_plan.cpp", "bx_partition.cpp", "bx_capi.cpp", "bx_bnb.cpp", "bx_exec.hip",
           "bx_k_i32_s0.hip", "bx_k_i32_s1.hip", "bx_k_f32_s0.hip", "bx_k_f32_s1.hip", "bx_k_fs_s0.hip",
           "bx_k_fs_s1.hip", "bx_k_misc.hip", "bx_stream.hip",
           "bx_mlp.hip", "bx_cand.hip"]
ARCH = "gfx950"

# HIP code is compiled without packed-FP32 instructions (the compiler would
# otherwise form v_pk_* from scalar float code).
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False, jobs: int = 0) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(build_dir, src + ".o")
        if src.endswith(".hip"):
            cmd = [hipcc, f"--offload-arch={ARCH}", *COMMON, *DEVICE_FLAGS, "-c", path, "-o", obj]
        else:
            cmd = ["g++", *COMMON, "-c", path, "-o", obj]
        cmds.append(cmd)
        objs.append(obj)

    def run(cmd):
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    jobs = jobs or min(len(cmds), max(1, min(os.cpu_count() or 1, 8)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for f in [ex.submit(run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
