"""Build libsre2.so (gfx950) in-tree with hipcc.

    python -m paper_2512_24685_amd.build

Every HIP translation unit is compiled with packed-FP32 instructions disabled
(-Xclang -target-feature -Xclang -packed-fp32-ops): the kernels use scalar
float arithmetic only.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsre2.so")
PROBE = os.path.join(HERE, "probe_mall")  # memory-hierarchy probe (bench.py --mall-probe)
PROBE_LDS = os.path.join(HERE, "probe_lds")  # LDS bank-conflict probe (run under rocprofv3)
PROBE_STORE = os.path.join(HERE, "probe_store")  # HBM store-rate probe of slab layouts
SOURCES = ["sre2_kernels.hip", "sre2_api.hip", "sre2_server.hip", "sre2_sim.hip",
           "sre2_noalloc.hip", "sre2_queries.hip"]
ARCH = "gfx950"

HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False, jobs: int = 4) -> str:
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = ["hipcc", *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
        objs.append(obj)
        if len(procs) >= jobs:
            for p in procs:
                if p.wait() != 0:
                    raise RuntimeError("hipcc failed")
            procs = []
    for p in procs:
        if p.wait() != 0:
            raise RuntimeError("hipcc failed")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    for o in objs:
        os.remove(o)
    for src, exe in (("probe_mall.hip", PROBE), ("probe_lds.hip", PROBE_LDS),
                     ("probe_store.hip", PROBE_STORE)):
        cmd = ["hipcc", *HIP_FLAGS, os.path.join(CSRC, src), "-o", exe + ".tmp"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(exe + ".tmp", exe)
    return LIB


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
