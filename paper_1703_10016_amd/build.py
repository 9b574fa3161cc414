"""Build libsgbem.so for gfx950 in-tree (paper_1703_10016_amd/libsgbem.so).

Every HIP unit is compiled with hipcc --offload-arch=gfx950 and packed FP32
instructions disabled; the host planner is plain C++.  Objects go to
paper_1703_10016_amd/_build/ (ignored by git), units compile in parallel.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libsgbem.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

HIP_UNITS = ["api.hip", "kernels.hip", "solve.hip", "batch.hip", "serve.hip", "dlayer.hip", "colloc.hip", "knots.hip", "arc.hip",
             "asm_wq_f64.hip", "asm_wq_f32.hip", "asm_ebe_f64.hip", "asm_ebe_f32.hip"]
CXX_UNITS = ["planner.cpp", "planner_knots.cpp", "planner_open.cpp"]
# the register-resident LU panel needs its 64 x 64 column loop fully unrolled
UNIT_FLAGS = {"solve.hip": ["-mllvm", "-pragma-unroll-threshold=1000000"]}
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # hipcc's host pass does not know the packed-fp32 feature; that warning is expected
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and "warning generated" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(jobs: int = 8, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_instances.py")])
    cmds = []
    objs = []
    for u in HIP_UNITS:
        o = os.path.join(BUILD, u + ".o")
        objs.append(o)
        cmds.append([HIPCC] + HIP_FLAGS + UNIT_FLAGS.get(u, []) + ["-c", os.path.join(CSRC, u), "-o", o])
    for u in CXX_UNITS:
        o = os.path.join(BUILD, u + ".o")
        objs.append(o)
        cmds.append(["g++", "-O2", "-std=c++17", "-fPIC", "-pthread", "-Wall", "-c", os.path.join(CSRC, u), "-o", o])
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(_run, cmds):
            if verbose and out.strip():
                print(out)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
