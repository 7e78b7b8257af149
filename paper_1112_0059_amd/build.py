"""Build liblnbnn.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "liblnbnn.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "rerank.hip", "api.cpp", "serve.cpp", "noalloc.hip"]
INSTANCE_SRC = "dist_inst.hip"
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def instances():
    """(tag, policy, list length) of every distance-kernel instance set,
    read from the LNBNN_DIST_INSTANCES list in internal.h."""
    with open(os.path.join(CSRC, "internal.h")) as f:
        text = f.read()
    return re.findall(r"X\((\w+), (\w+), \w+, (\d+)\)", text)


def _compile(job) -> str:
    src, obj_name, defines = job
    obj = os.path.join(BUILD, obj_name)
    cmd = ["hipcc", "-x", "hip", *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed for {obj_name}")
    return obj


def build(jobs: int = 0) -> str:
    os.makedirs(BUILD, exist_ok=True)
    work = [(s, os.path.splitext(s)[0] + ".o", []) for s in SOURCES]
    for tag, policy, kp in instances():
        work.append((INSTANCE_SRC, f"dist_{tag}_{kp}.o",
                     [f"-DLNBNN_OP={policy}", f"-DLNBNN_KP={kp}", f"-DLNBNN_SYM=dist_kernel_{tag}_{kp}"]))
    # longest jobs first: the instance sets dominate the build
    work.sort(key=lambda w: w[0] != INSTANCE_SRC)
    n = jobs or min(len(work), os.cpu_count() or 4, 16)
    with ThreadPoolExecutor(n) as ex:
        objs = list(ex.map(_compile, work))
    tmp = OUT + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build())
