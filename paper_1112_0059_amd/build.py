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


# host-code sanitizers: every -fsanitize= applies to the host pass only
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
                  "-Xarch_host", "-g"]


def _compile(job) -> str:
    src, obj_name, defines = job
    obj = os.path.join(BUILD, obj_name) if not os.path.isabs(obj_name) else obj_name
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


def asan_runtime() -> str:
    """The AddressSanitizer runtime of the compiler hipcc drives (a process
    that loads a sanitized build preloads it)."""
    r = subprocess.run(["hipcc", "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        raise RuntimeError("hipcc's libclang_rt.asan-x86_64.so not found")
    return path


def build_sanitized(out_dir: str) -> str:
    """liblnbnn.so with its host code built under AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unchanged), into out_dir: the
    host sources are recompiled there, the distance-kernel instance objects
    of the regular build are reused (built first if missing)."""
    os.makedirs(out_dir, exist_ok=True)
    inst = [os.path.join(BUILD, f"dist_{tag}_{kp}.o") for tag, _, kp in instances()]
    if not all(os.path.exists(o) for o in inst):
        build()
    work = [(s, os.path.join(out_dir, os.path.splitext(s)[0] + ".o"), SANITIZE_FLAGS) for s in SOURCES]
    with ThreadPoolExecutor(min(len(work), os.cpu_count() or 4, 16)) as ex:
        objs = list(ex.map(_compile, work))
    out = os.path.join(out_dir, "liblnbnn.so")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libsan",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           *objs, *inst, "-o", out, "-lpthread"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(build())
