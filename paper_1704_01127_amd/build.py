"""Build libqsim.so (HIP for gfx950) in-tree with hipcc.

Every source is compiled with the packed-FP32 instructions disabled
(``-target-feature -packed-fp32-ops``): the kernels use plain FP32 FMAs and
the FP32 / FP64 matrix cores only.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqsim.so")
SOURCES = ["qsim_kernels.hip", "qsim_mlp.hip", "qsim_api.cpp", "qsim_batch.cpp", "scheduler.cpp", "stages.cpp", "learned.cpp", "qsim_noalloc.hip"]
ARCH = os.environ.get("QSIM_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def common_flags():
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc(), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + common_flags()
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        return obj

    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "-pthread", "--offload-arch=" + ARCH, "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    # measurement tool: streaming-bandwidth probe and traffic-counter calibration kernel
    probe = os.path.join(HERE, "stream_probe")
    cmd = [hipcc(), os.path.join(CSRC, "stream_probe.hip"), "-o", probe + ".tmp"] + common_flags()
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for stream_probe.hip:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(probe + ".tmp", probe)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
