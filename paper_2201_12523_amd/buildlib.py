"""Compile the BLCO library for gfx950 into ``paper_2201_12523_amd/libblco.so``.

Host builder (``csrc/blco_host.cpp``) with g++; device runtime and MTTKRP
kernels (``csrc/blco_device.hip``), the CP-ALS driver (``csrc/blco_cpals.hip``) and
the GPU builder (``csrc/blco_build_gpu.hip``) and its sort and compaction
(``csrc/blco_sort.hip``) with hipcc; linked with hipcc.  Run as
``python -m paper_2201_12523_amd.buildlib``.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libblco.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-munsafe-fp-atomics",
    # keep the compiler from forming packed fp32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    t = time.time()
    subprocess.check_call(cmd)
    return time.time() - t


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    host_o = os.path.join(BUILD_DIR, "blco_host.o")
    dev_o = os.path.join(BUILD_DIR, "blco_device.o")
    als_o = os.path.join(BUILD_DIR, "blco_cpals.o")
    gb_o = os.path.join(BUILD_DIR, "blco_build_gpu.o")
    sort_o = os.path.join(BUILD_DIR, "blco_sort.o")
    t = time.time()
    # the objects compile in parallel
    procs = [subprocess.Popen(["g++", "-std=c++17", "-O3", "-fPIC", "-Wall", "-c",
                               os.path.join(CSRC, "blco_host.cpp"), "-o", host_o]),
             subprocess.Popen([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "blco_device.hip"),
                               "-o", dev_o]),
             subprocess.Popen([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "blco_cpals.hip"),
                               "-o", als_o]),
             subprocess.Popen([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "blco_build_gpu.hip"),
                               "-o", gb_o]),
             subprocess.Popen([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "blco_sort.hip"),
                               "-o", sort_o])]
    codes = [p.wait() for p in procs]
    if any(codes):
        raise subprocess.CalledProcessError(max(codes, key=abs), "compile")
    t1 = t2 = time.time() - t
    tmp = OUT + ".tmp"
    t3 = _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", host_o, dev_o, als_o, gb_o, sort_o,
               "-o", tmp, "-lpthread"])
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT} (compile {t1:.1f}s, link {t3:.1f}s)", file=sys.stderr)
    return OUT


if __name__ == "__main__":
    build()
