"""Builds the in-tree shared library paper_1901_01685_amd/_lib/libpmg.so.

Host setup sources (C++17) are compiled with g++ -ffp-contract=off so every
setup sum is evaluated in the order written; the device translation unit is
compiled by hipcc for gfx950 only.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT, "libpmg.so")
HOST_SRCS = ["setup_assembly.cpp", "setup_ilut.cpp"]
DEV_SRCS = ["pmg_device.hip", "pmg_serve.hip", "setup_device.hip"]
ARCH = "gfx950"


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout)
        raise RuntimeError(f"build step failed: {cmd[0]} ({r.returncode})")
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT, exist_ok=True)
    objs = []
    for s in HOST_SRCS:
        o = os.path.join(OUT, s + ".o")
        _run(["g++", "-std=c++17", "-O3", "-fPIC", "-ffp-contract=off", "-Wall", "-c",
              os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    hipcc = _hipcc()
    for s in DEV_SRCS:
        o = os.path.join(OUT, s + ".o")
        # the device ILUT reproduces the host factorisation's rounding: no FMA contraction
        extra = ["-ffp-contract=off"] if s == "setup_device.hip" else []
        _run([hipcc, "-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument"] + extra + ["-c", os.path.join(CSRC, s), "-o", o])
        objs.append(o)
    tmp = LIB + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + ["-lpthread"])
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
