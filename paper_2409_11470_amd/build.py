"""Build libapr.so for gfx950 with hipcc (one object per source, then link).

Every HIP source is compiled with packed FP32 instructions disabled
(-packed-fp32-ops) and for gfx950 only."""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libapr.so")
ROOT = os.path.dirname(HERE)

SOURCES = ["abi.cpp", "sort.hip", "cells.hip", "density.hip", "forces.hip", "neighbours.hip",
           "integrate.hip", "splitmerge.hip", "adjoint.hip", "candidates.hip", "relax.hip",
           "bins.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-Wall",
         "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]


def _compile(src):
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, obj, r


def build(verbose=False, jobs=8):
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for src, obj, r in ex.map(_compile, SOURCES):
            msg = (r.stdout + r.stderr).strip()
            # hipcc's host pass does not know the device-only feature flag
            msg = "\n".join(l for l in msg.splitlines()
                            if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
            if r.returncode != 0:
                raise RuntimeError("hipcc failed on %s:\n%s" % (src, msg))
            if verbose and msg:
                print(msg, file=sys.stderr)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
