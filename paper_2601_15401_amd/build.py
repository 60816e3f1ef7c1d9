"""Builds libmick.so and the mick_rates probe in the package directory with
hipcc for gfx950.  Translation units compile in parallel."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libmick.so")
RATES = os.path.join(PKG, "mick_rates")
HIP_SOURCES = ["ntt.hip", "tensor.hip", "rns.hip", "api.hip", "queue.hip", "tree.hip", "bconv.hip"]
HOST_SOURCES = ["host_math.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 instructions are kept out of every kernel.
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
             "-packed-fp32-ops", "-mcode-object-version=5", "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s" % (" ".join(cmd), out))
    return out


def _jobs() -> int:
    return max(1, min(8, int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))


def build(verbose: bool = False) -> str:
    obj_dir = os.path.join(ROOT, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    steps = []
    objs = []
    for src in HIP_SOURCES:
        o = os.path.join(obj_dir, src + ".o")
        steps.append([HIPCC] + HIP_FLAGS + ["-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    for src in HOST_SOURCES:
        o = os.path.join(obj_dir, src + ".o")
        steps.append(["g++", "-O2", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    rates_tmp = RATES + ".tmp"
    steps.append([HIPCC] + HIP_FLAGS + [os.path.join(CSRC, "rates.hip"), "-o", rates_tmp])
    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        list(ex.map(_run, steps))
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp])
    os.replace(tmp, LIB)
    os.replace(rates_tmp, RATES)
    if verbose:
        print("built", LIB, "and", RATES)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
