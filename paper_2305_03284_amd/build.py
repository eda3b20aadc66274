"""Build the HIP library libddh.so for gfx950 with hipcc (in-tree).

Usage: python -m paper_2305_03284_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OUT = os.path.join(HERE, "libddh.so")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["ddh_kernels.hip", "ddh_runtime.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("DDH_OFFLOAD_ARCH", "gfx950")
# packed FP32 instructions are disabled for all device code (see design
# notes); no implicit contraction of a*b+c into FMAs: explicit FMAs are
# written where wanted, so a formula rounds the same in every kernel that
# evaluates it (the persistent work-list kernel and the per-stage kernels
# share their block bodies and give bit-identical results)
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + INCLUDE, "-I" + CSRC]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    noise = ("packed-fp32-ops",)
    msg = "\n".join(l for l in p.stdout.splitlines() if not any(n in l for n in noise))
    if p.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + msg)
    return msg


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(BUILD, src + ".o")
        objs.append(obj)
        cmds.append([HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for msg in ex.map(_run, cmds):
            if verbose and msg.strip():
                print(msg)
    tmp = OUT + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
