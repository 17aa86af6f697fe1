"""Builds libregc_hip.so in-tree with hipcc for gfx950.

Every translation unit is compiled with -Xclang -target-feature -Xclang -packed-fp32-ops
(no packed FP32 instructions).  The sweep kernels (plain and learned proposal) are
compiled twice: FP64 with -ffp-contract=off (parity mode) and FP32.  The exchange kernel is compiled without
FP contraction so its FP64 acceptance matches a plain sequential evaluation.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libregc_hip.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = [f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]

UNITS = [
    ("sweep.hip", "sweep_f64.o", ["-DREGC_FP64", "-ffp-contract=off"]),
    ("sweep.hip", "sweep_f32.o", ["-DREGC_FP32"]),
    ("learned.hip", "learned_f64.o", ["-DREGC_FP64", "-ffp-contract=off"]),
    ("learned.hip", "learned_f32.o", ["-DREGC_FP32"]),
    ("swap.hip", "swap.o", ["-ffp-contract=off"]),
    ("obs.hip", "obs.o", ["-ffp-contract=off"]),
    ("mbar.hip", "mbar.o", []),
    ("mlp.hip", "mlp.o", []),
    ("api.cpp", "api.o", ["-x", "hip"]),
]


def _compile(unit):
    src, obj, extra = unit
    cmd = [HIPCC, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", os.path.join(BUILD, obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile of {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return r.stderr


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(UNITS), os.cpu_count() or 1)) as ex:
        for msg in ex.map(_compile, UNITS):
            if verbose and msg.strip():
                print(msg, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
          [os.path.join(BUILD, u[1]) for u in UNITS]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
