"""Build libucac.so (the HIP library behind include/ucac.h) for gfx950, in-tree.

Every kernel file is its own translation unit.  The Newton kernel's file lets
hipcc contract a*b+c into FMA (-ffp-contract=fast-honor-pragmas: functions that
declare contraction off inside it -- the unit side it shares a launch with, the
bus QP's per-end sums -- keep plain IEEE rounding); the other kernels are compiled
without contraction so that their few flops round exactly like plain IEEE FP64
code.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libucac.so")
ARCH = "gfx950"

SOURCES = {
    "ucac_api.hip": "off",
    "k_units.hip": "off",
    "k_branch.hip": "fast-honor-pragmas",
    "k_bar.hip": "off",
    "k_ctl.hip": "off",
    "k_mlp.hip": "off",
}

COMMON = ["-O3", f"--offload-arch={ARCH}", "-fPIC", "-std=c++17", "-Wall",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def _compile(name, contract, verbose):
    src = os.path.join(CSRC, name)
    obj = os.path.join(BUILD, name.replace(".hip", ".o"))
    cmd = [hipcc()] + COMMON + [f"-ffp-contract={contract}", "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{r.stderr}")
    return obj


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
