"""Build the HIP library libicarus_hip.so in-tree for gfx950.

    python -m paper_2501_15923_amd.build

Each translation unit is compiled on its own (in parallel), then linked.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libicarus_hip.so")
OBJ_DIR = os.path.join(PKG, "_build")
SOURCES = [os.path.join(PKG, "csrc", f)
           for f in ("icr_kernels.hip", "icr_stage_lds.hip", "icr_ensemble.hip", "icr_api.hip",
                     "icr_nn.hip", "icr_amr.hip")]
HEADERS = [os.path.join(PKG, "csrc", f) for f in ("icr_kernels.hpp", "icr_device.hpp")] + \
    [os.path.join(ROOT, "include", "icarus_hip.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # multiply-adds fused only within one source expression: every copy of an
    # expression the compiler makes (peeled iterations, other kernels) rounds
    # the same way, so tilings, plane chunks and ensemble runs agree bitwise
    "-ffp-contract=on",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
    return res.returncode


def build(verbose: bool = False, jobs: int = 5) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = "-I" + os.path.join(ROOT, "include")
    objs = [os.path.join(OBJ_DIR, os.path.basename(src)[:-4] + ".o") for src in SOURCES]
    cmds = [[hipcc, *HIPCC_FLAGS, inc, "-c", "-o", obj, src] for src, obj in zip(SOURCES, objs)]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        codes = list(ex.map(lambda c: _run(c, verbose), cmds))
    if any(codes):
        raise RuntimeError("hipcc failed compiling libicarus_hip.so")
    tmp = LIB + ".tmp"
    if _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose):
        raise RuntimeError("hipcc failed linking libicarus_hip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
