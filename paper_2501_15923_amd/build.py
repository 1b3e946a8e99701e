"""Build the HIP library libicarus_hip.so in-tree for gfx950.

    python -m paper_2501_15923_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libicarus_hip.so")
SOURCES = [os.path.join(PKG, "csrc", f)
           for f in ("icr_kernels.hip", "icr_stage_lds.hip", "icr_ensemble.hip", "icr_api.hip",
                     "icr_nn.hip")]
HEADERS = [os.path.join(PKG, "csrc", f) for f in ("icr_kernels.hpp", "icr_device.hpp")] + \
    [os.path.join(ROOT, "include", "icarus_hip.h")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # multiply-adds fused only within one source expression: every copy of an
    # expression the compiler makes (peeled iterations, other kernels) rounds
    # the same way, so tilings, plane chunks and ensemble runs agree bitwise
    "-ffp-contract=on",
    # no packed-FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libicarus_hip.so")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
