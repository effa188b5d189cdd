"""Build librdct.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_1402_6034_amd.build [--verbose]
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librdct.so")
ARCH = "gfx950"

SOURCES = ["rdct_kernels.hip", "rdct_quality.hip", "rdct_codec.hip", "rdct_api.cpp",
           "rdct_batch.cpp", "rdct_server.cpp", "rdct_tune.cpp", "rdct_transforms.cpp",
           "rdct_quality_api.cpp", "rdct_codec_api.cpp"]

# Packed FP32 instructions are disabled for all device code; the compiler still
# uses ordinary scalar and 16-bit packed integer instructions.
HIP_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIP_FLAGS, "-shared", "-o", tmp, *[_as_hip(s) for s in srcs],
           "-lpthread"]
    cmd = [c for part in cmd for c in (part if isinstance(part, list) else [part])]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building librdct.so")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


def _as_hip(path: str):
    # .cpp sources hold host code that includes HIP headers; compile them as HIP.
    return ["-x", "hip", path] if path.endswith(".cpp") else [path]


if __name__ == "__main__":
    print(build(verbose="--verbose" in sys.argv))
