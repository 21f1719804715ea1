"""Build libcosmos.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcosmos.so")
SOURCES = [os.path.join(HERE, "csrc", "cosmos.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def hipcc_cmd(out: str, extra=()) -> list:
    return [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # multiply-adds are fused only inside one source expression, so every kernel that
            # inlines the same point evaluation rounds identically (batched == plain, bitwise)
            "-ffp-contract=on",
            # packed FP32 instructions are disabled for all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *extra, "-o", out, *SOURCES]


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp, extra)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libcosmos.so")
    if resource_usage or verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv)
