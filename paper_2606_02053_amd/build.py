"""Build libcosmos.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libcosmos.so")
SOURCES = [os.path.join(HERE, "csrc", "cosmos.hip")]
# machine probes (STREAM triad, FP64 FMA rate) for the benchmark's achievable rooflines
PROBE_LIB = os.path.join(HERE, "libcosmos_probe.so")
PROBE_SOURCES = [os.path.join(HERE, "csrc", "probes.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def hipcc_cmd(out: str, extra=(), sources=None) -> list:
    return [HIPCC, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            # multiply-adds are fused only inside one source expression, so every kernel that
            # inlines the same point evaluation rounds identically (batched == plain, bitwise)
            "-ffp-contract=on",
            # packed FP32 instructions are disabled for all device code
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *extra, "-o", out, *(SOURCES if sources is None else sources)]


def _compile(lib: str, sources, verbose: bool, resource_usage: bool) -> str:
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    tmp = lib + ".tmp"
    cmd = hipcc_cmd(tmp, extra, sources)
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=ROOT, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    if resource_usage or verbose:
        sys.stderr.write(r.stderr)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False, resource_usage: bool = False) -> str:
    _compile(PROBE_LIB, PROBE_SOURCES, verbose, resource_usage)
    return _compile(LIB, SOURCES, verbose, resource_usage)


if __name__ == "__main__":
    build(verbose=True, resource_usage="--usage" in sys.argv)
