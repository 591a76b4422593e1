"""Builds the HIP library libtrig.so for gfx950 in-tree with hipcc.

    python -m paper_1810_11966_amd.build          # library
    python -m paper_1810_11966_amd.build --isa    # also the gfx950 assembly

Flags that the floating point contract depends on (include/trig.h):
  -ffp-contract=off                      no fused multiply-add contraction
  -fno-gpu-flush-denormals-to-zero       binary32 subnormals preserved
  -fhip-fp32-correctly-rounded-divide-sqrt  IEEE division (slope window)
  -Xclang -target-feature -Xclang -packed-fp32-ops
                                         no packed fp32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libtrig.so")
ISA = os.path.join(ROOT, "_build", "trig-gfx950.s")
SOURCES = [os.path.join(CSRC, "trig.hip"), os.path.join(CSRC, "probe.hip"), os.path.join(CSRC, "serve.hip"),
           os.path.join(CSRC, "filter.hip"), os.path.join(CSRC, "events.hip")]
HEADERS = [os.path.join(CSRC, "trig_device.hpp"), os.path.join(CSRC, "trig_block.hpp"),
           os.path.join(CSRC, "serve_core.hpp"), os.path.join(INCLUDE, "trig.h"),
           os.path.join(INCLUDE, "trig_probe.h"), os.path.join(INCLUDE, "trig_serve.h"),
           os.path.join(INCLUDE, "trig_filter.h"), os.path.join(INCLUDE, "trig_events.h"),
           os.path.join(CSRC, "scan_i64.hpp")]
ARCH = "gfx950"

COMMON = ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-ffp-contract=off",
          "-fno-gpu-flush-denormals-to-zero", "-fhip-fp32-correctly-rounded-divide-sqrt",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(isa: bool = False, verbose: bool = False) -> str:
    """Compile every source into libtrig.so (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *COMMON, "-fPIC", "-shared", *SOURCES, "-o", tmp, "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if isa:
        build_isa(verbose)
    return LIB


def build_isa(verbose: bool = False) -> str:
    """gfx950 assembly of the kernels built here (for the instruction checks)."""
    os.makedirs(os.path.dirname(ISA), exist_ok=True)
    cmd = [hipcc(), *COMMON, "--cuda-device-only", "-S", SOURCES[0], "-o", ISA]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return ISA


if __name__ == "__main__":
    build(isa="--isa" in sys.argv, verbose=True)
    print(LIB)
