"""Build the HIP library ``libga.so`` in-tree for gfx950."""

from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SOURCES = [os.path.join(PKG, "csrc", "ga_kernels.hip"), os.path.join(PKG, "csrc", "ga_serve.hip")]
LIB = os.path.join(PKG, "libga.so")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result",
    # branch targets reached only by a jump start on a 32-byte boundary (the
    # padding after an unconditional branch never executes): the sweep's
    # per-step decisions take several such jumps
    "-mllvm", "-align-all-nofallthru-blocks=5",
    # the iterative ILP machine scheduler: same occupancy for every kernel,
    # and the one-wave 32-slot sweep fits two waves per SIMD (252 VGPRs
    # against 302 with accumulation-register traffic under the default)
    "-mllvm", "-amdgpu-sched-strategy=iterative-ilp",
    "-I" + os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every HIP source into ``libga.so`` (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = [hipcc()] + HIPCC_FLAGS + SOURCES + ["-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libga.so")
    if verbose:
        sys.stderr.write(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
