"""Build the gfx950 HIP library libedupic.so in-tree.

hipcc, FP64 with -ffp-contract=off (no fused multiply-add, so the push and
collision arithmetic round exactly as written), packed-FP32 instructions
disabled.  Machine-level loop-invariant code motion is off: it hoists the
FP64 polynomial constants of every transcendental function in a loop body
(sin, cos, log, exp, atan, tan) into registers ahead of the loop, which in
the particle kernels' scattering loop costs about 60 registers and, under the
128-register budget of four workgroups per CU, spills to scratch.  Re-created
inside loops they cost one move each.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libedupic.so")
SOURCES = ["csrc/kernels.hip", "csrc/capi.hip"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.exists(c) or c == "hipcc":
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-disable-machine-licm",
           "-Wall", "-Wno-unused-result",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           *[os.path.join(HERE, s) for s in SOURCES], "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
