"""Build libfciqmc.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfciqmc.so")

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # every floating-point decision keeps the written operation order
    "-ffp-contract=off",
    # no packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-value", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    # kernels_w2.hip: the same kernels for two-word determinants (namespace fq::w2)
    srcs = [os.path.join(CSRC, f) for f in ("kernels.hip", "kernels_w2.hip", "engine.hip")]
    cmd = ["hipcc", *HIPCC_FLAGS, "-o", LIB + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
