"""Compile the FP64 C oracle into oracle/liboracle_nufft.so (gcc, OpenMP).

Test infrastructure: the oracle is the plain reference the GPU library is
checked against; it is never part of the product path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nufft_oracle.c")
LIB = os.path.join(HERE, "liboracle_nufft.so")

# -ffp-contract=off keeps the single rounded multiply u = omega * K/(2 pi)
# that fixes the interpolation window (no fused multiply-add anywhere).
CFLAGS = ["-O2", "-std=gnu99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-fPIC", "-shared", "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
