"""Build the FP64 CPU oracle (test infrastructure only) with gcc.

The oracle is compiled with -ffp-contract=off so that the C source is
evaluated as written, without fused multiply-adds.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbl_oracle.c")
LIB = os.path.join(HERE, "liblbl_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=gnu11", "-O2", "-fopenmp", "-ffp-contract=off", "-fPIC",
        "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter",
        SRC, "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
