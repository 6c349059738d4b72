"""Build the FP64 oracle shared library (test infrastructure only).

gcc, -O2 without fast-math and without FMA contraction, so that every
operation in lsp_oracle.c is the plain IEEE operation it reads as.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lsp_oracle.c")
LIB = os.path.join(HERE, "liblsp_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
        "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
        "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
