"""Build the oracle's shared library (plain C, FP64, no FMA contraction, no fast-math; OpenMP
for its row loops, whose results do not depend on the thread count).

TEST INFRASTRUCTURE: the oracle is only loaded by the tests, the smoke check and the CPU-baseline
leg of the benchmark.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vplbm_oracle.c")
LIB = os.path.join(HERE, "libvplbm_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-Wall", "-Wextra",
           "-fopenmp", "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
