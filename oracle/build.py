"""Build step of the CPU oracle (test infrastructure only).

Compiles oracle.c and batch.c into liborc.so with gcc, without contraction of
multiply-adds, and with OpenMP for the batched drivers.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
SOURCES = ["oracle.c", "batch.c"]


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-fopenmp", "-std=c99", "-Wall"]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
