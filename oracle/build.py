"""Build the FP64 oracle library (test infrastructure only).

The oracle is compiled with -ffp-contract=off so that every product and
sum is rounded on its own, exactly as the C source reads.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblbmref.so")


def build(verbose=False):
    src = os.path.join(HERE, "lbmref.c")
    cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
           "-Wall", "-Wextra", "-shared", "-fPIC", "-o", LIB + ".tmp", src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
