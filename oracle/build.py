"""Compile the FP64 oracle into oracle/liboracle.so (gcc, OpenMP).

Test infrastructure: the oracle is built beside the GPU library but never
linked into it.  -ffp-contract=off keeps every multiply and add a separately
rounded IEEE double operation; x86-64-v3 (AVX2) keeps the binary portable
between the build host and the benchmark host.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fe_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False):
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-o", LIB + ".tmp", SRC,
           "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
