"""Build the CPU oracle (plain C, FP64) into oracle/liboracle.so.

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg load the result; the GPU library never does.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
        "-fPIC", "-shared", "-fopenmp",
        "-D_DEFAULT_SOURCE",
        os.path.join(HERE, "lbm_oracle.c"),
        "-o", LIB + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
