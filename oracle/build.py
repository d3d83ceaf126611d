"""Build the oracle's shared library (plain C, gcc, FP64, no FMA contraction).

Test infrastructure only: the tests, the smoke check and the benchmark's
CPU-baseline leg load the library this builds.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["rsv_oracle.c"]
LIB = os.path.join(HERE, "liborsv.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", LIB]
    cmd += [os.path.join(HERE, s) for s in SOURCES]
    cmd += ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    return LIB


def up_to_date() -> bool:
    if not os.path.exists(LIB):
        return False
    lib_t = os.path.getmtime(LIB)
    deps = SOURCES + ["rsv_oracle.h"]
    return all(os.path.getmtime(os.path.join(HERE, d)) <= lib_t for d in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
