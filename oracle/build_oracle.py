"""Compiles the oracle's C sources into oracle/liboracle.so (gcc, -O2; OpenMP
for the level-parallel CPU baseline).

Building the checker is part of the build step; only the test suite, the
smoke check and the bench's CPU-baseline leg load the result.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    srcs = [os.path.join(HERE, f) for f in ("lz_oracle.c", "lz_levels_omp.c", "lz_rans.c")]
    out = os.path.join(HERE, "liboracle.so")
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC"] + srcs + ["-o", out, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose=True)
