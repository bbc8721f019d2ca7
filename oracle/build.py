"""Compile the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP, no target-specific flags (the library is built here and may
run on another host's CPU).  build(native=True) compiles liboracle_native.so
with -O3 -march=native for the host it runs on: the timed CPU baseline builds
that copy on the machine that times it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sbp_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")
OUT_NATIVE = os.path.join(HERE, "liboracle_native.so")


def build(verbose: bool = False, native: bool = False) -> str:
    out = OUT_NATIVE if native else OUT
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc"] + opt + ["-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-Wall", "-Wextra", "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
