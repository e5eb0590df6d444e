"""Build the SGP4 oracle shared library (test infrastructure only).

Plain g++: optimised, but with no fast-math and no fused multiply-add
contraction, so every operation rounds as written in the source.  The
default build is portable (it travels with the repository); native=True adds
-march=native for timing the oracle on the machine that builds it (the
rounding is the same: without fast-math the compiler may vectorise but not
reassociate or contract).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sgp4_oracle.cpp")
LIB = os.path.join(HERE, "liboracle_sgp4.so")


def flags(native: bool = False):
    f = ["-O3", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread", "-Wall",
         "-Wextra"]
    return f + (["-march=native"] if native else [])


def build(verbose: bool = False, native: bool = False, out: str = None) -> str:
    lib = out or LIB
    cmd = ["g++"] + flags(native) + ["-o", lib + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
