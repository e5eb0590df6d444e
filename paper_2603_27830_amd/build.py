"""Build the HIP library libsgp4mi.so for gfx950 (in-tree, next to this file)."""
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libsgp4mi.so")
CALIB_LIB = os.path.join(HERE, "libsgp4mi_calib.so")
CALIB_SRC = os.path.join(HERE, "calib", "calib.hip")
ARCH = "gfx950"


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def command(out, srcs):
    return ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Wall", "-Wno-unused-command-line-argument",
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-o", out] + srcs


def _compile(lib, srcs, verbose):
    tmp = lib + ".tmp"
    cmd = command(tmp, srcs)
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in p.stderr.splitlines() if "packed-fp32-ops" not in l and "is not a recognized feature" not in l]
    if p.returncode != 0:
        sys.stderr.write("\n".join(noise) + "\n")
        raise RuntimeError(f"hipcc failed building {os.path.basename(lib)}")
    if verbose and noise:
        sys.stderr.write("\n".join(noise) + "\n")
    os.replace(tmp, lib)


def build(verbose: bool = False) -> str:
    _compile(LIB, sources(), verbose)
    _compile(CALIB_LIB, [CALIB_SRC], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
