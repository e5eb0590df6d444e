"""CPU proof that the plan-less ragged search stays in bounds and terminates.

The ragged call without a plan does not check the CSR offsets on the host, so
its in-kernel owner search must be safe for any offsets (paper section 2.2:
invalid input becomes a per-point code, never an abort).  The search is a
host/device header; here it is compiled for the CPU with the address and
undefined-behaviour sanitizers and run over well-formed and adversarial int64
offsets through a bounds-checked view (any read outside offsets[0..n] aborts).
Well-formed offsets must give exactly the owning satellite of every point.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "csrc", "ragged_search_check.cpp")
INC = os.path.join(ROOT, "paper_2603_27830_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_ragged_search_in_bounds_and_exact(tmp_path):
    exe = str(tmp_path / "ragged_search_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", INC, "-o", exe, SRC]
    subprocess.run(cmd, check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert p.returncode == 0, p.stdout + p.stderr
    assert p.stdout.startswith("ok:"), p.stdout
    print(p.stdout.strip())
