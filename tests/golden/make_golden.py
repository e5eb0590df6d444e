"""Write the oracle regression fixture for the 64-satellite smoke catalogue.

Calls only the oracle (and the seeded catalogue generator): the stored values
guard the oracle against unintended change; they are not GPU results.
Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c0_oracle_sample.txt")


def main():
    cat = synth.config0()
    cols = [0, 33, 66, 99]
    r, v, err = oracle.propagate(cat.elem, cat.t[cols])
    with open(OUT, "w") as f:
        f.write("# oracle FP64 states for the 64 x 100 smoke catalogue (seed 0) at time columns 0, 33, 66, 99\n")
        f.write("# sat t_min code rx ry rz (km) vx vy vz (km/s)\n")
        for i in range(cat.n):
            for k, j in enumerate(cols):
                vals = [r[0, i, k], r[1, i, k], r[2, i, k], v[0, i, k], v[1, i, k], v[2, i, k]]
                f.write(f"{i} {cat.t[j]:.17g} {err[i, k]} " + " ".join(f"{x:.17g}" for x in vals) + "\n")


if __name__ == "__main__":
    main()
