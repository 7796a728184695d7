"""Writes the oracle regression locks in this folder.

The paper prints no worked example (no tap values, no image values), so the
stored values here are the oracle's own, frozen so that any later change to its
arithmetic shows up.  This script calls only ``oracle`` and the input
generators.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1912_05529_amd import synth  # noqa: E402

ROWS = [0, 100, 255, 511]
SAMPLES = [(0, 62), (20, 40), (41, 62), (41, 60), (60, 90), (127, 5)]


def main():
    s = synth.config1()
    tab, mg, pe, sc = oracle.design_table(s.desc)
    img = oracle.migrate(s.desc, tab, s.omega, s.vel, s.data)
    out = {
        "about": "FP64 oracle regression lock for config 1 (constant velocity, "
                 "one scatterer, seed 1); written by make_golden.py",
        "table_rows": {str(j): [[float(c.real), float(c.imag)] for c in tab[j]] for j in ROWS},
        "maxgain": {str(j): float(mg[j]) for j in ROWS},
        "passerr": {str(j): float(pe[j]) for j in ROWS},
        "image_samples": [[iz, ix, float(img[iz, ix])] for iz, ix in SAMPLES],
        "image_l2": float(np.linalg.norm(img)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "config1_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
