"""Writes the stored oracle fixtures in this folder.  Calls only ``oracle``
and ``workloads``; run from the repository root:

    python tests/golden/make_golden.py
"""
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads as W  # noqa: E402


def main():
    img, _ = W.ellipse_phantom_2d(1)
    g = oracle.parallel_2d((64, 64), (1.0, 1.0), 95, 1.0, 90, math.pi)
    p = oracle.forward(img, g)[::15, 0, :]
    np.savetxt(
        os.path.join(HERE, "parallel2d_64_forward.txt"), p, fmt="%.17g",
        header="oracle forward projection, 64x64 image (10 ellipses, seed 1, 1 mm), "
               "90 parallel views over 180 deg, 95 bins at 1 mm; rows = views 0, 15, ..., 75",
    )


if __name__ == "__main__":
    main()
