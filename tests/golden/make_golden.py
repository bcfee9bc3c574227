"""Writes tests/golden/bump2d_128_m16_samples.json: sampled U values of the
oracle's 128^2 + 16-cell Gaussian-bump run (quadratic ramp to 2, dt = 0.5,
500 steps).  Calls only the oracle and the input generators.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synthetic  # noqa: E402


def main():
    steps = 500
    w = synthetic.bump2d(128, 16, steps)
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    fin, _ = oracle.run(g, oracle.start(g, w.U0), steps)
    rng = np.random.default_rng(123)
    cells = [[int(rng.integers(0, 160)), int(rng.integers(0, 160))] for _ in range(64)]
    cells += [[16, 16], [79, 79], [80, 80], [143, 16], [0, 0], [159, 159]]
    out = {"steps": steps, "cells": cells,
           "U": [float(fin.U[y, x]) for y, x in cells],
           "_note": "(y, x) cell indices into the 160x160 grid, x fastest"}
    with open(os.path.join(HERE, "bump2d_128_m16_samples.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
