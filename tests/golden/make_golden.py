"""Writes the stored expected values under tests/golden/ (calls only oracle/).

sphere40_f64.json: a 40^3 FP64 sphere (r = 0.3 at the centre, F = 1, dx =
1/40, dt = dx/2), 6 full-grid steps of the upwind update (Eq. 3-5), then the
band tile lists (8^3 tiles, gamma = 3 dx, Eq. 6 / Eq. 11 in tile form) of the
result and phi at a fixed set of sample points, written with repr() so the
values round-trip exactly.  Regenerate with
    python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def sphere_case():
    n = 40
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    zz, yy, xx = np.meshgrid(x, x, x, indexing="ij")
    phi = np.sqrt((xx - 0.5) ** 2 + (yy - 0.5) ** 2 + (zz - 0.5) ** 2) - 0.3
    F = np.ones_like(phi)
    return phi, F, dx, 0.5 * dx


SAMPLES = [(0, 0, 0), (20, 20, 20), (5, 20, 33), (20, 3, 20), (39, 39, 39), (7, 8, 9), (20, 20, 8), (31, 12, 27)]


def compute():
    phi, F, dx, dt = sphere_case()
    out = oracle.run_full(phi, F, dx, dt, 6)
    gamma = np.float32(3 * dx)
    return {
        "steps": 6,
        "band_u": oracle.band_tiles(out.astype(np.float32), (8, 8, 8), gamma, True).tolist(),
        "band_a": oracle.band_tiles(out.astype(np.float32), (8, 8, 8), gamma, False).tolist(),
        "samples": [[k, j, i, repr(float(out[k, j, i]))] for k, j, i in SAMPLES],
    }


if __name__ == "__main__":
    with open(os.path.join(HERE, "sphere40_f64.json"), "w") as fh:
        json.dump(compute(), fh, indent=1)
