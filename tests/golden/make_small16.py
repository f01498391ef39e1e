"""Writes small16.json: FP64 oracle results on the 16-view 128x128 scan.

The paper prints no worked example, so these stored values come from the
oracle alone (this script imports only ``oracle`` and the input generator) and
serve as a regression record of it: any change to the oracle's arithmetic that
moves them must say which passage of the paper, or which reading of it,
justifies the change.

Run from the repository root:  python tests/golden/make_small16.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1806_02637_amd import inputs  # noqa: E402


def main():
    w = inputs.WORKLOADS["small16"]
    g = w.geom
    P, intr = g.projection_matrices(), g.intrinsics()
    grid = oracle.SinoGrid(g.W, g.H, w.n_alpha, w.n_t, w.ds_px)
    imgs = inputs.project(g, w.phantom())
    sino = oracle.FullSinograms.build(imgs, grid, intr)
    params = oracle.EccParams(w.K, w.R_mm)
    thetas = np.concatenate([np.zeros((1, g.n_views, 6)), inputs.random_motion(1001, 2, g.n_views)])
    out = {"workload": "small16", "K": w.K, "R_mm": w.R_mm, "motion_seed": 1001, "hypotheses": []}
    for th in thetas:
        cost, e, d, N = oracle.ecc_cost(P, intr, th, grid, sino, params)
        out["hypotheses"].append({"cost": cost, "d": d.tolist(), "N": N.tolist()})
    cells = [(0, 0, 90), (3, 45, 100), (7, 90, 60), (15, 179, 120), (9, 180, 33)]
    out["sinogram_cells"] = [[v, m, k, float(sino.data[v, m, k])] for v, m, k in cells]
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "small16.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
