"""Exact gradient of the total cost with respect to the per-view motion
parameters (test infrastructure).

Each e_ab depends on theta_a and theta_b only, so the per-pair code of
``ecc.py`` is run on dual numbers with 12 tangent slots (theta_a then
theta_b) and the two 6-vectors are added into the per-view gradient.  Discrete
decisions (hit tests, floor cells, folds) are held at their values, so this
is the derivative of the piecewise-smooth cost on the current cell pattern.
"""
from __future__ import annotations

import numpy as np

from .ecc import EccParams, as_rows, ecc_pair_grad, pair_list


def ecc_grad(P, intr, theta, grid, sino, params: EccParams, pairs=None):
    """Returns (cost, grad [N, 6], per-pair gradient [n_pairs, 12])."""
    n = len(P)
    if pairs is None:
        pairs = pair_list(n)
    grad = np.zeros((n, 6))
    per_pair = np.zeros((len(pairs), 12))
    cost = 0.0
    for i, (a, b) in enumerate(pairs):
        e, g = ecc_pair_grad(as_rows(P[a]), as_rows(P[b]), [float(x) for x in theta[a]],
                             [float(x) for x in theta[b]], intr[a], intr[b], grid, sino, a, b, params)
        cost += e
        per_pair[i] = g
        grad[a] += g[:6]
        grad[b] += g[6:]
    return cost, grad, per_pair
