"""The storage-rounding error model of the 16-bit sinogram forms, evaluated
with the oracle's own S values (shared by the precision and serving tests).

Unit roundoff u (2^-8 BF16, 2^-11 FP16, round to nearest even): each tap
carries noise of variance <= u^2 S^2 / 3, so a pair's mean of squared
differences is biased upwards by about (2 u^2 / 3) mean((S_a^2 + S_b^2) / 2)
and carries a zero-mean term of order 2 u sqrt(d mean(S^2) / N).  The
functions return the relative error of a hypothesis' total cost the model
predicts; tests assert 4x that plus the FP32 bar of 1e-5."""
import math

import numpy as np

from oracle.ecc import as_rows, lookup, pair_geometry, pair_list

U = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


def model_bound(P, intr, theta, grid, sino, params, u, pairs=None):
    """Per-hypothesis relative error bound of the storage-rounding model."""
    bias = 0.0
    noise2 = 0.0
    total = 0.0
    for a, b in pairs or pair_list(len(P)):
        g = pair_geometry(as_rows(P[a]), as_rows(P[b]), list(theta[a]), list(theta[b]), params)
        Sa, ha = lookup(g["l_a"], intr[a], grid, sino, a)
        Sb, hb = lookup(g["l_b"], intr[b], grid, sino, b)
        h = ha & hb
        if not h.any():
            continue
        ms = np.mean(0.5 * (Sa[h] ** 2 + Sb[h] ** 2))
        d = np.mean((Sa[h] - Sb[h]) ** 2)
        total += d
        bias += (2 * u * u / 3) * ms
        noise2 += (2 * u) ** 2 * d * ms / h.sum()
    return (bias + math.sqrt(noise2)) / total
