"""Epipolar-consistency cost, FP64, one view pair at a time (test
infrastructure).

Steps, in the paper's order:
* moved projection P' = P T(theta) and its source (end of "Optimized
  Algorithm"; "Optimization");
* pencil of epipolar planes about the baseline, kappa -> E^kappa
  ("Epipolar Consistency", Eq. 3);
* epipolar lines without pseudo-inverse, Eqs. 13-14;
* lookup of S_lam, Eq. 1's intermediate function, stored per view beforehand, along each line
  (Eq. 1, "Epipolar Consistency");
* d = mean over planes hitting both detectors of (S_a - S_b)^2 (Eq. 15),
  e = d / (1 + d / c) (Eq. 16), cost = sum over pairs a < b of e (Eq. 17).

Every function is generic over floats and ``Dual`` numbers; ``grad.py``
differentiates this same code.

Readings (the paper is silent):
* lookup geometry: line l = (l1, l2, l3) in pixels, centred offset
  l3c = l3 + l1 u0 + l2 v0, alpha = atan2(l2, l1), t = -l3c / |(l1, l2)|;
  alpha is folded into [0, pi) with t -> -t and the value negated (odd
  symmetry of the derivative sinogram);
* "hits the detector": |t| <= (W/2)|cos alpha| + (H/2)|sin alpha|, the closed
  rectangle of pixel edges; N_kappa counts planes hitting both detectors and
  d = 0 when none does;
* bilinear interpolation in (alpha / dalpha, (t + t_max) / dt) on the floor
  cell, taps beyond the t grid read as zero, the last alpha row interpolates
  into the symmetric pad row;
* S = sign * (1 + t^2 / f^2) * interpolated value (Grangeat's weight on a flat
  detector, see ``sinogram.py``);
* pairs a < b only, c = inf meaning e = d;
* sampled arc of the pencil: the planes meeting the object sphere
  (``pencil``), or, the other reading of which planes count, the connected
  arc around kappa = 0 whose lines meet both detectors (kappa_range =
  "detector", ``detector_kappa_arc``); K midpoint samples either way, and a
  pair whose arc is empty contributes e = 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .dual import Dual, ops, value
from .geometry import (arc_end, detector_kappa_arc, epipolar_line, epipolar_planes, moved_projection, pencil,
                       pencil_basis_lines, plane_angles, plane_angles_between, source_position)
from .sinogram import SinoGrid


@dataclass(frozen=True)
class EccParams:
    """K planes per pair; R_mm the object-sphere radius; c Eq. 16's Cauchy
    parameter.  kappa_range picks the sampled arc of the pencil: "object",
    the planes meeting the sphere of radius R_mm about the isocentre, or
    "detector", the planes around kappa = 0 whose lines meet both detectors
    (R_mm unused)."""
    K: int
    R_mm: float
    c: float = math.inf
    kappa_range: str = "object"


def pair_list(n_views: int):
    """Pairs (a, b), a < b, in row-major triangle order."""
    return [(a, b) for a in range(n_views) for b in range(a + 1, n_views)]


def pair_index(a: int, b: int, n_views: int) -> int:
    return a * n_views - a * (a + 1) // 2 + (b - a - 1)


def as_rows(P):
    return [[float(P[i][j]) for j in range(4)] for i in range(3)]


def _taps(sino, view, m, k, n_t):
    ok = (k >= 0) & (k < n_t)
    out = np.zeros(m.shape, dtype=np.float64)
    if ok.any():
        out[ok] = sino.cells(view, m[ok], k[ok])
    return out


def lookup(l, intr, grid: SinoGrid, sino, view):
    """Value of S_lam along each image line l and whether the line hits the
    detector.  Returns (S, hit)."""
    l1, l2, l3 = l
    f, u0, v0 = (float(x) for x in intr)
    l3c = l3 + l1 * u0 + l2 * v0
    r = ops.sqrt(l1 * l1 + l2 * l2)
    ok = value(r) > 0.0
    r = ops.where(ok, r, 1.0)
    alpha = ops.arctan2(l2, l1)
    t = -l3c / r
    av = value(alpha)
    neg = av < 0.0
    big = av >= math.pi
    flip = neg | big
    alpha = ops.where(neg, alpha + math.pi, ops.where(big, alpha - math.pi, alpha))
    t = ops.where(flip, -t, t)
    sign = np.where(flip, -1.0, 1.0)
    av, tv = value(alpha), value(t)
    hit = ok & (np.abs(tv) <= 0.5 * grid.W * np.abs(np.cos(av)) + 0.5 * grid.H * np.abs(np.sin(av)))

    a = alpha / grid.dalpha
    m = np.clip(np.floor(value(a)), 0, grid.n_alpha - 1).astype(np.int64)
    fa = a - m
    tau = (t + grid.t_max) / grid.dt
    tau_v = np.where(np.isfinite(value(tau)), value(tau), -10.0)
    k = np.clip(np.floor(tau_v), -10, grid.n_t + 10).astype(np.int64)
    ft = tau - k
    s00 = _taps(sino, view, m, k, grid.n_t)
    s01 = _taps(sino, view, m, k + 1, grid.n_t)
    s10 = _taps(sino, view, m + 1, k, grid.n_t)
    s11 = _taps(sino, view, m + 1, k + 1, grid.n_t)
    interp = (1.0 - fa) * ((1.0 - ft) * s00 + ft * s01) + fa * ((1.0 - ft) * s10 + ft * s11)
    weight = 1.0 + t * t / (f * f)
    S = sign * weight * interp
    return S, hit


ARC_TIE = 1e-9  # rad: two views' arc ends this close are one kink


def pair_kappa_arc(Pa, Pb, C_a, u1, u2, detector):
    """The arc both detectors see: the part around kappa = 0 of the
    intersection of the two views' ``detector_kappa_arc``; None when it is
    empty.  A view that sees every plane leaves the other view's arc as it
    is (that arc may reach past +-pi/2); two partial arcs, each shorter than
    pi and containing 0, meet around 0 in [max of the lows, min of the
    highs].  detector = (intr_a, intr_b, W, H).

    With Dual geometry the ends are Dual: each is the zero angle of the
    corner that fixes it.  Where the two views' ends agree within ARC_TIE
    (a circular orbit without motion makes them equal) the end is a kink
    between two smooth branches; its derivative is taken as their mean, the
    value central differences give there."""
    intr_a, intr_b, W, H = detector
    full = (-0.5 * math.pi, 0.5 * math.pi)
    arcs = []
    for P, intr in ((Pa, intr_a), (Pb, intr_b)):
        La, Lb = pencil_basis_lines(P, C_a, u1, u2, intr)
        arc = detector_kappa_arc(La, Lb, W, H, ends=True)
        if arc is None:
            return None
        arcs.append((arc, La, Lb))
    (a, La_a, Lb_a), (b, La_b, Lb_b) = arcs
    dual = isinstance(La_a[0], Dual)

    def end(i, view):  # end i (0 low, 1 high) of one view's arc
        arc, La, Lb = arcs[view]
        src = arc[2 + i]
        return arc[i] if (src is None or not dual) else arc_end(La, Lb, W, H, src)

    def pick(i, better):
        if a[:2] == full:
            return end(i, 1)
        if b[:2] == full:
            return end(i, 0)
        if abs(a[i] - b[i]) <= ARC_TIE:
            return 0.5 * (end(i, 0) + end(i, 1)) if dual else better(a[i], b[i])
        return end(i, 0) if better(a[i], b[i]) == a[i] else end(i, 1)

    return pick(0, max), pick(1, min)


def pair_geometry(P_a, P_b, theta_a, theta_b, params: EccParams, detector=None):
    """Moved projections, sources, sampled angles, planes and both lines.
    With params.kappa_range == "detector" the angles sample the arc both
    detectors see (``detector`` = (intr_a, intr_b, W, H) is then required);
    kappa is None when that arc is empty."""
    Pa = moved_projection(P_a, theta_a)
    Pb = moved_projection(P_b, theta_b)
    C_a = source_position(Pa)
    C_b = source_position(Pb)
    u1, u2, kappa_max = pencil(C_a, C_b, params.R_mm)
    if params.kappa_range == "object":
        kappa = plane_angles(kappa_max, params.K)
    elif params.kappa_range == "detector":
        arc = pair_kappa_arc(Pa, Pb, C_a, u1, u2, detector)
        if arc is None:
            return dict(Pa=Pa, Pb=Pb, C_a=C_a, C_b=C_b, u1=u1, u2=u2, kappa_max=kappa_max, kappa=None, E=None,
                        l_a=None, l_b=None, arc=None)
        kappa = plane_angles_between(arc[0], arc[1], params.K)
    else:
        raise ValueError(f"unknown kappa_range {params.kappa_range!r}")
    E = epipolar_planes(u1, u2, C_a, kappa)
    l_a, _ = epipolar_line(Pa, E)
    l_b, _ = epipolar_line(Pb, E)
    return dict(Pa=Pa, Pb=Pb, C_a=C_a, C_b=C_b, u1=u1, u2=u2, kappa_max=kappa_max, kappa=kappa, E=E,
                l_a=l_a, l_b=l_b)


def inconsistency(S_a, S_b, hit):
    """Eq. 15: d = (1/N) sum over planes hitting both detectors of (S_a - S_b)^2."""
    N = int(np.count_nonzero(hit))
    if N == 0:
        return 0.0, 0
    diff = S_a - S_b
    return ops.sum(diff * diff, mask=hit) / float(N), N


def robust(d, c):
    """Eq. 16 (Cauchy): e = d / (1 + d / c); c = inf gives e = d."""
    if math.isinf(c):
        return d
    return d / (1.0 + d / c)


def ecc_pair(P_a, P_b, theta_a, theta_b, intr_a, intr_b, grid: SinoGrid, sino, a, b, params: EccParams):
    """(e_ab, d_ab, N_kappa) for one view pair."""
    g = pair_geometry(P_a, P_b, theta_a, theta_b, params, (intr_a, intr_b, grid.W, grid.H))
    if g["kappa"] is None:
        return robust(0.0, params.c), 0.0, 0
    S_a, hit_a = lookup(g["l_a"], intr_a, grid, sino, a)
    S_b, hit_b = lookup(g["l_b"], intr_b, grid, sino, b)
    d, N = inconsistency(S_a, S_b, hit_a & hit_b)
    return robust(d, params.c), d, N


def ecc_cost(P, intr, theta, grid: SinoGrid, sino, params: EccParams, pairs=None):
    """Total cost (Eq. 17's sum over a < b) for one motion hypothesis theta
    [N, 6] and the per-pair (e, d, N) arrays, in ``pairs`` order (default: all
    pairs, row-major triangle)."""
    n = len(P)
    if pairs is None:
        pairs = pair_list(n)
    e = np.zeros(len(pairs))
    d = np.zeros(len(pairs))
    N = np.zeros(len(pairs), dtype=np.int64)
    for i, (a, b) in enumerate(pairs):
        ei, di, Ni = ecc_pair(as_rows(P[a]), as_rows(P[b]), [float(x) for x in theta[a]],
                              [float(x) for x in theta[b]], intr[a], intr[b], grid, sino, a, b, params)
        e[i], d[i], N[i] = float(value(ei)), float(value(di)), Ni
    return float(e.sum()), e, d, N


def ecc_pair_grad(P_a, P_b, theta_a, theta_b, intr_a, intr_b, grid, sino, a, b, params: EccParams):
    """e_ab and its exact derivative w.r.t. (theta_a, theta_b) (12 values).
    With the detector-bounded range the arc's ends move with theta through
    the zero angles of the corners that fix them; that motion is part of the
    derivative (the choice of corner is held, as the choice of cell is)."""
    ta = [Dual.variable(theta_a[i], i, 12) for i in range(6)]
    tb = [Dual.variable(theta_b[i], 6 + i, 12) for i in range(6)]
    e, _, _ = ecc_pair(P_a, P_b, ta, tb, intr_a, intr_b, grid, sino, a, b, params)
    if not isinstance(e, Dual):
        return float(e), np.zeros(12)
    return float(e.v), np.array(e.d, dtype=np.float64)
