"""Projective-geometry steps of the method, FP64, written out component by
component (test infrastructure; generic over floats, NumPy arrays and
``Dual`` so the same code yields exact derivatives).

Objects are plain Python sequences: a plane or point is 4 scalars, a line is
the 6 Pluecker coordinates (p, q, r, s, t, u), matrices are lists of rows.
Each scalar may be a float, an array (one entry per sampled plane) or a Dual.

Readings of the paper taken here (it is silent or inconsistent):
* Eq. 5 as printed puts -p in row 0 and +p in row 1; with (p..u) from Eq. 4
  that matrix does not annihilate the two planes the line came from.  The
  matrix used is the one that does: row 0 = (0, p, -q, r), row 1 =
  (-p, 0, s, -t), rows 2-3 as printed.
* Rigid motion: T(theta) = [[Rz(rz) Ry(ry) Rx(rx), (tx, ty, tz)], [0, 1]],
  angles in degrees, applied as P' = P T (the composition P_lam T_lam of the
  "Optimization" subsection).
"""
from __future__ import annotations

import math

from .dual import ops

PLANE_AT_INFINITY = (0.0, 0.0, 0.0, 1.0)  # the plane pi_inf of the "Projective Geometry" subsection


def meet(a, b):
    """Eq. 4: Pluecker coordinates of the line common to planes a and b."""
    ax, ay, az, aw = a
    bx, by, bz, bw = b
    p = az * bw - aw * bz
    q = ay * bw - aw * by
    r = ay * bz - az * by
    s = ax * bw - aw * bx
    t = ax * bz - az * bx
    u = ax * by - ay * bx
    return (p, q, r, s, t, u)


def plucker_matrix(L):
    """Eq. 5 (sign of the p entries corrected, see module header): the 4x4
    antisymmetric L_K whose product with a plane is the point where the line
    pierces that plane."""
    p, q, r, s, t, u = L
    return [
        [0.0, p, -q, r],
        [-p, 0.0, s, -t],
        [q, -s, 0.0, u],
        [-r, t, -u, 0.0],
    ]


def matvec(M, x):
    return [sum(M[i][j] * x[j] for j in range(len(x))) for i in range(len(M))]


def matmul(A, B):
    n, k, m = len(A), len(B), len(B[0])
    return [[sum(A[i][j] * B[j][c] for j in range(k)) for c in range(m)] for i in range(n)]


def transpose(A):
    return [[A[i][j] for i in range(len(A))] for j in range(len(A[0]))]


def meet_line_plane(L, plane):
    """Eq. 5: point common to line L and a plane, x = L_K p."""
    return matvec(plucker_matrix(L), plane)


def motion_matrix(theta):
    """4x4 rigid transform T(theta), theta = (rx, ry, rz [deg], tx, ty, tz [mm])."""
    rx, ry, rz = (theta[i] * (math.pi / 180.0) for i in range(3))
    cx, sx = ops.cos(rx), ops.sin(rx)
    cy, sy = ops.cos(ry), ops.sin(ry)
    cz, sz = ops.cos(rz), ops.sin(rz)
    Rx = [[1.0, 0.0, 0.0], [0.0, cx, -sx], [0.0, sx, cx]]
    Ry = [[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]]
    Rz = [[cz, -sz, 0.0], [sz, cz, 0.0], [0.0, 0.0, 1.0]]
    Rm = matmul(Rz, matmul(Ry, Rx))
    return [
        [Rm[0][0], Rm[0][1], Rm[0][2], theta[3]],
        [Rm[1][0], Rm[1][1], Rm[1][2], theta[4]],
        [Rm[2][0], Rm[2][1], Rm[2][2], theta[5]],
        [0.0, 0.0, 0.0, 1.0],
    ]


def moved_projection(P, theta):
    """P' = P T(theta) ("Optimization" subsection)."""
    return matmul(P, motion_matrix(theta))


def source_position(P):
    """Source of a 3x4 projection matrix (end of the "Optimized Algorithm"
    subsection): the rows of P are planes through the source; the line where
    rows 0 and 1 meet (Eq. 4) pierces row 2 (Eq. 5) at the source.  Returned
    dehomogenised (3 components)."""
    L = meet(P[0], P[1])
    X = meet_line_plane(L, P[2])
    return [X[0] / X[3], X[1] / X[3], X[2] / X[3]]


def dot3(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def cross3(a, b):
    return [a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]]


def _value(x):
    return x.v if hasattr(x, "v") else x


def pencil(C_a, C_b, R_mm):
    """Pencil of epipolar planes about the baseline C_a C_b (the angle ->
    plane mapping of the "Epipolar Consistency" subsection, whose basis and
    range the paper leaves open).  Returns (u1, u2, kappa_max):
    n(kappa) = cos(kappa) u1 + sin(kappa) u2 is the unit normal of the plane
    at angle kappa; u2 points from the baseline towards the isocentre, so the
    plane lies h |sin kappa| from the isocentre (h = baseline-isocentre
    distance) and the planes meeting the object sphere of radius R_mm are
    |kappa| <= asin(min(1, R/h))."""
    b = [C_b[i] - C_a[i] for i in range(3)]
    nb = ops.sqrt(dot3(b, b))
    bh = [b[i] / nb for i in range(3)]
    ca_b = dot3(C_a, bh)
    w = [-C_a[i] + ca_b * bh[i] for i in range(3)]
    h = ops.sqrt(dot3(w, w))
    if float(_value(h)) < 1e-9:
        # baseline through the isocentre: every plane of the pencil meets the
        # sphere, kappa covers the whole half circle and u2 only fixes where
        # the samples sit.  u2 = the part of the z axis (the orbit's rotation
        # axis) perpendicular to the baseline, or of the x axis for a
        # baseline within 60 degrees of z: a choice no rounding can tip
        bv = [float(_value(x)) for x in bh]
        e = [0.0, 0.0, 1.0] if abs(bv[2]) < 0.5 else [1.0, 0.0, 0.0]
        eb = dot3(e, bh)
        w = [e[i] - eb * bh[i] for i in range(3)]
        nw = ops.sqrt(dot3(w, w))
        u2 = [w[i] / nw for i in range(3)]
        kappa_max = math.pi / 2
    else:
        u2 = [w[i] / h for i in range(3)]
        ratio = R_mm / h
        kappa_max = ops.arcsin(ratio) if float(_value(ratio)) < 1.0 else math.pi / 2
    u1 = cross3(bh, u2)
    return u1, u2, kappa_max


def plane_angles(kappa_max, K):
    """Midpoint sampling of [-kappa_max, kappa_max] with K planes,
    kappa_k = -kappa_max + (k + 1/2) * 2 kappa_max / K, k = 0..K-1 (Eq. 15's
    sum read as K terms)."""
    import numpy as np

    frac = (np.arange(K, dtype=np.float64) + 0.5) * (2.0 / K) - 1.0
    return kappa_max * frac


def plane_angles_between(lo, hi, K):
    """Midpoint sampling of an arbitrary arc [lo, hi] with K planes,
    kappa_k = lo + (k + 1/2) (hi - lo) / K."""
    import numpy as np

    frac = (np.arange(K, dtype=np.float64) + 0.5) / K
    return lo + ((hi - lo) * frac)


def pencil_basis_lines(P, C_a, u1, u2, intr):
    """Image lines, offset about the principal point (l3 + l1 u0 + l2 v0), of
    the pencil's two basis planes: normal u1 (kappa = 0) and normal u2
    (kappa = pi/2), both through C_a.  Eqs. 13-14 are linear in the plane and
    the plane at kappa is cos(kappa) E(u1) + sin(kappa) E(u2), so its line is
    cos(kappa) La + sin(kappa) Lb."""
    f, u0, v0 = (float(x) for x in intr)
    out = []
    for n in (u1, u2):
        E = [n[0], n[1], n[2], -dot3(n, C_a)]
        l, _ = epipolar_line(P, E)
        out.append([l[0], l[1], l[2] + l[0] * u0 + l[1] * v0])
    return out[0], out[1]


def detector_kappa_arc(La, Lb, W, H, ends=False):
    """The arc of plane angles around kappa = 0 whose lines meet the closed
    detector rectangle [-W/2, W/2] x [-H/2, H/2] (coordinates about the
    principal point).  Returns (lo, hi) with lo <= 0 <= hi, None when the
    plane at kappa = 0 misses the detector, and (-pi/2, pi/2) when every
    plane meets it (the epipole lies on the detector).

    A line meets the rectangle exactly when its value l . (x, y, 1) at the
    four corners is not of one strict sign.  At corner c that value is
    A_c cos(kappa) + B_c sin(kappa), which changes sign only at its zeros
    kappa = atan2(-A_c, B_c) (mod pi); between consecutive zeros the
    decision is constant.  The arc is found by stepping from 0 through the
    sorted zeros in each direction until an interval misses.  Plain floats
    (the values of Dual numbers are taken).

    With ends=True, also returns for each end the (corner, m) for which the
    end equals atan2(-A_c, B_c) + m pi (None for the fixed ends of a whole
    half circle), so that a caller can follow the ends' dependence on the
    lines."""
    La = [float(_value(x)) for x in La]
    Lb = [float(_value(x)) for x in Lb]
    corners = detector_corners(W, H)
    AB = [(La[0] * x + La[1] * y + La[2], Lb[0] * x + Lb[1] * y + Lb[2]) for x, y in corners]

    def meets(k):
        c, s = math.cos(k), math.sin(k)
        v = [A * c + B * s for A, B in AB]
        return min(v) <= 0.0 <= max(v)

    if not meets(0.0):
        return None
    raw = [math.atan2(-A, B) for A, B in AB]
    # zero of each corner, into [-pi/2, pi/2), with its corner
    zeros = sorted(((r + 0.5 * math.pi) % math.pi - 0.5 * math.pi, c) for c, r in enumerate(raw))

    def walk(steps):
        prev, src = 0.0, None
        for k, c in steps:
            if not meets(0.5 * (prev + k)):
                return prev, src
            prev, src = k, c
        return None

    up = walk([(z, c) for z, c in zeros if z > 0.0] + [(z + math.pi, c) for z, c in zeros if z <= 0.0])
    if up is None:
        return (-0.5 * math.pi, 0.5 * math.pi, None, None) if ends else (-0.5 * math.pi, 0.5 * math.pi)
    down = walk([(z, c) for z, c in reversed(zeros) if z < 0.0] +
                [(z - math.pi, c) for z, c in reversed(zeros) if z >= 0.0])
    (hi, c_hi), (lo, c_lo) = up, down
    if not ends:
        return lo, hi

    def end(k, c):
        return None if c is None else (c, round((k - raw[c]) / math.pi))

    return lo, hi, end(lo, c_lo), end(hi, c_hi)


def detector_corners(W, H):
    """The four corners of the detector rectangle about the principal point."""
    return [(sx * 0.5 * W, sy * 0.5 * H) for sx in (-1.0, 1.0) for sy in (-1.0, 1.0)]


def arc_end(La, Lb, W, H, end):
    """An arc end given as (corner, m) by ``detector_kappa_arc``, as
    atan2(-A_c, B_c) + m pi of the lines La, Lb (generic over Dual)."""
    c, m = end
    x, y = detector_corners(W, H)[c]
    A = La[0] * x + La[1] * y + La[2]
    B = Lb[0] * x + Lb[1] * y + Lb[2]
    return ops.arctan2(-A, B) + m * math.pi


def epipolar_planes(u1, u2, C_a, kappa):
    """E^kappa = (n, -n . C_a) for every sampled angle (homogeneous planes)."""
    c, s = ops.cos(kappa), ops.sin(kappa)
    n = [c * u1[i] + s * u2[i] for i in range(3)]
    return [n[0], n[1], n[2], -dot3(n, C_a)]


def epipolar_line(P, E):
    """Eqs. 13-14: L = meet(E, pi_inf); [l]_x = P L_K P^T; l = (S12, S20, S01)."""
    L = meet(E, PLANE_AT_INFINITY)
    S = matmul(matmul(P, plucker_matrix(L)), transpose(P))
    return [S[1][2], S[2][0], S[0][1]], S
