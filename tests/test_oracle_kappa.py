"""Pins of the oracle's detector-bounded plane range (the reading in which
Eq. 15's planes are those whose lines meet both detectors): the arc walk
against a brute-force scan of the pencil, with every plane's line computed
from the plane itself; the closed-form case of an epipole on the detector
(every plane of the pencil meets it); the arc ends passing through a
detector corner; containment of the object-sphere range at zero motion; and
the empty case."""
import math

import numpy as np
import pytest

import oracle
from oracle.ecc import as_rows, ecc_pair, pair_kappa_arc
from oracle.geometry import (detector_kappa_arc, epipolar_line, epipolar_planes, moved_projection, pencil,
                             pencil_basis_lines, source_position)
from paper_1806_02637_amd import inputs

N_SCAN = 40000  # brute-force samples over the half circle of plane angles


def _setup(P_a, P_b, th_a, th_b, R):
    Pa, Pb = moved_projection(as_rows(P_a), list(th_a)), moved_projection(as_rows(P_b), list(th_b))
    C_a, C_b = source_position(Pa), source_position(Pb)
    u1, u2, km = pencil(C_a, C_b, R)
    return Pa, Pb, C_a, C_b, u1, u2, km


def _meets(P, C_a, u1, u2, kappa, intr, W, H):
    """Whether each plane's line meets the detector, from the plane itself:
    E(kappa) -> Eqs. 13-14 -> |t| <= (W/2)|cos a| + (H/2)|sin a| in the
    line's normal form (the lookup's test)."""
    E = epipolar_planes(u1, u2, C_a, kappa)
    l, _ = epipolar_line(P, E)
    f, u0, v0 = intr
    l1, l2 = np.asarray(l[0]), np.asarray(l[1])
    l3c = np.asarray(l[2]) + l1 * u0 + l2 * v0
    r = np.hypot(l1, l2)
    return np.abs(l3c) <= 0.5 * W * np.abs(l1) + 0.5 * H * np.abs(l2) + 1e-12 * r


def _brute_arc(mask, grid):
    """Connected run of True around kappa = 0 on a periodic grid over
    [-pi/2, pi/2); None when the sample at 0 is False, 'full' when all
    are True, else the outermost True samples (lo, hi)."""
    n = len(grid)
    i0 = int(np.argmin(np.abs(grid)))
    if not mask[i0]:
        return None
    if mask.all():
        return "full"
    hi = i0
    while mask[(hi + 1) % n]:
        hi += 1
    lo = i0
    while mask[(lo - 1) % n]:
        lo -= 1
    step = math.pi / n
    return grid[i0] + (lo - i0) * step, grid[i0] + (hi - i0) * step


def _pairs_under_test():
    g = inputs.ScanGeometry(11, 160, 120, 2.4)  # views 20 degrees apart: 0 and 9 are opposite
    P, intr = g.projection_matrices(), g.intrinsics()
    R = g.default_object_radius()
    rng = np.random.default_rng(5)
    cases = []
    zero = np.zeros(6)
    for a, b in ((0, 1), (0, 4), (2, 9), (0, 9), (3, 10), (1, 6)):
        cases.append((g, P, intr, R, a, b, zero, zero))
        for _ in range(2):
            th_a = np.concatenate([rng.normal(0, 3, 3), rng.normal(0, 40, 3)])
            th_b = np.concatenate([rng.normal(0, 3, 3), rng.normal(0, 40, 3)])
            cases.append((g, P, intr, R, a, b, th_a, th_b))
    # one view sees every plane, the other's arc reaches past +-pi/2
    cases.append((g, P, intr, R, 0, 10, np.array([-3.717, -4.609, -2.289, 13.212, -60.577, -12.551]),
                  np.array([-0.796, 2.704, 1.073, 21.322, -39.23, -7.777])))
    cases.append((g, P, intr, R, 0, 10, np.array([-3.773, 8.446, -1.437, 94.464, -25.967, -44.129]),
                  np.array([1.249, 5.157, 0.805, -35.132, -80.473, -84.091])))
    # a view shifted 900 mm along the rotation axis: the isocentre leaves its detector
    cases.append((g, P, intr, R, 0, 4, zero, np.array([0, 0, 0, 0.0, 0.0, 900.0])))
    return cases


def test_arc_matches_brute_force_scan():
    grid = (np.arange(N_SCAN) + 0.5) * (math.pi / N_SCAN) - 0.5 * math.pi
    step = math.pi / N_SCAN
    seen = {"full": 0, "arc": 0, "none": 0, "wide": 0}
    for g, P, intr, R, a, b, th_a, th_b in _pairs_under_test():
        Pa, Pb, C_a, C_b, u1, u2, km = _setup(P[a], P[b], th_a, th_b, R)
        for Pv, iv in ((Pa, intr[a]), (Pb, intr[b])):
            La, Lb = pencil_basis_lines(Pv, C_a, u1, u2, iv)
            arc = detector_kappa_arc(La, Lb, g.W, g.H)
            brute = _brute_arc(_meets(Pv, C_a, u1, u2, grid, iv, g.W, g.H), grid)
            if brute is None:
                assert arc is None
                seen["none"] += 1
            elif brute == "full":
                assert arc == (-0.5 * math.pi, 0.5 * math.pi)
                seen["full"] += 1
            else:
                assert arc is not None and arc != (-0.5 * math.pi, 0.5 * math.pi)
                assert abs(arc[0] - brute[0]) <= step + 1e-12 and abs(arc[1] - brute[1]) <= step + 1e-12
                seen["arc"] += 1
        # the pair's arc is the intersection of the two views' arcs
        pa = pair_kappa_arc(Pa, Pb, C_a, u1, u2, (intr[a], intr[b], g.W, g.H))
        ma = _meets(Pa, C_a, u1, u2, grid, intr[a], g.W, g.H) & _meets(Pb, C_a, u1, u2, grid, intr[b], g.W, g.H)
        bp = _brute_arc(ma, grid)
        if bp is None:
            assert pa is None
        elif bp == "full":
            assert pa == (-0.5 * math.pi, 0.5 * math.pi)
        else:
            assert abs(pa[0] - bp[0]) <= step + 1e-12 and abs(pa[1] - bp[1]) <= step + 1e-12
            seen["wide"] += pa[0] < -0.5 * math.pi or pa[1] > 0.5 * math.pi
    assert min(seen.values()) > 0, seen


def _epipole_on_detector(P, C_other, intr, W, H):
    x = np.asarray(P, dtype=np.float64) @ np.append(np.asarray(C_other, dtype=np.float64), 1.0)
    if abs(x[2]) < 1e-12 * np.abs(x).max():
        return False
    u, v = x[0] / x[2] - intr[1], x[1] / x[2] - intr[2]
    return abs(u) <= 0.5 * W and abs(v) <= 0.5 * H


def test_full_arc_exactly_when_the_epipole_is_on_the_detector():
    """Every line through a point of the rectangle meets it, and for a point
    outside some line through it misses: so a view's arc is the whole half
    circle exactly when the other source projects onto its detector."""
    n_full = n_part = 0
    for g, P, intr, R, a, b, th_a, th_b in _pairs_under_test():
        Pa, Pb, C_a, C_b, u1, u2, km = _setup(P[a], P[b], th_a, th_b, R)
        for Pv, iv, Cother in ((Pa, intr[a], C_b), (Pb, intr[b], C_a)):
            La, Lb = pencil_basis_lines(Pv, C_a, u1, u2, iv)
            arc = detector_kappa_arc(La, Lb, g.W, g.H)
            full = arc == (-0.5 * math.pi, 0.5 * math.pi)
            assert full == _epipole_on_detector(Pv, Cother, iv, g.W, g.H)
            n_full += full
            n_part += not full
    assert n_full > 0 and n_part > 0


def test_arc_ends_pass_through_a_corner():
    """A finite arc end is a plane whose line touches the rectangle at a
    corner, in one of the two views."""
    corners = [(sx * 0.5, sy * 0.5) for sx in (-1, 1) for sy in (-1, 1)]
    n = 0
    for g, P, intr, R, a, b, th_a, th_b in _pairs_under_test():
        Pa, Pb, C_a, C_b, u1, u2, km = _setup(P[a], P[b], th_a, th_b, R)
        arc = pair_kappa_arc(Pa, Pb, C_a, u1, u2, (intr[a], intr[b], g.W, g.H))
        if arc is None or arc == (-0.5 * math.pi, 0.5 * math.pi):
            continue
        for k in arc:
            best = math.inf
            for Pv, iv in ((Pa, intr[a]), (Pb, intr[b])):
                E = epipolar_planes(u1, u2, C_a, np.array([k]))
                l, _ = epipolar_line(Pv, E)
                l1, l2, l3 = (float(np.ravel(x)[0]) for x in l)
                l3c = l3 + l1 * iv[1] + l2 * iv[2]
                for cx, cy in corners:
                    best = min(best, abs(l1 * cx * g.W + l2 * cy * g.H + l3c) / math.hypot(l1, l2))
            assert best <= 1e-6, (a, b, k, best)
            n += 1
    assert n > 0


def test_detector_arc_contains_the_object_range_at_zero_motion():
    """The default object sphere's shadow lies inside every detector, so
    every plane meeting the sphere meets both detectors."""
    g = inputs.ScanGeometry(24, 200, 150, 1.6)
    P, intr = g.projection_matrices(), g.intrinsics()
    R = g.default_object_radius()
    for a in range(0, 24, 3):
        for b in range(a + 1, 24, 4):
            Pa, Pb, C_a, C_b, u1, u2, km = _setup(P[a], P[b], np.zeros(6), np.zeros(6), R)
            lo, hi = pair_kappa_arc(Pa, Pb, C_a, u1, u2, (intr[a], intr[b], g.W, g.H))
            assert lo <= -km and hi >= km, (a, b, lo, hi, km)


def test_empty_arc_gives_zero_and_detector_mode_cost():
    """A pair whose plane at kappa = 0 misses a detector contributes e = 0
    with N = 0; elsewhere the detector range counts all K planes."""
    g = inputs.ScanGeometry(5, 64, 48, 4.0)
    P, intr = g.projection_matrices(), g.intrinsics()
    imgs = inputs.project(g, inputs.random_phantom(4, 6))
    grid = oracle.SinoGrid(g.W, g.H, 60, 61, 0.5)
    sino = oracle.FullSinograms.build(imgs, grid, intr)
    params = oracle.EccParams(16, g.default_object_radius(), kappa_range="detector")
    far = [0.0, 0.0, 0.0, 0.0, 0.0, 900.0]
    e, d, N = ecc_pair(as_rows(P[0]), as_rows(P[2]), [0.0] * 6, far, intr[0], intr[2], grid, sino, 0, 2, params)
    assert (e, d, N) == (0.0, 0.0, 0)
    e, d, N = ecc_pair(as_rows(P[0]), as_rows(P[2]), [0.0] * 6, [0.0] * 6, intr[0], intr[2], grid, sino, 0, 2,
                       params)
    assert N == 16 and e > 0.0
    e, g = oracle.ecc.ecc_pair_grad(as_rows(P[0]), as_rows(P[2]), [0.0] * 6, far, intr[0], intr[2], grid, sino, 0, 2,
                                    params)
    assert e == 0.0 and not g.any()


@pytest.mark.parametrize("motion", ["zero", "small", "wild"])
def test_detector_range_gradient_matches_central_differences(small16, motion):
    """The dual-number derivative, arc ends included (each end moves as the
    zero angle of the corner that fixes it), against FP64 central
    differences of the cost; h small enough that no cell boundary or arc
    decision changes.  'wild' motion gives pairs of every arc kind; at
    'zero' motion the circular orbit makes both views' arc ends equal, a
    kink whose central difference is the mean of the two branches."""
    s = small16
    n = s["geom"].n_views
    if motion == "zero":
        th = np.zeros((n, 6))
    elif motion == "small":
        th = inputs.random_motion(3, 1, n)[0]
    else:
        rng = np.random.default_rng(0)
        th = np.concatenate([rng.normal(0, 5, (n, 3)), rng.normal(0, 60, (n, 3))], 1)
    params = oracle.EccParams(s["params"].K, s["params"].R_mm, kappa_range="detector")
    cost, grad, _ = oracle.ecc_grad(s["P"], s["intr"], th, s["grid"], s["sino_c"], params)
    c_ref = oracle.ecc_cost(s["P"], s["intr"], th, s["grid"], s["sino_c"], params)[0]
    assert math.isclose(cost, c_ref, rel_tol=1e-12)
    h = 1e-5
    views = [0, 5, 12]
    fd = np.zeros((len(views), 6))
    for i, v in enumerate(views):
        for p in range(6):
            tp, tm = th.copy(), th.copy()
            tp[v, p] += h
            tm[v, p] -= h
            fd[i, p] = (oracle.ecc_cost(s["P"], s["intr"], tp, s["grid"], s["sino_c"], params)[0]
                        - oracle.ecc_cost(s["P"], s["intr"], tm, s["grid"], s["sino_c"], params)[0]) / (2 * h)
    # at the kink the central difference carries an O(h) term (the two
    # branches' curvatures differ), elsewhere O(h^2)
    bar = 3e-5 if motion == "zero" else 1e-6
    assert np.linalg.norm(fd - grad[views]) <= bar * np.linalg.norm(fd), np.abs(fd - grad[views]).max()
