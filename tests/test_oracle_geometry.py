"""Pins of the oracle's projective-geometry steps (Eqs. 4, 5, 13, 14 and the
source construction) against independent routes: incidence identities,
numpy.linalg pseudo-inverses, cofactor matrices, null spaces and scipy
rotations."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import geometry as G
from oracle.ecc import as_rows, pair_geometry, pair_list
from paper_1806_02637_amd import inputs


def _rand_planes(rng, n):
    return [tuple(rng.normal(size=4)) for _ in range(n)]


def test_meet_matrix_annihilates_both_planes(rng):
    # a line built as the meet of planes a, b (Eq. 4) lies in both planes, so
    # its Eq. 5 matrix maps each of them to the zero point
    for a, b in zip(_rand_planes(rng, 20), _rand_planes(rng, 20)):
        LK = np.array(G.plucker_matrix(G.meet(a, b)), dtype=float)
        scale = np.abs(LK).max() * np.linalg.norm(a)
        assert np.abs(LK @ np.array(a)).max() <= 1e-12 * scale
        assert np.abs(LK @ np.array(b)).max() <= 1e-12 * scale
        assert np.allclose(LK, -LK.T)


def test_printed_eq5_sign_is_inconsistent_with_eq4(rng):
    # Eq. 5 exactly as printed (row 0 = (0, -p, -q, r), row 1 = (p, 0, s, -t))
    # does not annihilate the generating planes: this is why the oracle uses
    # the sign-corrected matrix.
    worst = 0.0
    for a, b in zip(_rand_planes(rng, 20), _rand_planes(rng, 20)):
        p, q, r, s, t, u = G.meet(a, b)
        printed = np.array([[0, -p, -q, r], [p, 0, s, -t], [q, -s, 0, u], [-r, t, -u, 0]])
        worst = max(worst, np.abs(printed @ np.array(a)).max() / (np.abs(printed).max() * np.linalg.norm(a)))
    assert worst > 1e-2


def test_meet_line_plane_is_the_common_point(rng):
    # the point L_K c lies on all three planes a, b, c
    for a, b, c in zip(_rand_planes(rng, 10), _rand_planes(rng, 10), _rand_planes(rng, 10)):
        X = np.array(G.meet_line_plane(G.meet(a, b), c))
        for pl in (a, b, c):
            assert abs(np.dot(pl, X)) <= 1e-12 * np.linalg.norm(pl) * np.linalg.norm(X)


def test_motion_matrix_matches_scipy_extrinsic_xyz(rng):
    for _ in range(10):
        th = np.concatenate([rng.uniform(-30, 30, 3), rng.normal(size=3) * 10])
        T = np.array(G.motion_matrix(list(th)), dtype=float)
        Rref = Rotation.from_euler("xyz", th[:3], degrees=True).as_matrix()
        assert np.allclose(T[:3, :3], Rref, atol=1e-14)
        assert np.allclose(T[:3, 3], th[3:])
        assert np.allclose(T[3], [0, 0, 0, 1])


@pytest.mark.parametrize("moved", [False, True])
def test_source_is_null_space_of_moved_projection(moved, rng):
    geom = inputs.ScanGeometry(12, 300, 200, 1.0)
    P = geom.projection_matrices()
    C0, _ = geom.frames()
    for lam in range(geom.n_views):
        th = list(rng.normal(size=6)) if moved else [0.0] * 6
        Pm = np.array(G.moved_projection(as_rows(P[lam]), th), dtype=float)
        C = np.array(G.source_position(Pm.tolist()), dtype=float)
        # P' C = 0 (homogeneous)
        assert np.abs(Pm @ np.append(C, 1.0)).max() <= 1e-9 * np.abs(Pm).max()
        # independent route: the moved source is T^-1 applied to the generator's source
        T = np.array(G.motion_matrix(th), dtype=float)
        expect = (np.linalg.inv(T) @ np.append(C0[lam], 1.0))[:3]
        assert np.allclose(C, expect, atol=1e-9)
        # and the right null vector from an SVD
        v = np.linalg.svd(Pm)[2][-1]
        assert np.allclose(C, v[:3] / v[3], atol=1e-8)


def _pairs_geometry(P, theta, params, pairs):
    for a, b in pairs:
        yield a, b, pair_geometry(as_rows(P[a]), as_rows(P[b]), list(theta[a]), list(theta[b]), params)


@pytest.fixture(scope="module")
def moved_scan():
    w = inputs.WORKLOADS["small16"]
    geom = w.geom
    P = geom.projection_matrices()
    theta = inputs.random_motion(77, 1, geom.n_views)[0]
    from oracle import EccParams

    params = EccParams(32, w.R_mm)
    pairs = pair_list(geom.n_views)[::7]
    return P, theta, params, pairs


def test_lines_equal_pseudo_inverse_lines(moved_scan):
    # The two routes give equal results (Sec. "Results"): Eq. 14's line is
    # the pseudo-inverse line l = (P P^T)^-1 P E up to a scale whose sign
    # does not change between views or planes.
    P, theta, params, pairs = moved_scan
    signs = set()
    for a, b, g in _pairs_geometry(P, theta, params, pairs):
        E = np.array([np.asarray(x, float) for x in g["E"]])  # [4, K]
        for Pm, l in ((g["Pa"], g["l_a"]), (g["Pb"], g["l_b"])):
            Pm = np.array(Pm, dtype=float)
            l = np.array([np.asarray(x, float) for x in l])  # [3, K]
            lp = np.linalg.pinv(Pm).T @ E
            cos = np.sum(l * lp, 0) / (np.linalg.norm(l, axis=0) * np.linalg.norm(lp, axis=0))
            assert np.all(np.abs(cos) >= 1 - 1e-12)
            signs.update(np.sign(cos).tolist())
    assert len(signs) == 1


def test_lines_pass_through_epipoles(moved_scan):
    P, theta, params, pairs = moved_scan
    for a, b, g in _pairs_geometry(P, theta, params, pairs):
        for Pm, l, Cother in ((g["Pa"], g["l_a"], g["C_b"]), (g["Pb"], g["l_b"], g["C_a"])):
            e = np.array(Pm, dtype=float) @ np.append(np.array(Cother, dtype=float), 1.0)
            l = np.array([np.asarray(x, float) for x in l])
            rel = np.abs(e @ l) / (np.linalg.norm(e) * np.linalg.norm(l, axis=0))
            assert rel.max() <= 1e-12


def test_back_projected_planes_coincide(moved_scan):
    # P_a^T l_a and P_b^T l_b are both the epipolar plane E (up to one common scale sign)
    P, theta, params, pairs = moved_scan
    for a, b, g in _pairs_geometry(P, theta, params, pairs):
        E = np.array([np.asarray(x, float) for x in g["E"]])
        planes = []
        for Pm, l in ((g["Pa"], g["l_a"]), (g["Pb"], g["l_b"])):
            l = np.array([np.asarray(x, float) for x in l])
            planes.append(np.array(Pm, dtype=float).T @ l)
        for pl in planes:
            cos = np.sum(pl * E, 0) / (np.linalg.norm(pl, axis=0) * np.linalg.norm(E, axis=0))
            assert np.all(cos >= 1 - 1e-12)  # same orientation as E (det M > 0 for every view)


def test_line_is_cofactor_times_normal(moved_scan):
    # [P L P^T]_x with L the line at infinity of normal n gives l = cof(M) n
    # (cofactor matrix from numpy: det(M) M^-T), with M the left 3x3 of P'
    P, theta, params, pairs = moved_scan
    for a, b, g in _pairs_geometry(P, theta, params, pairs):
        n = np.array([np.asarray(x, float) for x in g["E"][:3]])
        for Pm, l in ((g["Pa"], g["l_a"]), (g["Pb"], g["l_b"])):
            M = np.array(Pm, dtype=float)[:, :3]
            cof = np.linalg.det(M) * np.linalg.inv(M).T
            l = np.array([np.asarray(x, float) for x in l])
            ref = cof @ n
            assert np.allclose(l, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_pencil_planes_contain_both_sources_and_touch_sphere(moved_scan):
    P, theta, params, pairs = moved_scan
    for a, b, g in _pairs_geometry(P, theta, params, pairs):
        E = np.array([np.asarray(x, float) for x in g["E"]])
        n = E[:3]
        assert np.allclose(np.linalg.norm(n, axis=0), 1.0)
        for C in (g["C_a"], g["C_b"]):
            assert np.abs(np.append(np.array(C, float), 1.0) @ E).max() <= 1e-9
        # distance of every sampled plane from the isocentre <= R, the extreme
        # samples within one step of it (midpoint rule)
        dist = np.abs(E[3])
        assert dist.max() <= params.R_mm * (1 + 1e-12)
        km = float(g["kappa_max"])
        assert math.isclose(abs(g["kappa"][0]), km * (1 - 1.0 / params.K), rel_tol=1e-12)


def test_baseline_through_isocentre_picks_a_stable_pencil():
    # h < 1e-9: every plane of the pencil meets the sphere (kappa_max = pi/2)
    # and u2 is the part of z perpendicular to the baseline (x for a baseline
    # near z); rounding-level changes of the sources, which decide which
    # near-zero component of the baseline direction is smaller, must not
    # rotate the pencil
    ref = None
    for dy, dz in ((0.0, 0.0), (1e-13, -2e-13), (-3e-13, 1e-13), (2e-13, 2e-13)):
        Ca, Cb = [785.0, 0.0, 0.0], [-785.0, dy, dz]
        u1, u2, km = G.pencil(Ca, Cb, 90.0)
        assert km == 0.5 * math.pi
        u = np.array([u1, u2], dtype=float)
        assert np.allclose(u @ u.T, np.eye(2), atol=1e-14)
        assert np.allclose(u2, [0, 0, 1], atol=1e-12)
        if ref is None:
            ref = u
        assert np.allclose(u, ref, atol=1e-12)
    u1, u2, km = G.pencil([0.0, 1e-13, 785.0], [0.0, 0.0, -785.0], 90.0)
    assert km == 0.5 * math.pi and np.allclose(u2, [1, 0, 0], atol=1e-12)
