"""Sanity of the synthetic scan generator (inputs shared by oracle and engine)."""
import math

import numpy as np

from paper_1806_02637_amd import inputs


def test_projection_matrices_match_the_stated_orbit():
    g = inputs.ScanGeometry(9, 64, 48, 1.5)
    P = g.projection_matrices()
    C, R = g.frames()
    assert np.allclose(np.linalg.norm(C, axis=1), inputs.SID_MM)
    ang = np.rad2deg(np.arctan2(C[:, 1], C[:, 0]))
    assert np.allclose(ang[[0, -1]], [0.0, 200.0 - 360.0])
    for i in range(g.n_views):
        assert np.allclose(P[i] @ np.append(C[i], 1.0), 0.0, atol=1e-9)
        iso = P[i] @ np.array([0.0, 0.0, 0.0, 1.0])
        assert np.allclose(iso[:2] / iso[2], [g.u0, g.v0])  # isocentre -> principal point
        assert np.linalg.det(P[i][:, :3]) > 0  # one detector handedness for all views
        assert np.allclose(R[i] @ R[i].T, np.eye(3)) and math.isclose(np.linalg.det(R[i]), 1.0)


def test_sphere_projection_is_the_chord_length():
    g = inputs.ScanGeometry(3, 33, 33, 4.0)
    img = inputs.project(g, inputs.sphere_phantom(50.0, 1.0), views=[1])[0]
    # central ray passes through the centre: chord 2 r
    assert math.isclose(float(img[16, 16]), 100.0, rel_tol=1e-6)
    # ray through pixel (i, j): distance of the ray from the centre gives the chord
    f = g.f_px
    for i, j in [(20, 16), (16, 25), (22, 9)]:
        x = np.array([(i - g.u0) / f, (j - g.v0) / f, 1.0])
        sin_t = np.linalg.norm(x[:2]) / np.linalg.norm(x)
        dist = inputs.SID_MM * sin_t
        chord = 2 * math.sqrt(max(0.0, 50.0 ** 2 - dist ** 2))
        assert math.isclose(float(img[j, i]), chord, rel_tol=1e-5, abs_tol=1e-4)


def test_phantom_draws_are_seeded_and_contained():
    a = inputs.random_phantom(2, 30)
    b = inputs.random_phantom(2, 30)
    assert np.array_equal(a.centers, b.centers) and a.n == 30
    assert np.all((a.semi_axes >= 10) & (a.semi_axes <= 60))
    assert np.all(np.linalg.norm(a.centers, axis=1) <= 60)
    c = inputs.random_phantom(1, 10, contained_radius=90.0)
    assert np.all(np.linalg.norm(c.centers, axis=1) + c.semi_axes.max(1) <= 90.0)
    for Q in a.axes:
        assert np.allclose(Q @ Q.T, np.eye(3), atol=1e-12)


def test_motion_hypotheses():
    th = inputs.random_motion(1002, 4, 10)
    assert th.shape == (4, 10, 6)
    assert np.array_equal(th[1], inputs.random_motion(1002, 4, 10)[1])
    big = inputs.random_motion(7, 64, 500)
    assert abs(big[..., :3].std() - 0.5) < 0.01 and abs(big[..., 3:].std() - 1.0) < 0.02


def test_workload_table():
    w = inputs.WORKLOADS["full496"]
    assert w.n_pairs == 122760 and w.K == 512 and (w.n_alpha, w.n_t) == (768, 1024)
    assert inputs.WORKLOADS["mid248"].n_pairs == 30628
    assert abs(inputs.WORKLOADS["small16"].R_mm - 94.68) < 0.01
    assert abs(inputs.WORKLOADS["mid248"].R_mm - 91.19) < 0.01
    assert [s.geom.n_views for s in inputs.serve_workloads()] == list(inputs.SERVE_VIEW_COUNTS)


def test_smooth_motion_recipe():
    from paper_1806_02637_amd import inputs

    th = inputs.smooth_motion(77, 496, peak=2.0, params=(5,))
    assert th.shape == (496, 6)
    assert np.all(th[:, :5] == 0.0)
    assert abs(th[:, 5].mean()) < 1e-12 and abs(np.abs(th[:, 5]).max() - 2.0) < 1e-12
    # smooth: view-to-view steps far below the peak
    assert np.abs(np.diff(th[:, 5])).max() < 0.1
    np.testing.assert_array_equal(th, inputs.smooth_motion(77, 496, peak=2.0, params=(5,)))
    two = inputs.smooth_motion(3, 100, peak=1.0, params=(0, 4))
    assert np.all(two[:, [1, 2, 3, 5]] == 0.0) and np.all(np.abs(two[:, [0, 4]]).max(axis=0) > 0.999)
