"""Pins of the oracle's FDK reconstruction (the check the paper makes of a
compensated scan, "Experiments"): the sampled ramp filter's frequency
response, Parker's weights summing to one over conjugate rays of this
orbit (with the fan-angle sign taken from the geometry itself), the
reconstructed density of a uniform sphere and the centroid of an
off-centre ellipsoid from analytic projections, and motion compensation
through P' = P T(theta) undoing a known motion."""
import math

import numpy as np

from oracle import fdk
from oracle.geometry import moved_projection
from paper_1806_02637_amd import inputs


def test_ramp_kernel_frequency_response():
    # the sampled Ram-Lak kernel's DTFT is |w| / (2 pi) on [-pi, pi]
    h = fdk.ramp_kernel(20000)
    n = np.arange(-20000, 20001)
    for w in (0.0, 0.3, 1.0, 2.0, math.pi):
        resp = float(np.sum(h * np.cos(w * n)))
        assert abs(resp - abs(w) / (2 * math.pi)) <= 2e-5, (w, resp)
    assert h[20000] == 0.25 and h[20002] == 0.0 and abs(h[20001] + 1 / math.pi ** 2) < 1e-15


def _conjugate(g: inputs.ScanGeometry, beta: float, u: float):
    """The other end of the midplane ray through column u at orbit angle
    beta, and that ray's column there, from the orbit's geometry."""
    D = g.sid_mm
    C = D * np.array([math.cos(beta), math.sin(beta)])
    e_u = np.array([-math.sin(beta), math.cos(beta)])
    e_w = -C / D
    d = e_w + (u - g.u0) / g.f_px * e_u
    d /= np.linalg.norm(d)
    s = -2.0 * C.dot(d)
    C2 = C + s * d
    beta2 = math.atan2(C2[1], C2[0]) % (2 * math.pi)
    e_u2 = np.array([-math.sin(beta2), math.cos(beta2)])
    e_w2 = -C2 / D
    back = -d  # the same line travelled from the other source
    u2 = g.u0 + g.f_px * back.dot(e_u2) / back.dot(e_w2)
    return beta2, u2


def test_parker_weights_sum_to_one_over_conjugate_rays():
    g = inputs.ScanGeometry(200, 160, 64, 2.0)
    arc = math.radians(g.arc_deg)
    delta = 0.5 * (arc - math.pi)
    rng = np.random.default_rng(3)
    n_pairs = 0
    for _ in range(400):
        beta = rng.uniform(0, arc)
        u = rng.uniform(0, g.W - 1)
        gamma = -math.atan((u - g.u0) / g.f_px)
        beta2, u2 = _conjugate(g, beta, u)
        gamma2 = -math.atan((u2 - g.u0) / g.f_px)
        # the convention the weights assume: conjugate at (beta + pi + 2 gamma, -gamma)
        assert abs(((beta + math.pi + 2 * gamma) - beta2 + math.pi) % (2 * math.pi) - math.pi) < 1e-9
        assert abs(gamma2 + gamma) < 1e-9
        w = fdk.parker_weights(beta, np.array([gamma]), delta)[0]
        if beta2 <= arc:
            w2 = fdk.parker_weights(beta2, np.array([gamma2]), delta)[0]
            assert abs(w + w2 - 1.0) < 1e-12
            n_pairs += 1
        else:
            assert w == 1.0
    assert n_pairs > 20


def _small_scan(n_views=121):
    g = inputs.ScanGeometry(n_views, 96, 96, 2.4)
    return g, g.projection_matrices(), g.intrinsics(), g.orbit_angles(), math.radians(g.arc_deg)


def test_uniform_sphere_density():
    g, P, intr, betas, arc = _small_scan()
    imgs = inputs.project(g, inputs.sphere_phantom(40.0, 0.5))
    vol = fdk.Volume(32, 32, 32, 3.0)
    rec = fdk.fdk(imgs, P, intr, betas, arc, g.sid_mm, vol)
    x, y, z = vol.centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    inside, outside = rec[r < 30.0], rec[r > 46.0]
    assert abs(inside.mean() - 0.5) < 2e-3 and inside.std() < 5e-3
    assert abs(outside.mean()) < 5e-3


def test_off_centre_ellipsoid_centroid_and_mass():
    g, P, intr, betas, arc = _small_scan()
    c0, a = np.array([18.0, -12.0, 9.0]), np.array([12.0, 9.0, 7.0])
    ph = inputs.Phantom(c0[None], a[None], np.eye(3)[None], np.array([1.0]))
    imgs = inputs.project(g, ph)
    vol = fdk.Volume(32, 32, 32, 3.0)
    rec = fdk.fdk(imgs, P, intr, betas, arc, g.sid_mm, vol)
    x, y, z = vol.centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    # a window of 1.7 semi-axes around the object keeps distant streaks out
    box = (np.abs(X - c0[0]) < 1.7 * a[0]) & (np.abs(Y - c0[1]) < 1.7 * a[1]) & (np.abs(Z - c0[2]) < 1.7 * a[2])
    m = rec * box
    c = np.array([float((m * A).sum() / m.sum()) for A in (X, Y, Z)])
    assert np.allclose(c, c0, atol=0.4), c
    # the integral over the window is the ellipsoid's mass 4/3 pi abc
    mass = float(m.sum()) * vol.voxel_mm ** 3
    assert abs(mass - 4.0 / 3.0 * math.pi * a.prod()) < 0.05 * mass
    inside = (((X - c0[0]) / a[0]) ** 2 + ((Y - c0[1]) / a[1]) ** 2 + ((Z - c0[2]) / a[2]) ** 2) < 0.5
    assert abs(rec[inside].mean() - 1.0) < 5e-3


def test_motion_compensation_undoes_known_motion():
    """Projections of an object translated by up to 6 mm, reconstructed
    with P' = P T(theta): close to the static reconstruction (the residual
    is the different detector sampling of the moved object, a floor of
    about 5 % of the object's RMS density for this phantom), while the
    uncompensated reconstruction and one with the inverse convention
    P T(-theta) are several times further off."""
    g, P, intr, betas, arc = _small_scan()
    ph = inputs.random_phantom(4, 6, contained_radius=0.9 * g.fov_radius())
    theta = inputs.smooth_motion(8, g.n_views, peak=6.0, params=(3, 4, 5))
    static = inputs.project(g, ph)
    moved = inputs.project(g, ph, motion=theta)
    vol = fdk.Volume(32, 32, 32, 3.0)
    ref = fdk.fdk(static, P, intr, betas, arc, g.sid_mm, vol)

    def moved_P(sign):
        return np.array([moved_projection([list(r) for r in P[i]], list(sign * theta[i]))
                         for i in range(g.n_views)])

    def rms(rec):
        return float(np.sqrt(np.mean((rec - ref) ** 2)))

    err_c = rms(fdk.fdk(moved, P, intr, betas, arc, g.sid_mm, vol, moved_P=moved_P(1.0)))
    err_p = rms(fdk.fdk(moved, P, intr, betas, arc, g.sid_mm, vol))
    err_i = rms(fdk.fdk(moved, P, intr, betas, arc, g.sid_mm, vol, moved_P=moved_P(-1.0)))
    assert err_c < 0.2 * err_p and err_i > err_p, (err_c, err_p, err_i)


def test_point_values_equal_the_full_reconstruction():
    """voxel_values (rows filtered on demand, for sampled checks at full
    size) gives the same numbers as the whole-volume route."""
    g = inputs.ScanGeometry(61, 64, 48, 3.6)
    P, intr = g.projection_matrices(), g.intrinsics()
    betas, arc = g.orbit_angles(), math.radians(g.arc_deg)
    imgs = inputs.project(g, inputs.random_phantom(4, 6, contained_radius=0.9 * g.fov_radius()))
    vol = fdk.Volume(12, 10, 8, 8.0)
    rec = fdk.fdk(imgs, P, intr, betas, arc, g.sid_mm, vol)
    x, y, z = vol.centres()
    idx = [(5, 4, 3), (7, 9, 0), (0, 0, 11), (3, 5, 6)]
    pts = np.array([[x[i], y[j], z[k]] for k, j, i in idx])
    vals = fdk.voxel_values(pts, lambda lam, r: imgs[lam][r], imgs.shape, P, intr, betas, arc, g.sid_mm)
    assert np.allclose(vals, [rec[k, j, i] for k, j, i in idx], rtol=1e-12, atol=1e-14)
