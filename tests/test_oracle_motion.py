"""Pins of the moved-scan generator against the oracle: projections taken
while the object moves along theta_true are consistent under the hypothesis
theta_true (Eq. 15 with P' = P T(theta)), markedly less so under zero motion
or the opposite motion.  This fixes the generator's motion convention to the
one the cost uses."""
import numpy as np

import oracle
from paper_1806_02637_amd import inputs


def test_moved_frames_match_moved_projection_matrices():
    from oracle.geometry import moved_projection

    g = inputs.ScanGeometry(12, 96, 80, 2.0)
    th = inputs.smooth_motion(3, g.n_views, peak=3.0, params=(0, 2, 4, 5))
    C2, R2 = inputs.moved_frames(g, th)
    P = g.projection_matrices()
    Kmat = np.array([[g.f_px, 0.0, g.u0], [0.0, g.f_px, g.v0], [0.0, 0.0, 1.0]])
    for v in range(g.n_views):
        P2 = np.asarray(moved_projection([list(r) for r in P[v]], list(th[v])), dtype=np.float64)
        ref = np.concatenate([Kmat @ R2[v], -(Kmat @ R2[v] @ C2[v])[:, None]], axis=1)
        np.testing.assert_allclose(P2, ref, rtol=0, atol=1e-9 * np.abs(ref).max())


def test_consistent_only_at_the_true_motion(small16):
    s = small16
    g, w = s["geom"], s["w"]
    th = inputs.smooth_motion(5, g.n_views, peak=4.0, params=(5,))
    imgs = inputs.project(g, w.phantom(contained=True), motion=th)
    sino = oracle.FullSinograms.build(imgs, s["grid"], s["intr"])
    cost = lambda t: oracle.ecc_cost(s["P"], s["intr"], t, s["grid"], sino, s["params"])[0]  # noqa: E731
    c_true, c_zero, c_neg = cost(th), cost(np.zeros_like(th)), cost(-th)
    assert c_true < 0.25 * c_zero, (c_true, c_zero)
    assert c_true < 0.1 * c_neg, (c_true, c_neg)
