"""Pins of the oracle's Akima motion model (Sec. "Optimization": each rigid
parameter follows an Akima spline through a few nodes) against a library
implementation of Akima's method, closed forms and finite differences."""
import numpy as np
import pytest
from scipy.interpolate import Akima1DInterpolator

from oracle import spline


def test_matches_library_akima():
    rng = np.random.default_rng(3)
    for n in (3, 5, 17):
        xn = np.sort(rng.uniform(0, 100, n))
        xn[0], xn[-1] = 0.0, 100.0
        yn = rng.normal(0, 2, n)
        xq = np.linspace(0, 100, 777)
        ref = Akima1DInterpolator(xn, yn, method="akima")(xq)
        got = spline.akima_values(xn, yn, xq)
        assert np.abs(got - ref).max() <= 1e-12 * (1 + np.abs(ref).max())


def test_interpolates_and_reproduces_lines():
    xn = spline.node_positions(248, 17)
    yn = 0.3 * xn - 4.0
    xq = np.arange(248.0)
    np.testing.assert_allclose(spline.akima_values(xn, yn, xq), 0.3 * xq - 4.0, rtol=0, atol=1e-12)
    rng = np.random.default_rng(4)
    yr = rng.normal(size=17)
    np.testing.assert_allclose(spline.akima_values(xn, yr, xn), yr, rtol=0, atol=1e-12)


def test_flat_runs_stay_flat():
    # Akima's locality: three equal slopes around a node give it the common
    # slope, so a plateau between two ramps is exactly flat
    xn = np.arange(8.0)
    yn = np.array([0.0, 1.0, 2.0, 2.0, 2.0, 2.0, 5.0, 9.0])
    xq = np.linspace(2.0, 5.0, 61)
    np.testing.assert_allclose(spline.akima_values(xn, yn, xq[(xq >= 3) & (xq <= 4)]), 2.0, atol=1e-15)
    # the derivative estimate at node 3 is 0 (|m3 - m2| = 0 weights m2 = 0)
    t = spline.node_slopes(list(xn), list(yn))
    assert t[3] == 0.0 and t[4] == 0.0


def test_jacobian_matches_central_differences():
    rng = np.random.default_rng(5)
    xn = spline.node_positions(60, 9)
    yn = rng.normal(0, 1.5, 9)
    xq = np.arange(60.0)
    J = spline.akima_jacobian(xn, yn, xq)
    h = 1e-6
    for j in range(9):
        e = np.zeros(9)
        e[j] = h
        lib = lambda y: Akima1DInterpolator(xn, y, method="akima")(xq)  # noqa: E731
        fd = (lib(yn + e) - lib(yn - e)) / (2 * h)
        np.testing.assert_allclose(J[:, j], fd, rtol=0, atol=2e-7)


def test_motion_chain_rule():
    rng = np.random.default_rng(6)
    n_views, n_nodes = 40, 7
    xn = spline.node_positions(n_views, n_nodes)
    nodes = rng.normal(0, 1, (6, n_nodes))
    theta = spline.spline_motion(xn, nodes, n_views)
    assert theta.shape == (n_views, 6)
    g = rng.normal(size=(n_views, 6))
    gn = spline.spline_motion_grad(xn, nodes, g)
    # directional derivative of <g, theta(nodes)> against differences
    dn = rng.normal(size=(6, n_nodes))
    h = 1e-6
    fd = (np.sum(g * spline.spline_motion(xn, nodes + h * dn, n_views)) -
          np.sum(g * spline.spline_motion(xn, nodes - h * dn, n_views))) / (2 * h)
    assert abs(np.sum(gn * dn) - fd) <= 1e-6 * (1 + abs(fd))


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        spline.node_slopes([0.0, 1.0], [0.0, 1.0])
    with pytest.raises(ValueError):
        spline.akima_values([0.0, 1.0, 2.0], [0.0, 1.0, 0.0], [2.5])
