"""Akima spline motion model (test infrastructure).

The motion-estimation experiment (Sec. "Optimization") models every rigid
parameter of T(theta) along the scan as an Akima spline (Akima 1970) through a
few nodes, so that the optimiser searches the node values only.  This module
restates Akima's interpolant plainly in FP64:

* segment slopes m_i = (y_{i+1} - y_i) / (x_{i+1} - x_i), extended by two
  linearly extrapolated slopes at each end (m_{-1} = 2 m_0 - m_1,
  m_{-2} = 2 m_{-1} - m_0, and the mirror image at the far end);
* node derivative t_i = (|m_{i+1} - m_i| m_{i-1} + |m_{i-1} - m_{i-2}| m_i)
  / (|m_{i+1} - m_i| + |m_{i-1} - m_{i-2}|), or (m_{i-1} + m_i) / 2 when both
  weights vanish;
* a cubic Hermite piece on every segment.

The code runs on floats or on ``Dual`` node values, which gives the exact
Jacobian of the interpolant with respect to the node values (the weights'
absolute values are differentiated on the side their value selects).
"""
from __future__ import annotations

import numpy as np

from .dual import Dual, value


def _abs(x):
    return -x if value(x) < 0 else x


def node_slopes(xn, yn):
    """Akima's derivative estimate at every node."""
    n = len(xn)
    if n < 3:
        raise ValueError("an Akima spline needs at least 3 nodes")
    m = [(yn[i + 1] - yn[i]) / (xn[i + 1] - xn[i]) for i in range(n - 1)]
    lo1 = 2.0 * m[0] - m[1]
    lo2 = 2.0 * lo1 - m[0]
    hi1 = 2.0 * m[-1] - m[-2]
    hi2 = 2.0 * hi1 - m[-1]
    ext = [lo2, lo1] + m + [hi1, hi2]  # ext[i + 2] = m_i
    t = []
    for i in range(n):
        m_2, m_1, m0, m1 = ext[i], ext[i + 1], ext[i + 2], ext[i + 3]
        w_hi = _abs(m1 - m0)
        w_lo = _abs(m_1 - m_2)
        if value(w_hi) + value(w_lo) == 0.0:
            t.append(0.5 * (m_1 + m0))
        else:
            t.append((w_hi * m_1 + w_lo * m0) / (w_hi + w_lo))
    return t


def segment_of(xn, x: float) -> int:
    """Index i of the segment [x_i, x_{i+1}] holding x (closed at the end)."""
    n = len(xn)
    if not (xn[0] <= x <= xn[-1]):
        raise ValueError("query outside the node range")
    i = int(np.searchsorted(np.asarray(xn, dtype=np.float64), x, side="right")) - 1
    return min(max(i, 0), n - 2)


def akima(xn, yn, xq):
    """The Akima interpolant through (xn, yn) at the points xq (a list of
    floats or Duals per point)."""
    t = node_slopes(xn, yn)
    out = []
    for x in np.atleast_1d(np.asarray(xq, dtype=np.float64)):
        i = segment_of(xn, float(x))
        h = xn[i + 1] - xn[i]
        s = (float(x) - xn[i]) / h
        s2, s3 = s * s, s * s * s
        h00 = 2 * s3 - 3 * s2 + 1
        h10 = s3 - 2 * s2 + s
        h01 = -2 * s3 + 3 * s2
        h11 = s3 - s2
        out.append(h00 * yn[i] + h10 * h * t[i] + h01 * yn[i + 1] + h11 * h * t[i + 1])
    return out


def akima_values(xn, yn, xq) -> np.ndarray:
    return np.array([float(v) for v in akima(list(map(float, xn)), [float(y) for y in yn], xq)])


def akima_jacobian(xn, yn, xq) -> np.ndarray:
    """d value(xq) / d yn as a [len(xq), len(yn)] array (forward mode)."""
    n = len(yn)
    yd = [Dual.variable(float(y), j, n) for j, y in enumerate(yn)]
    vals = akima(list(map(float, xn)), yd, xq)
    return np.stack([v.d if isinstance(v, Dual) else np.zeros(n) for v in vals])


def node_positions(n_views: int, n_nodes: int) -> np.ndarray:
    """Nodes spread evenly over the view index range [0, n_views - 1]."""
    return np.linspace(0.0, n_views - 1.0, n_nodes)


def spline_motion(xn, nodes, n_views: int) -> np.ndarray:
    """theta [n_views, 6] from node values [6, n_nodes] (parameter c of view
    lam = the spline of row c at lam)."""
    lam = np.arange(n_views, dtype=np.float64)
    return np.stack([akima_values(xn, nodes[c], lam) for c in range(6)], axis=1)


def spline_motion_grad(xn, nodes, grad_theta) -> np.ndarray:
    """Chain rule: d cost / d nodes [6, n_nodes] from d cost / d theta
    [n_views, 6]."""
    n_views = grad_theta.shape[0]
    lam = np.arange(n_views, dtype=np.float64)
    out = np.zeros(np.asarray(nodes).shape)
    for c in range(6):
        J = akima_jacobian(xn, nodes[c], lam)
        out[c] = J.T @ grad_theta[:, c]
    return out
