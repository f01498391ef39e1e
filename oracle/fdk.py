"""Feldkamp-Davis-Kress (FDK) reconstruction from a circular short scan with
per-view (motion-compensated) projection matrices, FP64 (test
infrastructure).

The reconstruction the paper inspects after compensation ("Experiments"):
the estimated rigid motion enters only through the projection matrices
P'_lam = P_lam T(theta_lam) used to back-project view lam.

Steps (Feldkamp, Davis and Kress 1984 for the cone-beam weights and the
back-projection; Kak and Slaney, "Principles of Computerized Tomographic
Imaging", ch. 3, for the discrete ramp filter; Parker 1982 for the
short-scan redundancy weights):

* per view and pixel (u, v): p_w = w_parker(beta, gamma(u)) * c(u, v) * p,
  with the cosine weight c = f / sqrt(f^2 + (u - u0)^2 + (v - v0)^2) (pixels);
* per detector row: Q(u) = (1 / tau) sum_k h(u - k) p_w(k), with the sampled
  ramp h(0) = 1/4, h(n) = -1 / (pi n)^2 for odd n, 0 for even n != 0, and
  tau = D / f the pixel pitch at the isocentre (D = source-isocentre
  distance);
* per voxel x: f(x) = sum over views of dbeta (D / z)^2 Q(u_x, v_x), where
  (u_x z, v_x z, z) = P'_lam (x, 1): z is the depth of x along the principal
  ray; Q is read by bilinear interpolation, zero off the detector.

Parker weights for a scan over [0, pi + 2 delta], delta = (arc - pi) / 2 >=
the half fan angle, with gamma the fan angle measured so that the ray
conjugate to (beta, gamma) is (beta + pi + 2 gamma, -gamma):
  sin^2(pi/4 beta / (delta - gamma))                 on [0, 2 delta - 2 gamma),
  1                                                  up to pi - 2 gamma,
  sin^2(pi/4 (pi + 2 delta - beta) / (delta + gamma))  up to pi + 2 delta.
For the orbit of ``inputs.ScanGeometry`` (source at D (cos b, sin b, 0),
columns along (-sin b, cos b, 0)) that fan angle is -atan((u - u0) / f).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Volume:
    """nx x ny x nz voxels of `voxel_mm`, centred on the isocentre; voxel
    (i, j, k) sits at ((i - (nx-1)/2) s, (j - (ny-1)/2) s, (k - (nz-1)/2) s)."""
    nx: int
    ny: int
    nz: int
    voxel_mm: float

    def centres(self):
        s = self.voxel_mm
        x = (np.arange(self.nx) - 0.5 * (self.nx - 1)) * s
        y = (np.arange(self.ny) - 0.5 * (self.ny - 1)) * s
        z = (np.arange(self.nz) - 0.5 * (self.nz - 1)) * s
        return x, y, z


def ramp_kernel(n_max: int) -> np.ndarray:
    """h(n) for n = -n_max..n_max (Kak and Slaney's sampled Ram-Lak filter,
    unit sample spacing)."""
    n = np.arange(-n_max, n_max + 1)
    h = np.zeros(n.shape)
    h[n == 0] = 0.25
    odd = (n % 2) != 0
    h[odd] = -1.0 / (math.pi * n[odd]) ** 2
    return h


def parker_weights(beta: float, gamma: np.ndarray, delta: float) -> np.ndarray:
    """Parker's short-scan weights at orbit angle beta for fan angles gamma."""
    g = np.asarray(gamma, dtype=np.float64)
    w = np.ones(g.shape)
    lo = beta < 2.0 * delta - 2.0 * g
    w[lo] = np.sin(0.25 * math.pi * beta / (delta - g[lo])) ** 2
    hi = beta > math.pi - 2.0 * g
    w[hi] = np.sin(0.25 * math.pi * (math.pi + 2.0 * delta - beta) / (delta + g[hi])) ** 2
    return w


def filter_row(row, r: int, intr_lam, beta: float, arc_rad: float, sid_mm: float) -> np.ndarray:
    """One detector row r of one view: Parker and cosine weights, then the
    ramp filter, Q(u) = (1 / tau) sum_k h(u - k) p_w(k)."""
    row = np.asarray(row, dtype=np.float64)
    W = row.shape[0]
    f, u0, v0 = (float(x) for x in intr_lam)
    u = np.arange(W) - u0
    gamma = -np.arctan(u / f)
    wp = parker_weights(float(beta), gamma, 0.5 * (arc_rad - math.pi))
    cosw = f / np.sqrt(f * f + u ** 2 + (r - v0) ** 2)
    tau = sid_mm / f
    # full linear convolution, then the W outputs aligned with the input
    return np.convolve(row * cosw * wp, ramp_kernel(W - 1))[W - 1:2 * W - 1] / tau


def filter_views(images, intr, betas, arc_rad: float, sid_mm: float) -> np.ndarray:
    """Parker- and cosine-weighted, ramp-filtered projections Q [N, H, W]."""
    imgs = np.asarray(images, dtype=np.float64)
    N, H, W = imgs.shape
    out = np.empty_like(imgs)
    for lam in range(N):
        for r in range(H):
            out[lam, r] = filter_row(imgs[lam, r], r, intr[lam], betas[lam], arc_rad, sid_mm)
    return out


def _bilinear(Q, u, v):
    """Q[v, u] at fractional (u, v) with zero outside the sample grid."""
    H, W = Q.shape
    u0 = np.floor(u).astype(np.int64)
    v0 = np.floor(v).astype(np.int64)
    fu, fv = u - u0, v - v0
    out = np.zeros(u.shape)
    for du, dv, wgt in ((0, 0, (1 - fu) * (1 - fv)), (1, 0, fu * (1 - fv)), (0, 1, (1 - fu) * fv),
                        (1, 1, fu * fv)):
        uu, vv = u0 + du, v0 + dv
        ok = (uu >= 0) & (uu < W) & (vv >= 0) & (vv < H)
        out[ok] += wgt[ok] * Q[vv[ok], uu[ok]]
    return out


def backproject(Q, Pm, vol: Volume, dbeta: float, sid_mm: float) -> np.ndarray:
    """f [nz, ny, nx] = sum_lam dbeta (D / z)^2 Q_lam(u_x, v_x) with the
    (moved) projection matrices Pm [N, 3, 4]."""
    x, y, z = vol.centres()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    Xh = np.stack([X, Y, Z, np.ones_like(X)], axis=-1)  # [nz, ny, nx, 4]
    f = np.zeros(X.shape)
    for lam in range(Q.shape[0]):
        p = Xh @ np.asarray(Pm[lam], dtype=np.float64).T  # [..., 3]
        depth = p[..., 2]
        u, v = p[..., 0] / depth, p[..., 1] / depth
        f += dbeta * (sid_mm / depth) ** 2 * _bilinear(Q[lam], u, v)
    return f


def fdk(images, P, intr, betas, arc_rad: float, sid_mm: float, vol: Volume, moved_P=None) -> np.ndarray:
    """Reconstruction [nz, ny, nx] (density, 1/mm) from line-integral images
    [N, H, W]; back-projection with moved_P (P'_lam = P_lam T(theta_lam)) when
    given, else with P.  Views are spaced evenly: dbeta = arc / (N - 1)."""
    N = len(images)
    Q = filter_views(images, intr, betas, arc_rad, sid_mm)
    dbeta = arc_rad / (N - 1)
    return backproject(Q, P if moved_P is None else moved_P, vol, dbeta, sid_mm)


def voxel_values(points, row_of, shape, P, intr, betas, arc_rad: float, sid_mm: float, moved_P=None):
    """f at a few points [M, 3] (mm) without filtering every row: the rows a
    point's bilinear cells need are filtered on first use.  row_of(lam, r)
    returns image row r of view lam; shape = (N, H, W)."""
    N, H, W = shape
    Pm = P if moved_P is None else moved_P
    dbeta = arc_rad / (N - 1)
    cache = {}

    def q_row(lam, r):
        if r < 0 or r >= H:
            return None
        key = (lam, r)
        if key not in cache:
            cache[key] = filter_row(row_of(lam, r), r, intr[lam], betas[lam], arc_rad, sid_mm)
        return cache[key]

    out = np.zeros(len(points))
    for i, x in enumerate(np.asarray(points, dtype=np.float64)):
        xh = np.append(x, 1.0)
        for lam in range(N):
            p = np.asarray(Pm[lam], dtype=np.float64) @ xh
            depth = p[2]
            u, v = p[0] / depth, p[1] / depth
            uf, vf = math.floor(u), math.floor(v)
            fu, fv = u - uf, v - vf
            val = 0.0
            for dv, wv in ((0, 1.0 - fv), (1, fv)):
                row = q_row(lam, vf + dv)
                if row is None:
                    continue
                for du, wu in ((0, 1.0 - fu), (1, fu)):
                    if 0 <= uf + du < W:
                        val += wv * wu * row[uf + du]
            out[i] += dbeta * (sid_mm / depth) ** 2 * val
    return out
