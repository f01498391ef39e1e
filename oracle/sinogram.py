"""Grangeat's intermediate function sampled on a flat detector: the
Radon-derivative ("d rho") sinogram of every projection (Eq. 1 and its
precomputation in the "Epipolar Consistency" subsection), FP64.

The paper defers the detector-domain form of Eq. 1 to the literature.  For a
flat detector at distance f (px) from the source and a detector line
x cos(alpha) + y sin(alpha) = t in centred pixel coordinates,
    dR f(n, d)/dd at d = n . c  =  (1 + t^2 / f^2) * dG/dt (alpha, t),
    G(alpha, t) = integral along the line of g(u, v) f / sqrt(f^2 + x^2 + y^2),
where n is the normal of the plane through the source and that line.  The
sinogram stores dG/dt; the factor (1 + t^2/f^2) is applied at lookup.

Discretisation (the paper gives none; sizes come from the workloads):
* t_max = sqrt(W^2 + H^2) / 2 px, alpha_m = m pi / n_alpha (m < n_alpha),
  t_k = -t_max + k * 2 t_max / (n_t - 1) (k < n_t);
* line samples s_j = (j - (n_s - 1)/2) ds, n_s = 2 ceil(t_max / ds) + 1,
  bilinear interpolation of the weighted image, zero outside it;
* d rho(alpha_m, t_k) = (G_{k+1} - G_{k-1}) / (2 dt) with G_{-1} = G_{n_t} = 0;
* row n_alpha stores d rho(pi, t_k) = -d rho(0, t_{n_t-1-k}), the odd
  symmetry d rho(alpha + pi, -t) = -d rho(alpha, t), so that bilinear
  interpolation across alpha = pi needs no wrap logic.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_sino.so")
_lib = None


def build_lib(force: bool = False) -> str:
    """Compile the plain-C line-integral routine with gcc (no fast-math)."""
    src = os.path.join(_HERE, "sino.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fno-fast-math", "-o", tmp, src, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build_lib()
        lib = ctypes.CDLL(_LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_line_integrals.argtypes = [dp, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                              ctypes.c_int, ip, ip, ctypes.c_long, dp]
        lib.oracle_line_integrals.restype = None
        _lib = lib
    return _lib


@dataclass(frozen=True)
class SinoGrid:
    W: int
    H: int
    n_alpha: int
    n_t: int
    ds: float = 0.5

    @property
    def t_max(self) -> float:
        return 0.5 * math.sqrt(self.W ** 2 + self.H ** 2)

    @property
    def dt(self) -> float:
        return 2.0 * self.t_max / (self.n_t - 1)

    @property
    def dalpha(self) -> float:
        return math.pi / self.n_alpha

    @property
    def n_s(self) -> int:
        return 2 * int(math.ceil(self.t_max / self.ds)) + 1


def cosine_weighted(img, f, u0, v0):
    """g(i, j) * f / sqrt(f^2 + (i - u0)^2 + (j - v0)^2): the radial weighting
    of the "Grangeat's Theorem" subsection, on pixel centres, in FP64."""
    img = np.asarray(img, dtype=np.float64)
    H, W = img.shape
    x = np.arange(W, dtype=np.float64) - u0
    y = np.arange(H, dtype=np.float64) - v0
    return img * (f / np.sqrt(f * f + x[None, :] ** 2 + y[:, None] ** 2))


def line_integrals(g_w, grid: SinoGrid, u0, v0, m, k):
    """G(alpha_m, t_k) for arrays of cell indices (0 <= m < n_alpha, 0 <= k < n_t)."""
    lib = _load()
    g_w = np.ascontiguousarray(g_w, dtype=np.float64)
    m = np.ascontiguousarray(m, dtype=np.int32).ravel()
    k = np.ascontiguousarray(k, dtype=np.int32).ravel()
    out = np.empty(m.shape[0], dtype=np.float64)
    if m.shape[0]:
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lib.oracle_line_integrals(g_w.ctypes.data_as(dp), grid.W, grid.H, float(u0), float(v0), grid.dalpha,
                                  grid.t_max, grid.dt, grid.ds, grid.n_s, m.ctypes.data_as(ip),
                                  k.ctypes.data_as(ip), m.shape[0], out.ctypes.data_as(dp))
    return out


def drho_cells(g_w, grid: SinoGrid, u0, v0, m, k):
    """Stored sinogram values at cells (m, k), 0 <= m <= n_alpha, 0 <= k < n_t
    (row n_alpha is the symmetric pad row)."""
    m = np.asarray(m, dtype=np.int64).ravel()
    k = np.asarray(k, dtype=np.int64).ravel()
    pad = m == grid.n_alpha
    mm = np.where(pad, 0, m)
    kk = np.where(pad, grid.n_t - 1 - k, k)
    # G at k + 1 and k - 1, zero beyond the grid
    hi_ok = kk + 1 <= grid.n_t - 1
    lo_ok = kk - 1 >= 0
    g_hi = np.zeros(m.shape[0])
    g_lo = np.zeros(m.shape[0])
    g_hi[hi_ok] = line_integrals(g_w, grid, u0, v0, mm[hi_ok], kk[hi_ok] + 1)
    g_lo[lo_ok] = line_integrals(g_w, grid, u0, v0, mm[lo_ok], kk[lo_ok] - 1)
    d = (g_hi - g_lo) / (2.0 * grid.dt)
    return np.where(pad, -d, d)


def full_sinogram(img, grid: SinoGrid, f, u0, v0):
    """All rows [n_alpha + 1, n_t] of one view's sinogram."""
    g_w = cosine_weighted(img, f, u0, v0)
    mm, kk = np.meshgrid(np.arange(grid.n_alpha), np.arange(grid.n_t), indexing="ij")
    G = line_integrals(g_w, grid, u0, v0, mm, kk).reshape(grid.n_alpha, grid.n_t)
    Gp = np.zeros((grid.n_alpha, grid.n_t + 2))
    Gp[:, 1:-1] = G
    d = (Gp[:, 2:] - Gp[:, :-2]) / (2.0 * grid.dt)
    out = np.empty((grid.n_alpha + 1, grid.n_t))
    out[:grid.n_alpha] = d
    out[grid.n_alpha] = -d[0, ::-1]
    return out


class FullSinograms:
    """Sinogram set held as an array [n_views, n_alpha + 1, n_t]."""

    def __init__(self, data, grid: SinoGrid):
        self.data = np.asarray(data, dtype=np.float64)
        self.grid = grid

    @classmethod
    def build(cls, images, grid: SinoGrid, intr):
        data = np.stack([full_sinogram(images[i], grid, *intr[i]) for i in range(len(images))])
        return cls(data, grid)

    def cells(self, view, m, k):
        return self.data[view][m, k]


class LazySinograms:
    """Sinogram set whose cells are computed on first use (for workloads whose
    full oracle sinograms would take hours on the host)."""

    def __init__(self, images, grid: SinoGrid, intr):
        self.images = images
        self.grid = grid
        self.intr = np.asarray(intr, dtype=np.float64)
        self._gw = {}
        self._rows = {}

    def _view(self, view):
        if view not in self._rows:
            f, u0, v0 = self.intr[view]
            self._gw[view] = cosine_weighted(self.images[view], f, u0, v0)
            self._rows[view] = np.full((self.grid.n_alpha + 1, self.grid.n_t), np.nan)
        return self._rows[view]

    def cells(self, view, m, k):
        rows = self._view(view)
        m = np.asarray(m)
        k = np.asarray(k)
        vals = rows[m, k]
        miss = np.isnan(vals)
        if miss.any():
            mu, ku = m[miss], k[miss]
            key = np.unique(mu.astype(np.int64) * self.grid.n_t + ku)
            um, uk = key // self.grid.n_t, key % self.grid.n_t
            f, u0, v0 = self.intr[view]
            rows[um, uk] = drho_cells(self._gw[view], self.grid, u0, v0, um, uk)
            vals = rows[m, k]
        return vals

    def prefetch(self, view, m, k):
        self.cells(view, m, k)
