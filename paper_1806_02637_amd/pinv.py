"""The pseudo-inverse route to the epipolar lines, kept as the comparison the
paper makes (Sec. "Introduction", "Optimized Algorithm" and "Experiments").

Before the method, each evaluation needed the pseudo-inverses P'^+ of all
moved projection matrices, computed on the CPU and shipped to the GPU, which
then mapped every epipolar plane E to its line l = P'^{+T} E.  This module is
that host half: P' = P T(theta) and P'^+ = P'^T (P' P'^T)^{-1} for every
(hypothesis, view) with NumPy, a pinned staging buffer and the upload; the
device half is ``ecc_cost_pinv``.  The method itself (``Scan.cost``) needs
none of it: the lines come from Eqs. 13-14 on the device.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import binding as B
from .engine import Scan, _stream_handle


def rigid_T(theta: np.ndarray) -> np.ndarray:
    """T(theta) = [[R_z R_y R_x, t], [0, 1]] for theta [..., 6] (degrees, mm)."""
    th = np.asarray(theta, dtype=np.float64)
    ax, ay, az = (np.deg2rad(th[..., i]) for i in range(3))
    cx, sx, cy, sy, cz, sz = np.cos(ax), np.sin(ax), np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    T = np.zeros(th.shape[:-1] + (4, 4))
    T[..., 0, 0] = cz * cy
    T[..., 0, 1] = cz * sy * sx - sz * cx
    T[..., 0, 2] = cz * sy * cx + sz * sx
    T[..., 1, 0] = sz * cy
    T[..., 1, 1] = sz * sy * sx + cz * cx
    T[..., 1, 2] = sz * sy * cx - cz * sx
    T[..., 2, 0] = -sy
    T[..., 2, 1] = cy * sx
    T[..., 2, 2] = cy * cx
    T[..., :3, 3] = th[..., 3:]
    T[..., 3, 3] = 1.0
    return T


def moved_pinv(P: np.ndarray, theta: np.ndarray, out: np.ndarray | None = None) -> np.ndarray:
    """Pseudo-inverses [B, N, 4, 3] of P'_lam = P_lam T(theta_{b, lam})."""
    Pm = np.asarray(P, dtype=np.float64)[None] @ rigid_T(theta)  # [B, N, 3, 4]
    PPt = Pm @ np.swapaxes(Pm, -1, -2)  # [B, N, 3, 3]
    res = np.swapaxes(Pm, -1, -2) @ np.linalg.inv(PPt)
    if out is not None:
        out[...] = res
        return out
    return res


class PinvRoute:
    """Evaluates the cost through the pseudo-inverse route: per call the host
    computes and uploads the pseudo-inverses, then ``ecc_cost_pinv`` runs."""

    def __init__(self, scan: Scan, P: np.ndarray, B_max: int):
        self.scan = scan
        self.P = np.asarray(P, dtype=np.float64)
        n = scan.n_views
        self.host = torch.empty((B_max, n, 4, 3), dtype=torch.float64).pin_memory()
        self.dev = torch.empty((B_max, n, 4, 3), dtype=torch.float64, device=scan.engine.device)
        self.host_ms = []  # host pseudo-inverse time per call
        self._copied = None  # event after the last upload from the staging buffer

    def cost(self, theta_host: np.ndarray, K: int, R_mm: float, c: float = math.inf, with_pairs: bool = False,
             kappa: str = "object"):
        th = np.asarray(theta_host, dtype=np.float64)
        if th.ndim == 2:
            th = th[None]
        Bn = th.shape[0]
        if self._copied is not None:
            self._copied.synchronize()  # the staging buffer is free again
        t0 = time.perf_counter()
        moved_pinv(self.P, th, out=self.host[:Bn].numpy())
        self.host_ms.append((time.perf_counter() - t0) * 1e3)
        dev = self.scan.engine.device
        self.dev[:Bn].copy_(self.host[:Bn], non_blocking=True)
        self._copied = torch.cuda.Event()
        self._copied.record()
        th_dev = torch.as_tensor(th, device=dev)
        out = torch.empty(Bn, dtype=torch.float64, device=dev)
        pairs = torch.empty((Bn, self.scan.n_pairs), dtype=torch.float32, device=dev) if with_pairs else None
        ws = self.scan.workspace(Bn, False)
        B.ecc_cost_pinv(self.scan.ctx, self.scan.id, Bn, th_dev.data_ptr(), self.dev.data_ptr(),
                        self.scan.params(K, R_mm, c, kappa=kappa), out.data_ptr(), pairs.data_ptr() if pairs is not None else 0,
                        ws.data_ptr(), ws.numel(), _stream_handle(dev))
        return (out, pairs) if with_pairs else out
