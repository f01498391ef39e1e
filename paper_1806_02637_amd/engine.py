"""Torch-facing wrapper of the C ABI: device tensors in, device tensors out.

PyTorch only supplies device memory and the current stream; every step runs
in the engine's HIP kernels.  ``Engine`` owns an ecc context, ``Scan`` one
resident scan.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import binding as B


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Engine:
    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("the ECC engine needs a ROCm GPU (torch.cuda.is_available() is False)")
        B.load_library()
        self.device = torch.device("cuda", device)
        self.ctx = B.ecc_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx:
            B.ecc_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def load_scan(self, P, intr, images, W: int | None = None, H: int | None = None) -> "Scan":
        """P [N,3,4], intr [N,3] (f, u0, v0) and images [N,H,W] FP32 (host
        array or device tensor)."""
        P = np.ascontiguousarray(P, dtype=np.float64)
        intr = np.ascontiguousarray(intr, dtype=np.float64)
        n = P.shape[0]
        if isinstance(images, torch.Tensor) and images.is_cuda:
            img = images.to(self.device, torch.float32).contiguous()
            H_, W_ = img.shape[1], img.shape[2]
            sid = B.ecc_scan_load(self.ctx, n, W_, H_, P.ctypes.data, intr.ctypes.data, img.data_ptr(), 1)
            torch.cuda.synchronize(self.device)
        else:
            img = np.ascontiguousarray(images, dtype=np.float32)
            H_, W_ = img.shape[1], img.shape[2]
            sid = B.ecc_scan_load(self.ctx, n, W_, H_, P.ctypes.data, intr.ctypes.data, img.ctypes.data, 0)
        return Scan(self, sid, n, W_, H_)


class Scan:
    def __init__(self, engine: Engine, scan_id: int, n_views: int, W: int, H: int):
        self.engine = engine
        self.id = scan_id
        self.n_views = n_views
        self.W, self.H = W, H
        self.n_pairs = n_views * (n_views - 1) // 2
        self.n_alpha = self.n_t = None
        self._ws = {}
        self._fdk_ws = None

    @property
    def ctx(self):
        return self.engine.ctx

    def build_sinograms(self, n_alpha: int, n_t: int, ds_px: float = 0.5, dtype: str = "f32"):
        B.ecc_scan_build_sinograms(self.ctx, self.id, n_alpha, n_t, ds_px, B.DTYPES[dtype],
                                   _stream_handle(self.engine.device))
        self.n_alpha, self.n_t = n_alpha, n_t

    def set_sinograms(self, sino, dtype: str = "f32"):
        """sino [N, n_alpha + 1, n_t] FP32 computed elsewhere."""
        if isinstance(sino, torch.Tensor) and sino.is_cuda:
            s = sino.to(self.engine.device, torch.float32).contiguous()
            torch.cuda.synchronize(self.engine.device)
            B.ecc_scan_set_sinograms(self.ctx, self.id, s.shape[1] - 1, s.shape[2], s.data_ptr(), 1, B.DTYPES[dtype])
        else:
            s = np.ascontiguousarray(sino, dtype=np.float32)
            B.ecc_scan_set_sinograms(self.ctx, self.id, s.shape[1] - 1, s.shape[2], s.ctypes.data, 0,
                                     B.DTYPES[dtype])
        self.n_alpha, self.n_t = s.shape[1] - 1, s.shape[2]

    def read_sinogram(self, view: int) -> np.ndarray:
        out = np.empty((self.n_alpha + 1, self.n_t), dtype=np.float32)
        B.ecc_scan_read_sinogram(self.ctx, self.id, view, out.ctypes.data)
        return out

    def resident_bytes(self) -> int:
        return B.ecc_scan_bytes(self.ctx, self.id)

    def free(self):
        B.ecc_scan_free(self.ctx, self.id)
        self._fdk_ws = None

    def workspace(self, Bn: int, with_grad: bool) -> torch.Tensor:
        key = (Bn, bool(with_grad))
        ws = self._ws.get(key)
        if ws is None:
            nbytes = B.ecc_workspace_bytes(self.ctx, self.id, Bn, int(with_grad))
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.engine.device)
            self._ws[key] = ws
        return ws

    @staticmethod
    def params(K: int, R_mm: float, c: float = math.inf, geom: str = "f32", kappa: str = "object") -> B.EvalParams:
        """kappa: "object" (planes meeting the object sphere of radius R_mm)
        or "detector" (the arc around kappa = 0 both detectors see)."""
        if kappa not in ("object", "detector"):
            raise ValueError(f"kappa must be 'object' or 'detector', got {kappa!r}")
        return B.EvalParams(int(K), B.ECC_GEOM_F64 if geom == "f64" else B.ECC_GEOM_F32, float(R_mm),
                            0.0 if math.isinf(c) else float(c),
                            B.ECC_KAPPA_DETECTOR if kappa == "detector" else B.ECC_KAPPA_OBJECT, 0)

    def _theta(self, theta) -> torch.Tensor:
        th = torch.as_tensor(theta, dtype=torch.float64)
        if th.dim() == 2:
            th = th[None]
        if th.shape[1:] != (self.n_views, 6):
            raise ValueError(f"theta must be [B, {self.n_views}, 6], got {tuple(th.shape)}")
        return th.to(self.engine.device).contiguous()

    def cost(self, theta, K: int, R_mm: float, c: float = math.inf, geom: str = "f32", with_pairs: bool = False,
             workspace: torch.Tensor | None = None, kappa: str = "object", with_counts: bool = False):
        """Returns cost [B] (FP64 device tensor), then e [B, n_pairs] if
        with_pairs and the plane counts N_kappa [B, n_pairs] (int32) if
        with_counts."""
        th = self._theta(theta)
        Bn = th.shape[0]
        dev = self.engine.device
        out = torch.empty(Bn, dtype=torch.float64, device=dev)
        pairs = torch.empty((Bn, self.n_pairs), dtype=torch.float32, device=dev) if with_pairs else None
        ws = self.workspace(Bn, False) if workspace is None else workspace
        prm = self.params(K, R_mm, c, geom, kappa)
        pp = pairs.data_ptr() if pairs is not None else 0
        counts = None
        if with_counts:
            counts = torch.empty((Bn, self.n_pairs), dtype=torch.int32, device=dev)
            B.ecc_cost_counts(self.ctx, self.id, Bn, th.data_ptr(), prm, out.data_ptr(), pp, counts.data_ptr(),
                              ws.data_ptr(), ws.numel(), _stream_handle(dev))
        else:
            B.ecc_cost(self.ctx, self.id, Bn, th.data_ptr(), prm, out.data_ptr(), pp, ws.data_ptr(), ws.numel(),
                       _stream_handle(dev))
        res = (out,) + ((pairs,) if with_pairs else ()) + ((counts,) if with_counts else ())
        return res if len(res) > 1 else out

    def fdk(self, images, vol, theta=None) -> torch.Tensor:
        """FDK reconstruction [nz, ny, nx] (FP32 device tensor) of this scan's
        geometry from line-integral images [N, H, W] (FP32, device); vol =
        (nx, ny, nz, voxel_mm) centred on the isocentre; theta [N, 6] the
        motion to compensate (back-projection with P T(theta)), None for
        none."""
        dev = self.engine.device
        imgs = torch.as_tensor(images, dtype=torch.float32, device=dev).contiguous()
        if tuple(imgs.shape) != (self.n_views, self.H, self.W):
            raise ValueError(f"images must be [{self.n_views}, {self.H}, {self.W}], got {tuple(imgs.shape)}")
        nx, ny, nz, vox = vol
        th = None
        if theta is not None:
            th = torch.as_tensor(theta, dtype=torch.float64, device=dev).reshape(self.n_views, 6).contiguous()
        out = torch.empty((int(nz), int(ny), int(nx)), dtype=torch.float32, device=dev)
        nbytes = B.ecc_fdk_workspace_bytes(self.ctx, self.id)
        if self._fdk_ws is None or self._fdk_ws.numel() < nbytes:
            self._fdk_ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        ws = self._fdk_ws
        B.ecc_fdk(self.ctx, self.id, th.data_ptr() if th is not None else 0, imgs.data_ptr(),
                  B.EccVolume(int(nx), int(ny), int(nz), 0, float(vox)), out.data_ptr(), ws.data_ptr(), ws.numel(),
                  _stream_handle(dev))
        return out

    def release_fdk_workspace(self):
        """Drops the cached FDK workspace (the filtered views)."""
        self._fdk_ws = None

    def cost_grad(self, theta, K: int, R_mm: float, c: float = math.inf, geom: str = "f32",
                  with_pair_grads: bool = False, workspace: torch.Tensor | None = None, kappa: str = "object"):
        """Returns cost [B] FP64, grad [B, N, 6] FP32 (and per-pair [B, n_pairs, 12])."""
        th = self._theta(theta)
        Bn = th.shape[0]
        dev = self.engine.device
        out = torch.empty(Bn, dtype=torch.float64, device=dev)
        grad = torch.empty((Bn, self.n_views, 6), dtype=torch.float32, device=dev)
        pg = torch.empty((Bn, self.n_pairs, 12), dtype=torch.float32, device=dev) if with_pair_grads else None
        ws = self.workspace(Bn, True) if workspace is None else workspace
        B.ecc_cost_grad(self.ctx, self.id, Bn, th.data_ptr(), self.params(K, R_mm, c, geom, kappa), out.data_ptr(),
                        grad.data_ptr(), pg.data_ptr() if pg is not None else 0, ws.data_ptr(), ws.numel(),
                        _stream_handle(dev))
        return (out, grad, pg) if with_pair_grads else (out, grad)
