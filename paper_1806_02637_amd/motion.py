"""Rigid motion estimation with the consistency cost (Sec. "Optimization").

Each of the six rigid parameters of T(theta) along the scan is an Akima
spline through a few nodes; the optimiser searches the node values of the
selected parameters (the experiment estimates t_z, the out-of-plane
translation, through 17 nodes).  One evaluation runs entirely on the GPU:
nodes -> per-view theta (``ecc_spline_motion``), cost and gradient
(``ecc_cost_grad``), chain rule back to the nodes
(``ecc_spline_motion_grad``); only the node vector and its gradient cross to
the host, where a limited-memory BFGS (L-BFGS-B) chooses the next nodes.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B
from .engine import Scan, _stream_handle


class SplineMotion:
    """Device-side Akima motion model of one scan: n_nodes nodes spread
    evenly over the view index range."""

    def __init__(self, scan: Scan, n_nodes: int):
        self.scan = scan
        self.n_views = scan.n_views
        self.n_nodes = int(n_nodes)
        self.node_x = np.ascontiguousarray(np.linspace(0.0, self.n_views - 1.0, self.n_nodes))
        self.device = scan.engine.device

    def theta(self, nodes: torch.Tensor) -> torch.Tensor:
        """nodes [B, 6, n_nodes] FP64 (device) -> theta [B, n_views, 6] FP64."""
        nodes = nodes.contiguous()
        Bn = nodes.shape[0]
        assert nodes.shape == (Bn, 6, self.n_nodes) and nodes.dtype == torch.float64 and nodes.is_cuda
        th = torch.empty((Bn, self.n_views, 6), dtype=torch.float64, device=self.device)
        B.ecc_spline_motion(self.scan.ctx, Bn, self.n_views, self.n_nodes, self.node_x.ctypes.data, nodes.data_ptr(),
                            th.data_ptr(), _stream_handle(self.device))
        return th

    def grad(self, nodes: torch.Tensor, grad_theta: torch.Tensor) -> torch.Tensor:
        """d cost / d nodes [B, 6, n_nodes] FP64 from d cost / d theta [B, n_views, 6] FP32."""
        nodes = nodes.contiguous()
        grad_theta = grad_theta.contiguous()
        Bn = nodes.shape[0]
        assert grad_theta.shape == (Bn, self.n_views, 6) and grad_theta.dtype == torch.float32
        out = torch.empty((Bn, 6, self.n_nodes), dtype=torch.float64, device=self.device)
        B.ecc_spline_motion_grad(self.scan.ctx, Bn, self.n_views, self.n_nodes, self.node_x.ctypes.data,
                                 nodes.data_ptr(), grad_theta.data_ptr(), out.data_ptr(),
                                 _stream_handle(self.device))
        return out


@dataclass
class MotionResult:
    nodes: np.ndarray              # [6, n_nodes] estimated node values
    theta: np.ndarray              # [n_views, 6] the motion they describe
    cost: float
    cost0: float
    n_evals: int
    n_iter: int
    seconds: float                 # wall-clock of the whole estimation
    eval_ms: list = field(default_factory=list)  # wall-clock per evaluation (device work + transfers)
    history: list = field(default_factory=list)  # cost per evaluation
    message: str = ""


def estimate_motion(scan: Scan, K: int, R_mm: float, n_nodes: int = 17, params=(5,), c: float = math.inf,
                    init: np.ndarray | None = None, max_iter: int = 60, gtol: float = 1e-9,
                    scale: float = 1.0, callback=None, kappa: str = "object") -> MotionResult:
    """Minimises the cost over the spline nodes of the selected parameters
    (indices into theta: 0-2 rotations in degrees, 3-5 translations in mm).

    ``scale`` divides the cost seen by the optimiser (the cost's magnitude
    depends on the data; a scale near the initial cost keeps L-BFGS-B's
    tolerances meaningful).  ``init`` gives the starting nodes [6, n_nodes]
    (zero motion by default).  ``kappa`` selects the sampled plane range
    ("object" sphere of radius R_mm, or "detector"-bounded)."""
    from scipy.optimize import minimize

    model = SplineMotion(scan, n_nodes)
    dev = model.device
    params = tuple(int(p) for p in params)
    nodes0 = np.zeros((6, n_nodes)) if init is None else np.array(init, dtype=np.float64).reshape(6, n_nodes)
    nodes_dev = torch.tensor(nodes0[None], dtype=torch.float64, device=dev)
    ws = scan.workspace(1, True)
    sel = torch.tensor(params, device=dev)
    history, eval_ms = [], []

    def fun(x):
        t0 = time.perf_counter()
        nodes_dev[0, sel] = torch.as_tensor(x.reshape(len(params), n_nodes), dtype=torch.float64, device=dev)
        th = model.theta(nodes_dev)
        cost, g_th = scan.cost_grad(th, K, R_mm, c, workspace=ws, kappa=kappa)
        g_nodes = model.grad(nodes_dev, g_th)
        f = float(cost[0]) / scale
        g = g_nodes[0, sel].reshape(-1).cpu().numpy() / scale
        eval_ms.append((time.perf_counter() - t0) * 1e3)
        history.append(f * scale)
        return f, g

    t_start = time.perf_counter()
    res = minimize(fun, nodes0[list(params)].reshape(-1), jac=True, method="L-BFGS-B", callback=callback,
                   options={"maxiter": max_iter, "gtol": gtol, "ftol": 1e-12})
    seconds = time.perf_counter() - t_start
    nodes = nodes0.copy()
    nodes[list(params)] = res.x.reshape(len(params), n_nodes)
    nodes_dev[0] = torch.as_tensor(nodes, dtype=torch.float64, device=dev)
    theta = model.theta(nodes_dev)[0].cpu().numpy()
    return MotionResult(nodes=nodes, theta=theta, cost=float(res.fun) * scale, cost0=history[0],
                        n_evals=len(history), n_iter=int(res.nit), seconds=seconds, eval_ms=eval_ms,
                        history=history, message=str(res.message))
