"""Python face of the engine's continuous-batching server (ecc_server_* in
include/ecc.h): submit requests as they arrive, collect results and
latencies.  Scheduling, admission and device work all happen in the engine.
"""
from __future__ import annotations

import math
import threading
import time
from dataclasses import dataclass

import numpy as np

from . import binding as B
from .engine import Scan


@dataclass
class Result:
    request_id: int
    cost: np.ndarray
    grad: np.ndarray | None
    queue_ms: float
    run_ms: float
    total_ms: float
    slot: int


class Server:
    def __init__(self, engine, n_slots: int = 4, arena_bytes: int = 8 << 30, work_cap: float = 0.0):
        self.engine = engine
        self.srv = B.ecc_server_create(engine.ctx, n_slots, arena_bytes)
        if work_cap:
            B.ecc_server_set_work_cap(self.srv, work_cap)
        self._meta = {}
        self._lock = threading.Lock()

    def close(self):
        if self.srv:
            B.ecc_server_destroy(self.srv)
            self.srv = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def request_bytes(self, scan: Scan, Bn: int, with_grad: bool) -> int:
        return B.ecc_server_request_bytes(self.srv, scan.id, Bn, int(with_grad))

    def submit(self, scan: Scan, theta, K: int, R_mm: float, with_grad: bool = False, c: float = math.inf,
               geom: str = "f32", kappa: str = "object") -> int:
        th = np.ascontiguousarray(theta, dtype=np.float64)
        if th.ndim == 2:
            th = th[None]
        rid = B.ecc_server_submit(self.srv, scan.id, th.shape[0], th.ctypes.data,
                                  Scan.params(K, R_mm, c, geom, kappa), int(with_grad))
        with self._lock:
            self._meta[rid] = (th.shape[0], scan.n_views, bool(with_grad))
        return rid

    def done(self, rid: int) -> bool:
        return B.ecc_server_poll(self.srv, rid)

    def wait(self, rid: int) -> Result:
        with self._lock:
            Bn, n_views, with_grad = self._meta.pop(rid)
        cost = np.empty(Bn, dtype=np.float64)
        grad = np.empty((Bn, n_views, 6), dtype=np.float32) if with_grad else None
        st = B.ecc_server_wait(self.srv, rid, cost.ctypes.data, grad.ctypes.data if grad is not None else 0)
        return Result(rid, cost, grad, st.queue_ms, st.run_ms, st.total_ms, st.slot)


def poisson_arrivals(rate_per_s: float, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))


def replay(server: Server, trace):
    """trace: list of (arrival_s, scan, theta, K, R_mm, with_grad).  Submits
    each request at its arrival time (relative to the start) from this
    thread, then waits for all; returns (results in trace order, makespan_s)."""
    t0 = time.perf_counter()
    ids = []
    for arrival, scan, theta, K, R_mm, with_grad in trace:
        now = time.perf_counter() - t0
        if arrival > now:
            time.sleep(arrival - now)
        ids.append(server.submit(scan, theta, K, R_mm, with_grad))
    results = [server.wait(rid) for rid in ids]
    return results, time.perf_counter() - t0


def latency_summary(results) -> dict:
    lat = np.array([r.total_ms for r in results])
    return {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()), "max_ms": float(lat.max()), "n": int(lat.size)}
