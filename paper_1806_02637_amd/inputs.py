"""Seeded synthetic scans: C-arm short-scan geometry, ellipsoid phantoms,
analytic cone-beam projections and per-view rigid-motion hypotheses.

This module is the single source of inputs shared by the FP64 oracle and the
HIP engine.  It holds none of the consistency method's arithmetic (no
sinogram, no epipolar geometry, no cost): it only simulates what a scanner
would deliver -- projection matrices, intrinsics and line-integral images --
plus the random motion parameters the cost is evaluated at.

Conventions (the paper fixes none of them; Sec. "Experiments" only gives a
short scan over 200 degrees with 496 projections):

* World frame in mm, isocentre at the origin, rotation axis z.
* View lam of N sits at orbit angle phi = lam * 200deg / (N - 1) with the
  source at C = SID (cos phi, sin phi, 0), SID = 785 mm, SDD = 1200 mm.
* Detector axes e_u = (-sin phi, cos phi, 0) (columns), e_v = (0, 0, -1)
  (rows grow downwards) and viewing direction e_w = -(cos phi, sin phi, 0);
  (e_u, e_v, e_w) is right-handed.
* Intrinsics K = [[f, 0, u0], [0, f, v0], [0, 0, 1]], f = SDD / pitch in px,
  u0 = (W - 1) / 2, v0 = (H - 1) / 2; pixel (i, j) (column i, row j) has its
  centre at (u, v) = (i, j).  P = K [R | -R C] with R = rows (e_u, e_v, e_w).
* Rigid motion theta = (rx, ry, rz [deg], tx, ty, tz [mm]) per view.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SID_MM = 785.0
SDD_MM = 1200.0
ARC_DEG = 200.0


@dataclass(frozen=True)
class ScanGeometry:
    n_views: int
    W: int
    H: int
    pitch_mm: float
    sid_mm: float = SID_MM
    sdd_mm: float = SDD_MM
    arc_deg: float = ARC_DEG

    @property
    def f_px(self) -> float:
        return self.sdd_mm / self.pitch_mm

    @property
    def u0(self) -> float:
        return (self.W - 1) / 2.0

    @property
    def v0(self) -> float:
        return (self.H - 1) / 2.0

    def orbit_angles(self) -> np.ndarray:
        if self.n_views == 1:
            return np.zeros(1)
        return np.deg2rad(np.arange(self.n_views) * self.arc_deg / (self.n_views - 1))

    def frames(self):
        """Per view: source position C [N,3] and rotation R [N,3,3] (rows e_u, e_v, e_w)."""
        phi = self.orbit_angles()
        c, s = np.cos(phi), np.sin(phi)
        z = np.zeros_like(phi)
        C = self.sid_mm * np.stack([c, s, z], axis=1)
        e_u = np.stack([-s, c, z], axis=1)
        e_v = np.stack([z, z, -np.ones_like(phi)], axis=1)
        e_w = np.stack([-c, -s, z], axis=1)
        R = np.stack([e_u, e_v, e_w], axis=1)
        return C, R

    def intrinsics(self) -> np.ndarray:
        """[N,3] float64 rows {f_px, u0, v0}."""
        out = np.empty((self.n_views, 3))
        out[:, 0] = self.f_px
        out[:, 1] = self.u0
        out[:, 2] = self.v0
        return out

    def projection_matrices(self) -> np.ndarray:
        """[N,3,4] float64, pixels <- world mm."""
        C, R = self.frames()
        Kmat = np.array([[self.f_px, 0.0, self.u0], [0.0, self.f_px, self.v0], [0.0, 0.0, 1.0]])
        P = np.empty((self.n_views, 3, 4))
        for i in range(self.n_views):
            P[i, :, :3] = Kmat @ R[i]
            P[i, :, 3] = -(Kmat @ R[i] @ C[i])
        return P

    def default_object_radius(self) -> float:
        """0.95 x the radius of the isocentric sphere whose shadow fits the detector."""
        half = 0.5 * min(self.W, self.H) * self.pitch_mm
        return 0.95 * self.sid_mm * math.sin(math.atan(half / self.sdd_mm))

    def fov_radius(self) -> float:
        half = 0.5 * min(self.W, self.H) * self.pitch_mm
        return self.sid_mm * math.sin(math.atan(half / self.sdd_mm))


@dataclass(frozen=True)
class Phantom:
    centers: np.ndarray  # [E,3] mm
    semi_axes: np.ndarray  # [E,3] mm
    axes: np.ndarray  # [E,3,3], columns are the ellipsoid axes
    density: np.ndarray  # [E] 1/mm

    @property
    def n(self) -> int:
        return int(self.centers.shape[0])


def _quat_to_matrix(q: np.ndarray) -> np.ndarray:
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def random_phantom(seed: int, n_ellipsoids: int, contained_radius: float | None = None,
                   semi_range=(10.0, 60.0), centre_radius: float = 60.0,
                   density_range=(0.1, 1.0)) -> Phantom:
    """Seeded ellipsoid phantom.

    Draw order per ellipsoid: semi-axes (3 uniforms), centre radius (1 uniform,
    r = centre_radius * u^(1/3)), centre direction (3 normals), orientation
    quaternion (4 normals), density (1 uniform).  With ``contained_radius`` set,
    an ellipsoid whose bounding sphere |x_e| + max(a_e) exceeds it is redrawn, so
    that no detector row or column truncates the object.
    """
    rng = np.random.default_rng(seed)
    cs, ss, qs, rs = [], [], [], []
    while len(cs) < n_ellipsoids:
        a = rng.uniform(semi_range[0], semi_range[1], 3)
        r = centre_radius * rng.uniform() ** (1.0 / 3.0)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        rho = rng.uniform(density_range[0], density_range[1])
        if contained_radius is not None and r + a.max() > contained_radius:
            continue
        cs.append(r * d)
        ss.append(a)
        qs.append(_quat_to_matrix(q))
        rs.append(rho)
    return Phantom(np.array(cs), np.array(ss), np.array(qs), np.array(rs))


def sphere_phantom(radius_mm: float, density: float = 1.0) -> Phantom:
    """A single homogeneous sphere at the isocentre."""
    return Phantom(np.zeros((1, 3)), np.full((1, 3), float(radius_mm)), np.eye(3)[None],
                   np.array([float(density)]))


def rigid_rotation(rx_deg: float, ry_deg: float, rz_deg: float) -> np.ndarray:
    """R_z R_y R_x of the three angles (degrees), right-handed."""
    ax, ay, az = np.deg2rad([rx_deg, ry_deg, rz_deg])
    Rx = np.array([[1, 0, 0], [0, math.cos(ax), -math.sin(ax)], [0, math.sin(ax), math.cos(ax)]])
    Ry = np.array([[math.cos(ay), 0, math.sin(ay)], [0, 1, 0], [-math.sin(ay), 0, math.cos(ay)]])
    Rz = np.array([[math.cos(az), -math.sin(az), 0], [math.sin(az), math.cos(az), 0], [0, 0, 1]])
    return Rz @ Ry @ Rx


def moved_frames(geom: ScanGeometry, motion: np.ndarray):
    """Frames of a scan during which the object moved: the camera of view lam
    is P T(theta_lam) with T = [[R_z R_y R_x, t], [0, 1]], i.e. rotation
    R Rm and source Rm^T (C - t)."""
    C, R = geom.frames()
    C2, R2 = np.empty_like(C), np.empty_like(R)
    for i in range(geom.n_views):
        Rm = rigid_rotation(*motion[i, :3])
        R2[i] = R[i] @ Rm
        C2[i] = Rm.T @ (C[i] - motion[i, 3:])
    return C2, R2


def smooth_motion(seed: int, n_views: int, peak: float = 2.0, params=(5,)) -> np.ndarray:
    """theta [n_views, 6]: for each selected parameter a smooth random curve
    (three low-frequency sinusoids plus one smooth step, the kind of drift and
    sudden shift a patient makes), scaled to a peak deviation of ``peak``
    about its mean; other parameters 0."""
    rng = np.random.default_rng(seed)
    lam = np.arange(n_views, dtype=np.float64)
    th = np.zeros((n_views, 6))
    for p in params:
        periods = rng.uniform(n_views / 3.0, 2.0 * n_views, 3)
        phases = rng.uniform(0.0, 2 * math.pi, 3)
        amps = rng.normal(size=3)
        step_at, step_amp = rng.uniform(0.3, 0.7) * n_views, rng.normal()
        y = sum(a * np.sin(2 * math.pi * lam / T + ph) for a, T, ph in zip(amps, periods, phases))
        y = y + step_amp * np.tanh((lam - step_at) / (n_views / 20.0))
        y = y - y.mean()
        th[:, p] = peak * y / np.abs(y).max()
    return th


def project(geom: ScanGeometry, phantom: Phantom, views=None, device: str = "cpu",
            chunk_rows: int | None = None, as_tensor: bool = False, motion: np.ndarray | None = None):
    """Analytic line integrals through every pixel centre, FP64, returned FP32.

    Returns images [n_sel, H, W] (row v, column u) as a NumPy array, or as an
    FP32 torch tensor on ``device`` with ``as_tensor``.  ``device`` selects where
    torch evaluates the intersections ("cpu" or "cuda"); the arithmetic is
    FP64 either way.  For ray X = C + tau * omega (|omega| = 1) and an ellipsoid
    (x_e, a_e, Q_e): y = diag(1/a) Q^T (C - x_e), w = diag(1/a) Q^T omega,
    D = (y.w)^2 - |w|^2 (|y|^2 - 1); the chord length is 2 sqrt(D) / |w|^2 for D > 0.
    ``motion`` [n_views, 6] projects with the moved cameras of ``moved_frames``.
    """
    import torch

    C_all, R_all = geom.frames() if motion is None else moved_frames(geom, np.asarray(motion, dtype=np.float64))
    if views is None:
        views = range(geom.n_views)
    views = list(views)
    dev = torch.device(device)
    f, u0, v0 = geom.f_px, geom.u0, geom.v0
    W, H = geom.W, geom.H
    out = torch.empty((len(views), H, W), dtype=torch.float32, device=dev) if as_tensor else \
        np.empty((len(views), H, W), dtype=np.float32)
    cen = torch.as_tensor(phantom.centers, dtype=torch.float64, device=dev)
    inv_a = torch.as_tensor(1.0 / phantom.semi_axes, dtype=torch.float64, device=dev)
    QT = torch.as_tensor(np.transpose(phantom.axes, (0, 2, 1)).copy(), dtype=torch.float64, device=dev)
    rho = torch.as_tensor(phantom.density, dtype=torch.float64, device=dev)
    if chunk_rows is None:
        chunk_rows = max(1, min(H, (1 << 22) // max(W, 1)))
    uu = torch.arange(W, dtype=torch.float64, device=dev)
    for oi, lam in enumerate(views):
        C = torch.as_tensor(C_all[lam], dtype=torch.float64, device=dev)
        R = torch.as_tensor(R_all[lam], dtype=torch.float64, device=dev)
        # per ellipsoid source term y_c and the linear map omega -> w
        Y = inv_a * torch.einsum("eij,ej->ei", QT, C[None, :] - cen)  # [E,3]
        A = inv_a[:, :, None] * QT  # [E,3,3]
        img = torch.empty((H, W), dtype=torch.float64, device=dev)
        for r0 in range(0, H, chunk_rows):
            r1 = min(H, r0 + chunk_rows)
            vv = torch.arange(r0, r1, dtype=torch.float64, device=dev)
            xc = torch.empty((r1 - r0, W, 3), dtype=torch.float64, device=dev)
            xc[..., 0] = ((uu - u0) / f)[None, :]
            xc[..., 1] = ((vv - v0) / f)[:, None]
            xc[..., 2] = 1.0
            om = xc @ R  # camera -> world: omega = R^T x_c
            om = om / torch.linalg.norm(om, dim=-1, keepdim=True)
            acc = torch.zeros((r1 - r0, W), dtype=torch.float64, device=dev)
            for e in range(phantom.n):
                w = om @ A[e].T  # [rows,W,3]
                ww = (w * w).sum(-1)
                yw = (w * Y[e]).sum(-1)
                D = yw * yw - ww * (Y[e].dot(Y[e]) - 1.0)
                acc += rho[e] * torch.where(D > 0, 2.0 * torch.sqrt(D.clamp_min(0.0)) / ww,
                                            torch.zeros_like(D))
            img[r0:r1] = acc
        if as_tensor:
            out[oi] = img.to(torch.float32)
        else:
            out[oi] = img.to(torch.float32).cpu().numpy()
    return out


def random_motion(seed: int, B: int, n_views: int, rot_sd_deg: float = 0.5,
                  trans_sd_mm: float = 1.0) -> np.ndarray:
    """theta [B,N,6] float64: i.i.d. normal rotations (deg) and translations (mm);
    hypotheses are drawn in order, each as an [N,6] block of standard normals."""
    rng = np.random.default_rng(seed)
    th = rng.normal(size=(B, n_views, 6))
    th[..., :3] *= rot_sd_deg
    th[..., 3:] *= trans_sd_mm
    return th


@dataclass(frozen=True)
class Workload:
    """One synthetic scan plus the evaluation parameters of a workload."""
    name: str
    geom: ScanGeometry
    n_alpha: int
    n_t: int
    K: int
    B: int
    n_ellipsoids: int
    phantom_seed: int
    motion_seed: int | None  # None: zero motion
    ds_px: float = 0.5
    notes: str = ""

    @property
    def R_mm(self) -> float:
        return self.geom.default_object_radius()

    @property
    def n_pairs(self) -> int:
        n = self.geom.n_views
        return n * (n - 1) // 2

    def phantom(self, contained: bool = False) -> Phantom:
        lim = 0.95 * self.geom.fov_radius() if contained else None
        return random_phantom(self.phantom_seed, self.n_ellipsoids, contained_radius=lim)

    def motion(self, B: int | None = None) -> np.ndarray:
        B = self.B if B is None else B
        if self.motion_seed is None:
            return np.zeros((B, self.geom.n_views, 6))
        return random_motion(self.motion_seed, B, self.geom.n_views)


WORKLOADS = {
    "small16": Workload("small16", ScanGeometry(16, 128, 128, 2.4), 180, 181, 64, 1, 10, 1, None,
                        notes="16 views, 128x128 at 2.4 mm, 180x181 sinogram, K=64, no motion"),
    "mid248": Workload("mid248", ScanGeometry(248, 620, 480, 0.616), 360, 512, 256, 32, 30, 2, 1002,
                       notes="248 views, 620x480 at 0.616 mm, 360x512 sinogram, K=256, B=32"),
    "full496": Workload("full496", ScanGeometry(496, 1240, 960, 0.308), 768, 1024, 512, 32, 30, 2, 1003,
                        notes="496 views, 1240x960 at 0.308 mm, 768x1024 sinogram, K=512, B=32"),
    "adj248": Workload("adj248", ScanGeometry(248, 620, 480, 0.616), 360, 512, 256, 1, 30, 2, 1004,
                       notes="adjoint form: 248 views, K=256, gradient w.r.t. 1488 parameters"),
}

# motion-estimation experiment (Sec. "Optimization" / "Experiments"): the
# 496-view scan of an FOV-contained phantom acquired while the object drifts
# along z (smooth t_z curve, 2 mm peak); the estimate runs on 17 Akima nodes
MOTION_EXPERIMENT = dict(workload="full496", motion_seed=77, peak_mm=2.0, params=(5,), n_nodes=17)

# served form: 8 scans of uneven view counts; scans with <= 248 views use the
# 620x480 detector and a 360x512 sinogram with K=256, larger ones 1240x960,
# 768x1024 and K=512.
SERVE_VIEW_COUNTS = (60, 120, 248, 248, 372, 496, 496, 496)


def serve_workloads():
    out = []
    for i, n in enumerate(SERVE_VIEW_COUNTS):
        if n <= 248:
            g = ScanGeometry(n, 620, 480, 0.616)
            out.append(Workload(f"serve{i}_{n}", g, 360, 512, 256, 64, 30, 100 + i, 2000 + i))
        else:
            g = ScanGeometry(n, 1240, 960, 0.308)
            out.append(Workload(f"serve{i}_{n}", g, 768, 1024, 512, 64, 30, 100 + i, 2000 + i))
    return out
