"""Scene, camera motion and ray casting for synthetic structure-flow sequences.

Conventions
-----------
* Camera frame: x to the right (increasing column j), y down (increasing row i),
  z forward.  The world frame coincides with the camera frame at t = 0.
* Pixel (i, j) of a pinhole camera looks along the unit ray
  normalize(((j - cx) / fx, (i - cy) / fy, 1)).
* Inverse depth is rho = 1 / range (reference range 1 m), range measured along
  the unit ray, as in the paper's definition of depth and inverse depth (Section
  "Structure Flow", eq:depth and eq:inv_depth).  Rays that hit nothing (sky)
  get rho = 0, which is a valid value (infinitely far away).
* Ground-truth structure flow for a static scene is w = -Omega x eta - rho * v_c
  in rad/s (eq:homogeneous_flow with the point velocity set to zero, as the
  paper does for its own ground truth in Section "Ground truth evaluation").

Camera kinematics follow eq:camvel_dot / eq:totaldev_ppos: the inertial
velocity V is constant, so the body-frame velocity is v_c(t) = R(t)^T V, and the
body-frame angular velocity Omega(t) is prescribed (constant or sinusoidal).
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence as Seq

import numpy as np
import torch


# ----------------------------------------------------------------------------------------
# camera and motion
# ----------------------------------------------------------------------------------------
@dataclasses.dataclass
class Camera:
    rows: int
    cols: int
    fx: float
    fy: float
    cx: float
    cy: float

    def rays(self, device="cpu") -> "torch.Tensor":
        """Unit rays (rows, cols, 3) in the camera frame, float64."""
        j = torch.arange(self.cols, dtype=torch.float64, device=device)
        i = torch.arange(self.rows, dtype=torch.float64, device=device)
        x = ((j[None, :] - self.cx) / self.fx).expand(self.rows, self.cols)
        y = ((i[:, None] - self.cy) / self.fy).expand(self.rows, self.cols)
        r = torch.stack([x, y, torch.ones_like(x)], dim=-1)
        return r / torch.linalg.norm(r, dim=-1, keepdim=True)


def equiangular_rays(rows: int, cols: int, hfov_deg: float) -> np.ndarray:
    """Unit directions (rows, cols, 3) of an equiangular (longitude-latitude) grid centred on
    the optical axis: column j at longitude (j - (cols-1)/2) d, row i at latitude
    (i - (rows-1)/2) d, with d = hfov / (cols - 1); eta = (sin lon cos lat, sin lat,
    cos lon cos lat) (x right, y down, z forward).  A wide-angle grid on which pinhole pixels
    would be far from uniform."""
    d = np.radians(hfov_deg) / (cols - 1)
    lon = (np.arange(cols) - (cols - 1) / 2.0) * d
    lat = (np.arange(rows) - (rows - 1) / 2.0) * d
    La, Lo = np.meshgrid(lat, lon, indexing="ij")
    return np.stack([np.sin(Lo) * np.cos(La), np.sin(La), np.cos(Lo) * np.cos(La)], axis=-1)


@dataclasses.dataclass
class GridCamera(Camera):
    """A camera whose pixels look along a given grid of unit directions (rows, cols, 3);
    fx, fy, cx, cy describe a nominal pinhole of the same angular resolution (used to scale
    motion to a target image motion)."""
    eta: Optional[np.ndarray] = None

    def rays(self, device="cpu") -> "torch.Tensor":
        return torch.as_tensor(self.eta, dtype=torch.float64, device=device)


def _skew(w: np.ndarray) -> np.ndarray:
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _expm_so3(w: np.ndarray) -> np.ndarray:
    th = float(np.linalg.norm(w))
    K = _skew(w)
    if th < 1e-12:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * K @ K


@dataclasses.dataclass
class Trajectory:
    """Constant inertial velocity V plus body-frame angular velocity
    Omega(t) = omega0 + amp * sin(2 pi freq t + phase) (per axis)."""
    V: np.ndarray                      # world-frame linear velocity, m/s
    omega0: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    amp: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    freq: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    phase: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    p0: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros(3))
    substeps: int = 8

    def omega(self, t: float) -> np.ndarray:
        return self.omega0 + self.amp * np.sin(2 * np.pi * self.freq * t + self.phase)

    def omega_dot(self, t: float) -> np.ndarray:
        """d Omega / dt (body frame, rad/s^2)."""
        w = 2 * np.pi * self.freq
        return self.amp * w * np.cos(w * t + self.phase)

    def poses(self, times: np.ndarray):
        """Camera-to-world rotations R_k and positions p_k at the given increasing times
        (the first time is the reference where R = I)."""
        Rs, ps = [], []
        R = np.eye(3)
        t_prev = float(times[0])
        for t in times:
            t = float(t)
            if t > t_prev:
                h = (t - t_prev) / self.substeps
                for s in range(self.substeps):
                    tm = t_prev + (s + 0.5) * h
                    R = R @ _expm_so3(self.omega(tm) * h)   # dR/dt = R [Omega]x
                t_prev = t
            Rs.append(R.copy())
            ps.append(self.p0 + self.V * (t - float(times[0])))
        return Rs, ps


# ----------------------------------------------------------------------------------------
# textures
# ----------------------------------------------------------------------------------------
class ValueNoise:
    """Multi-octave 3-D lattice value noise with smoothstep interpolation, in [0, 1]."""

    def __init__(self, seed: int, spacings: Seq[float], amps: Seq[float], table_bits: int = 16):
        rng = np.random.default_rng(seed)
        self.table = rng.random(1 << table_bits)
        self.mask = (1 << table_bits) - 1
        self.spacings = list(spacings)
        self.amps = list(amps)
        self.offsets = rng.random((len(self.spacings), 3)) * 1000.0
        self._tables = {}

    def _table(self, device):
        key = str(device)
        if key not in self._tables:
            self._tables[key] = torch.as_tensor(self.table, dtype=torch.float64, device=device)
        return self._tables[key]

    def __call__(self, P: "torch.Tensor") -> "torch.Tensor":
        tab = self._table(P.device)
        out = torch.zeros(P.shape[:-1], dtype=torch.float64, device=P.device)
        for sp, amp, off in zip(self.spacings, self.amps, self.offsets):
            Q = P / sp + torch.as_tensor(off, dtype=torch.float64, device=P.device)
            i0 = torch.floor(Q)
            f = Q - i0
            s = f * f * (3.0 - 2.0 * f)
            i0 = i0.to(torch.int64)
            hx = [i0[..., 0] * 73856093, (i0[..., 0] + 1) * 73856093]
            hy = [i0[..., 1] * 19349663, (i0[..., 1] + 1) * 19349663]
            hz = [i0[..., 2] * 83492791, (i0[..., 2] + 1) * 83492791]
            wx = [1.0 - s[..., 0], s[..., 0]]
            wy = [1.0 - s[..., 1], s[..., 1]]
            wz = [1.0 - s[..., 2], s[..., 2]]
            acc = torch.zeros_like(out)
            for dx in (0, 1):
                for dy in (0, 1):
                    hxy = hx[dx] ^ hy[dy]
                    wxy = wx[dx] * wy[dy]
                    for dz in (0, 1):
                        acc += wxy * wz[dz] * tab[(hxy ^ hz[dz]) & self.mask]
            out += amp * acc
        return out / float(sum(self.amps))


# ----------------------------------------------------------------------------------------
# scenes: each maps world rays (origin o, unit directions d) to range, brightness
# ----------------------------------------------------------------------------------------
class SinusoidPlaneScene:
    """One infinite plane n.X = dist with a texture made of a sum of sinusoids in the
    plane's own 2-D coordinates, so brightness is attached to the surface."""

    def __init__(self, normal, dist, n_waves: int, rng: np.random.Generator,
                 freq_range=(0.5, 2.5)):
        self.n = np.asarray(normal, dtype=np.float64)
        self.n /= np.linalg.norm(self.n)
        self.dist = float(dist)
        a = np.cross(self.n, [1.0, 0.0, 0.0])
        if np.linalg.norm(a) < 1e-6:
            a = np.cross(self.n, [0.0, 1.0, 0.0])
        self.e1 = a / np.linalg.norm(a)
        self.e2 = np.cross(self.n, self.e1)
        fmag = rng.uniform(*freq_range, n_waves)
        ang = rng.uniform(0, 2 * np.pi, n_waves)
        self.freqs = np.stack([fmag * np.cos(ang), fmag * np.sin(ang)], axis=1)
        self.phases = rng.uniform(0, 2 * np.pi, n_waves)
        self.amps = rng.uniform(0.2, 1.0, n_waves)

    def cast(self, o: np.ndarray, d: "torch.Tensor"):
        dev = d.device
        n = torch.as_tensor(self.n, dtype=torch.float64, device=dev)
        den = d @ n
        lam = (self.dist - float(o @ self.n)) / den
        lam = torch.where((den > 1e-12) & (lam > 0), lam, torch.full_like(lam, float("inf")))
        P = torch.as_tensor(o, dtype=torch.float64, device=dev) + lam[..., None] * d
        a = P @ torch.as_tensor(self.e1, dtype=torch.float64, device=dev)
        b = P @ torch.as_tensor(self.e2, dtype=torch.float64, device=dev)
        fr = torch.as_tensor(self.freqs, dtype=torch.float64, device=dev)
        arg = 2 * np.pi * (a[..., None] * fr[:, 0] + b[..., None] * fr[:, 1]) + \
            torch.as_tensor(self.phases, dtype=torch.float64, device=dev)
        amps = torch.as_tensor(self.amps, dtype=torch.float64, device=dev)
        Y = 0.5 + 0.5 * (torch.sin(arg) @ amps) / float(self.amps.sum())
        return lam, Y


class BoxScene:
    """Axis-aligned boxes (thin ones act as planes), an optional ground plane y = ground_y
    (y points down) and either an enclosing box or an open sky (rho = 0)."""

    def __init__(self, boxes: List[tuple], noise: ValueNoise, gains, biases, offsets,
                 enclosure: Optional[float] = None, ground_y: Optional[float] = None,
                 ground_style: Optional[tuple] = None):
        self.boxes = [(np.asarray(lo, float), np.asarray(hi, float)) for lo, hi in boxes]
        self.noise = noise
        self.gains = list(gains)
        self.biases = list(biases)
        self.offsets = [np.asarray(o, float) for o in offsets]
        self.enclosure = enclosure
        self.ground_y = ground_y
        self.ground_style = ground_style

    @staticmethod
    def _slab(o, inv, lo, hi):
        tmin = None
        tmax = None
        for a in range(3):
            t1 = (float(lo[a]) - float(o[a])) * inv[a]
            t2 = (float(hi[a]) - float(o[a])) * inv[a]
            lo_a = torch.minimum(t1, t2)
            hi_a = torch.maximum(t1, t2)
            tmin = lo_a if tmin is None else torch.maximum(tmin, lo_a)
            tmax = hi_a if tmax is None else torch.minimum(tmax, hi_a)
        return tmin, tmax

    def cast(self, o: np.ndarray, d: "torch.Tensor"):
        d = torch.where(d.abs() < 1e-30, torch.full_like(d, 1e-30), d)
        inv = [1.0 / d[..., a] for a in range(3)]
        shape = d.shape[:-1]
        dev = d.device
        lam = torch.full(shape, float("inf"), dtype=torch.float64, device=dev)
        obj = torch.full(shape, -1, dtype=torch.int64, device=dev)
        for k, (lo, hi) in enumerate(self.boxes):
            tmin, tmax = self._slab(o, inv, lo, hi)
            hit = (tmax >= tmin) & (tmin > 1e-6) & (tmin < lam)
            lam = torch.where(hit, tmin, lam)
            obj = torch.where(hit, torch.full_like(obj, k), obj)
        if self.ground_y is not None:
            t = (self.ground_y - float(o[1])) * inv[1]
            hit = (d[..., 1] > 1e-9) & (t > 1e-6) & (t < lam)
            lam = torch.where(hit, t, lam)
            obj = torch.where(hit, torch.full_like(obj, len(self.boxes)), obj)
        if self.enclosure is not None:
            e = self.enclosure
            _, tmax = self._slab(o, inv, np.full(3, -e), np.full(3, e))
            hit = torch.isinf(lam)
            lam = torch.where(hit, tmax, lam)
            obj = torch.where(hit, torch.full_like(obj, len(self.boxes) + 1), obj)
        finite = torch.where(torch.isinf(lam), torch.zeros_like(lam), lam)
        P = torch.as_tensor(o, dtype=torch.float64, device=dev) + finite[..., None] * d
        n_obj = len(self.boxes) + 2
        offs = torch.as_tensor(np.stack(self.offsets), dtype=torch.float64, device=dev)
        gains = torch.as_tensor(np.asarray(self.gains, float), dtype=torch.float64, device=dev)
        biases = torch.as_tensor(np.asarray(self.biases, float), dtype=torch.float64, device=dev)
        oc = obj.clamp(min=0)
        tex = self.noise(P + offs[oc])
        Y = biases[oc] + gains[oc] * (tex - 0.5)
        # the open sky's brightness depends on the world direction only
        sky = 0.75 - 0.15 * d[..., 1] + 0.05 * torch.sin(3.0 * d[..., 0])
        Y = torch.where(obj < 0, sky, Y)
        return lam, Y.clamp(0.0, 1.0)


# ----------------------------------------------------------------------------------------
# sequences
# ----------------------------------------------------------------------------------------
@dataclasses.dataclass
class Frame:
    Y: "torch.Tensor"         # (rows, cols) float64 brightness in [0, 1]
    rho: "torch.Tensor"       # (rows, cols) float64 inverse depth (1/m), noisy if requested; 0 = sky
    w_gt: "torch.Tensor"      # (rows, cols, 3) float64 structure flow, rad/s, camera frame
    rho_true: "torch.Tensor"


class Sequence:
    """A lazily rendered seeded sequence: frame(k) renders frame k on demand, as float64
    torch tensors on `device` (the values do not depend on the device beyond rounding of
    the transcendental functions)."""

    def __init__(self, camera: Camera, scene, traj: Trajectory, dt: float, n_frames: int,
                 depth_noise: float = 0.0, noise_seed: int = 0):
        self.camera = camera
        self.scene = scene
        self.traj = traj
        self.dt = float(dt)
        self.n_frames = int(n_frames)
        self.depth_noise = float(depth_noise)
        self.noise_seed = int(noise_seed)
        times = np.arange(self.n_frames) * self.dt
        self.Rs, self.ps = traj.poses(times)
        self.times = times
        self._eta = {}

    @property
    def rows(self):
        return self.camera.rows

    @property
    def cols(self):
        return self.camera.cols

    def _rays(self, device):
        key = str(device)
        if key not in self._eta:
            self._eta[key] = self.camera.rays(device)
        return self._eta[key]

    def frame(self, k: int, device="cpu") -> Frame:
        R, p = self.Rs[k], self.ps[k]
        eta = self._rays(device)
        Rt = torch.as_tensor(R, dtype=torch.float64, device=device)
        d = eta @ Rt.T                                   # world directions
        lam, Y = self.scene.cast(p, d)
        rho_true = torch.where(torch.isinf(lam), torch.zeros_like(lam), 1.0 / lam)
        v_c = torch.as_tensor(R.T @ self.traj.V, dtype=torch.float64, device=device)
        Om = torch.as_tensor(self.traj.omega(self.times[k]), dtype=torch.float64, device=device)
        w = -torch.cross(Om.expand_as(eta), eta, dim=-1) - rho_true[..., None] * v_c
        rho = rho_true
        if self.depth_noise > 0:
            rng = np.random.default_rng((self.noise_seed, k))
            z = torch.as_tensor(rng.standard_normal(tuple(rho_true.shape)), device=device)
            rho = rho_true * (1.0 + self.depth_noise * z)
        return Frame(Y=Y, rho=rho, w_gt=w, rho_true=rho_true)

    def right_image(self, k: int, baseline: float, device="cpu") -> "torch.Tensor":
        """Brightness seen at frame k by the right camera of a rectified stereo pair: the same
        orientation and rays, its centre `baseline` metres along the left camera's x axis."""
        R, p = self.Rs[k], self.ps[k]
        eta = self._rays(device)
        Rt = torch.as_tensor(R, dtype=torch.float64, device=device)
        d = eta @ Rt.T
        _, Y = self.scene.cast(p + R @ np.array([baseline, 0.0, 0.0]), d)
        return Y

    def imu(self, k: int):
        """What an inertial measurement unit on the camera reports for the interval from frame
        k - 1 to frame k, as the filter takes it (constant over the interval): the body-frame
        angular velocity (rad/s) and its rate of change (rad/s^2) at mid-interval, and the
        inertial linear acceleration in the camera frame (m/s^2; zero, since the inertial
        velocity is constant).  Returns (omega, omega_dot, acc)."""
        tm = 0.5 * (self.times[k - 1] + self.times[k]) if k > 0 else self.times[0]
        return (np.asarray(self.traj.omega(tm), dtype=np.float64),
                np.asarray(self.traj.omega_dot(tm), dtype=np.float64), np.zeros(3))

    def pixel_flow(self, k: int = 0, device="cpu") -> "torch.Tensor":
        """Instantaneous ground-truth image motion in pixels per frame (rows, cols, 2),
        from the pinhole projection of eta_dot = P_eta w."""
        f = self.frame(k, device)
        eta = self._rays(device)
        w = f.w_gt
        eta_dot = w - eta * torch.sum(eta * w, dim=-1, keepdim=True)
        ez = eta[..., 2]
        u = self.camera.fx * (eta_dot[..., 0] * ez - eta[..., 0] * eta_dot[..., 2]) / ez ** 2
        v = self.camera.fy * (eta_dot[..., 1] * ez - eta[..., 1] * eta_dot[..., 2]) / ez ** 2
        return torch.stack([u, v], dim=-1) * self.dt

    def max_flow_px(self, k: int = 0, device="cpu") -> float:
        return float(torch.linalg.norm(self.pixel_flow(k, device), dim=-1).max())


def _flow_scale(seq_factory: Callable[[float, float], Sequence], target_px: float,
                rot_share: float, device="cpu") -> tuple:
    """Scale translation and rotation so that the frame-0 pixel flow reaches target_px,
    with about rot_share of it from rotation (flow is linear in both jointly)."""
    mt = seq_factory(1.0, 0.0).max_flow_px(0, device)
    mr = seq_factory(0.0, 1.0).max_flow_px(0, device) if rot_share > 0 else 0.0
    kt = (1.0 - rot_share) * target_px / mt if mt > 0 else 0.0
    kr = rot_share * target_px / mr if mr > 0 else 0.0
    m = seq_factory(kt, kr).max_flow_px(0, device)
    return kt * target_px / m, kr * target_px / m


def render_sequence(seq: Sequence, frames: Optional[Seq[int]] = None, device="cpu"):
    """Render frames into stacked float64 numpy arrays (Y, rho, w_gt) of shape
    (F, rows, cols[, 3])."""
    ks = range(seq.n_frames) if frames is None else frames
    fr = [seq.frame(k, device) for k in ks]
    return (torch.stack([f.Y for f in fr]).cpu().numpy(),
            torch.stack([f.rho for f in fr]).cpu().numpy(),
            torch.stack([f.w_gt for f in fr]).cpu().numpy())


# ----------------------------------------------------------------------------------------
# builders for the workload recipes
# ----------------------------------------------------------------------------------------
def sinusoid_plane_sequence(rows=64, cols=64, n_frames=20, seed=1, dt=1.0,
                            rho_range=(0.2, 1.0), max_flow_px=0.9, n_waves=16) -> Sequence:
    """One tilted textured plane whose inverse depth spans rho_range over the image, seen by a
    camera translating at a constant seeded velocity (no rotation)."""
    rng = np.random.default_rng(seed)
    f = cols / 1.0
    cam = Camera(rows, cols, f, f, (cols - 1) / 2.0, (rows - 1) / 2.0)
    eta = cam.rays().numpy()
    # tilt about the x axis; pick the tilt so that min/max of n.eta matches the rho ratio
    ratio = rho_range[0] / rho_range[1]
    lo_t, hi_t = 0.0, np.pi / 2 - 1e-3
    for _ in range(80):
        th = 0.5 * (lo_t + hi_t)
        n = np.array([0.0, -np.sin(th), np.cos(th)])
        ne = eta @ n
        r = ne.min() / ne.max()
        if r > ratio:
            lo_t = th
        else:
            hi_t = th
    n = np.array([0.0, -np.sin(th), np.cos(th)])
    ne = eta @ n
    dist = ne.max() / rho_range[1]
    scene = SinusoidPlaneScene(n, dist, n_waves, rng)
    direction = rng.standard_normal(3)
    direction /= np.linalg.norm(direction)

    def make(kt, kr):
        return Sequence(cam, scene, Trajectory(V=direction * kt / dt), dt, n_frames)

    kt, _ = _flow_scale(make, max_flow_px, 0.0)
    return make(kt, 0.0)


def box_sequence(rows=512, cols=512, n_frames=100, seed=2, dt=1.0 / 300.0, max_flow_px=8.0,
                 n_boxes=8, depth_range=(2.0, 50.0), depth_noise=0.01, hfov_deg=90.0,
                 rot_share=0.2, flow_margin=0.85, device="cpu") -> Sequence:
    """Seeded textured boxes and planes inside an enclosing box, a camera with constant
    linear velocity plus sinusoidal angular velocity, max image motion about max_flow_px."""
    rng = np.random.default_rng(seed)
    f = (cols / 2.0) / np.tan(np.radians(hfov_deg) / 2.0)
    cam = Camera(rows, cols, f, f, (cols - 1) / 2.0, (rows - 1) / 2.0)
    boxes = []
    dmin, dmax = depth_range
    for b in range(n_boxes):
        depth = float(np.exp(rng.uniform(np.log(dmin + 1.0), np.log(0.6 * dmax))))
        cx_ = rng.uniform(-0.8, 0.8) * depth
        cy_ = rng.uniform(-0.8, 0.8) * depth
        size = rng.uniform(0.4, 0.9, 3) * depth * np.array([0.6, 0.6, 0.6])
        if b % 2 == 1:                       # thin box = textured plane
            size[rng.integers(0, 3)] = 0.02 * depth
        c = np.array([cx_, cy_, depth + size[2] / 2.0])
        boxes.append((c - size / 2.0, c + size / 2.0))
    spac = np.array([1.6, 0.8, 0.4, 0.2]) * max(dmin, 1.0) / 2.0
    noise = ValueNoise(seed * 7919 + 1, spac, [1.0, 0.7, 0.5, 0.35])
    n_obj = n_boxes + 2
    gains = rng.uniform(0.6, 1.0, n_obj)
    biases = rng.uniform(0.35, 0.65, n_obj)
    offsets = rng.uniform(-500, 500, (n_obj, 3))
    scene = BoxScene(boxes, noise, gains, biases, offsets, enclosure=dmax)
    vdir = rng.standard_normal(3)
    vdir[2] *= 0.3
    vdir /= np.linalg.norm(vdir)
    odir = rng.standard_normal(3)
    odir /= np.linalg.norm(odir)
    freq = rng.uniform(1.0, 3.0, 3)
    phase = rng.uniform(0, 2 * np.pi, 3)

    def make(kt, kr):
        traj = Trajectory(V=vdir * kt / dt, amp=odir * kr / dt, freq=freq,
                          phase=np.full(3, np.pi / 2) if kr == 0 else phase)
        return Sequence(cam, scene, traj, dt, n_frames, depth_noise=depth_noise,
                        noise_seed=seed)

    kt, kr = _flow_scale(make, flow_margin * max_flow_px, rot_share, device)
    return make(kt, kr)


def driving_sequence(rows=1024, cols=2048, n_frames=200, seed=4, dt=1.0 / 200.0,
                     speed=15.0, n_boxes=30, max_flow_px=16.0, depth_noise=0.02,
                     cam_height=1.5, flow_margin=0.85, device="cpu") -> Sequence:
    """Ground plane plus seeded boxes, open sky (rho = 0), camera moving forward at `speed`.
    The focal length is the smallest of a few candidates whose image motion stays within
    flow_margin * max_flow_px on the first and the last frame."""
    rng = np.random.default_rng(seed)
    travel = speed * dt * n_frames
    boxes = []
    for b in range(n_boxes):
        z = rng.uniform(10.0 + travel, 120.0)
        x = rng.choice([-1.0, 1.0]) * rng.uniform(3.0, 15.0)
        w_, h_, d_ = rng.uniform(1.0, 4.0), rng.uniform(1.0, 5.0), rng.uniform(1.0, 6.0)
        lo = np.array([x - w_ / 2, cam_height - h_, z])
        hi = np.array([x + w_ / 2, cam_height, z + d_])
        boxes.append((lo, hi))
    noise = ValueNoise(seed * 7919 + 3, [1.2, 0.6, 0.3, 0.15], [1.0, 0.7, 0.5, 0.35])
    n_obj = n_boxes + 2
    gains = rng.uniform(0.6, 1.0, n_obj)
    biases = rng.uniform(0.3, 0.6, n_obj)
    offsets = rng.uniform(-500, 500, (n_obj, 3))
    scene = BoxScene(boxes, noise, gains, biases, offsets, ground_y=cam_height)

    def make_f(f):
        cam = Camera(rows, cols, f, f, (cols - 1) / 2.0, (rows - 1) / 2.0)
        traj = Trajectory(V=np.array([0.0, 0.0, speed]))
        return Sequence(cam, scene, traj, dt, n_frames, depth_noise=depth_noise,
                        noise_seed=seed)

    seq = None
    for scale in (0.5, 0.625, 0.75, 0.875, 1.0, 1.25, 1.5, 2.0, 3.0):
        seq = make_f(scale * cols)
        m = max(seq.max_flow_px(0, device), seq.max_flow_px(n_frames - 1, device))
        if m <= flow_margin * max_flow_px:
            break
    return seq
