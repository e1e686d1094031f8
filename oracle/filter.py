"""The pyramidal structure-flow filter, one frame at a time (Section "Filter
Architecture", Fig. "Pyramidal filter architecture"; Sections "State prediction",
"State update"; initial condition from Section "Ground truth evaluation").

State per level h (h = 1 finest, H coarsest), all in the filter's time unit of one frame
(w in rad/frame):
  * top level H:   w_H, rho_H, Yhat_H (brightness model of the last frame),
  * lower levels:  w_h (reconstructed), dw_h, rho_h, Yhat_h.

push(Y, rho, dt) for frame k+1:
  S1  pyramid of Y and rho                                   (pyramid.py)
  S2  brightness model Yhat, grad_Y per level                (models.py)
  S3  inverse-depth model grad_rho per level                 (models.py)
  S4  prediction of every level from its frame-k state       (predict.py)
  S5  least-squares update of w_H / dw_h                     (update.py)
  S6  N_s passes of 5x5 smoothing of the solved field        (update.py)
  S7  inverse-depth update                                   (update.py)
  S8  reconstruction w_h = up(w_{h+1}) + dw_h, h = H-1..1     (pyramid.py)
  S9  Yhat_h <- brightness model of the new frame
With the camera's angular velocity Omega (rad/s), angular acceleration dOmega (rad/s^2) and
linear acceleration a (m/s^2), all in the camera frame and taken as constant between the two
frames (Section "Structure Flow"), push(..., omega, omega_dot, acc) keeps the inertial source
terms that the paper drops by eq:assumption (predict.py): Omega dt, dOmega dt^2 and a dt^2 in
the filter's time unit.
The first frame only initialises: w = dw = 0, rho = measured rho (0 where missing),
Yhat from the frame.  dt (seconds) only converts the output to rad/s: the scheme runs in
frames.  When dt changes between frames, w and dw are rescaled by dt_new/dt_old so that
they stay in rad/frame (the PDE is invariant under w -> c w, t -> t/c).
"""
from __future__ import annotations

import numpy as np

from . import geometry, models, predict, pyramid, update
from .readings import DEFAULT_ALPHA, Readings, gammas, iterations

LevelGeometry = geometry.Grid


class Filter:
    def __init__(self, rows: int, cols: int, levels: int, max_flow_px: float, smooth_iters,
                 fx: float, fy: float, cx: float, cy: float, alpha=DEFAULT_ALPHA,
                 readings: Readings = Readings(), eta=None):
        """eta: None for the pinhole grid of the intrinsics, or the finest level's unit
        directions (rows, cols, 3) of a general grid (Section "Spherical image data
        structure"); fx then is the nominal focal length of the weights' scaling."""
        if levels < 1:
            raise ValueError("levels must be >= 1")
        self.rows, self.cols, self.levels = int(rows), int(cols), int(levels)
        self.max_flow_px = float(max_flow_px)
        self.smooth_iters = [int(s) for s in smooth_iters][:levels]
        if len(self.smooth_iters) != levels:
            raise ValueError("one smoothing count per level is needed")
        self.readings = readings
        self.alpha = tuple(float(a) for a in alpha)
        self.grids = [geometry.Grid(rows, cols, fx, fy, cx, cy, h, eta)
                      for h in range(1, levels + 1)]
        for g in self.grids:
            if g.rows < 2 or g.cols < 2:
                raise ValueError("every pyramid level needs at least 2x2 pixels")
        self.N = [iterations(self.max_flow_px, h) for h in range(1, levels + 1)]
        self.gamma = [gammas(self.alpha, g.fx) for g in self.grids]
        self.state = None
        self.dt_prev = None

    # ------------------------------------------------------------------------------------
    def _pyramid(self, Y, rho):
        Ys, rhos = [Y], [rho]
        for _ in range(1, self.levels):
            Ys.append(pyramid.downsample(Ys[-1]))
            rhos.append(pyramid.downsample_valid(rhos[-1]))
        return Ys, rhos

    def push(self, Y, rho, dt: float, omega=None, acc=None, omega_dot=None):
        Y = np.asarray(Y, dtype=np.float64)
        rho = np.asarray(rho, dtype=np.float64)
        if Y.shape != (self.rows, self.cols) or rho.shape != (self.rows, self.cols):
            raise ValueError("frame size does not match the filter")
        if not (np.isfinite(dt) and dt > 0):
            raise ValueError("dt must be positive and finite")
        Ys, rhos = self._pyramid(Y, rho)
        bright = [models.brightness_model(y) for y in Ys]
        depth = [models.depth_model(r) for r in rhos]
        H = self.levels
        if self.state is None:
            self.state = []
            for h in range(H):
                g = self.grids[h]
                st = {"w": np.zeros((g.rows, g.cols, 3)),
                      "rho": np.where(np.isnan(rhos[h]), 0.0, rhos[h]),
                      "Y": bright[h][0]}
                if h < H - 1:
                    st["dw"] = np.zeros((g.rows, g.cols, 3))
                self.state.append(st)
            self.dt_prev = float(dt)
            return
        if dt != self.dt_prev:
            c = dt / self.dt_prev
            for st in self.state:
                st["w"] = st["w"] * c
                if "dw" in st:
                    st["dw"] = st["dw"] * c
        imu = None
        if omega is not None or acc is not None or omega_dot is not None:
            def vec(v):
                return np.zeros(3) if v is None else np.asarray(v, dtype=np.float64)
            imu = (vec(omega) * dt, vec(omega_dot) * dt * dt, vec(acc) * dt * dt)
        x = [None] * H
        new_rho = [None] * H
        for h in range(H):
            g = self.grids[h]
            st = self.state[h]
            top = h == H - 1
            names = ("w", "rho") if top else ("w", "dw", "rho", "Y")
            pred = predict.predict(g, {k: st[k] for k in names}, self.N[h], self.readings, imu)
            Yhat_new, dY1, dY2 = bright[h]
            gradY = models.to_tangent(g.dmu, g.b1, g.b2, dY1, dY2)
            rhohat, dr1, dr2 = depth[h]
            gradrho = models.to_tangent(g.dmu, g.b1, g.b2, dr1, dr2)
            if top:
                x0, Yprev, rhoprev = pred["w"], st["Y"], st["rho"]
            else:
                x0, Yprev, rhoprev = pred["dw"], pred["Y"], pred["rho"]
            g1, g2, g3, g4, g5 = self.gamma[h]
            terms = update.ls_terms(g, gradY, Yhat_new, Yprev, gradrho, rhohat, rhoprev)
            xs = update.ls_solve(*terms, x0, g1, g2, g3)
            x[h] = update.smooth(xs, self.smooth_iters[h])
            new_rho[h] = update.rho_update(rhohat, pred["rho"], g4, g5)
        # reconstruction, coarse to fine
        self.state[H - 1]["w"] = x[H - 1]
        for h in range(H - 2, -1, -1):
            g = self.grids[h]
            self.state[h]["dw"] = x[h]
            self.state[h]["w"] = pyramid.upsample(self.state[h + 1]["w"], g.rows, g.cols) + x[h]
        for h in range(H):
            self.state[h]["rho"] = new_rho[h]
            self.state[h]["Y"] = bright[h][0]
        self.dt_prev = float(dt)

    # ------------------------------------------------------------------------------------
    def flow(self, kind: str = "w_rad_s") -> np.ndarray:
        """Finest-level output: 'w_rad_s' (rows, cols, 3) structure flow in rad/s;
        'tangent_px' (rows, cols, 2) = B^T P w / dmu and 'normal_px' (rows, cols) =
        <eta, w> / dmu in pixels per frame (eq:tangent_flow, eq:normal_flow);
        'w_frame' (rows, cols, 3) in rad/frame; 'rho' (rows, cols)."""
        if self.state is None:
            raise RuntimeError("no frame has been pushed")
        g = self.grids[0]
        w = self.state[0]["w"]
        if kind == "w_rad_s":
            return w / self.dt_prev
        if kind == "w_frame":
            return w.copy()
        if kind == "tangent_px":
            Pw = np.einsum("rcab,rcb->rca", g.P, w)
            return np.einsum("rcab,rca->rcb", g.B, Pw) / g.dmu[..., None]
        if kind == "normal_px":
            return np.sum(g.eta * w, axis=-1) / g.dmu
        if kind == "rho":
            return self.state[0]["rho"].copy()
        raise ValueError(kind)

    def get_state(self):
        return None if self.state is None else [{k: v.copy() for k, v in st.items()}
                                                 for st in self.state]

    def set_state(self, state, dt_prev: float):
        self.state = [{k: np.asarray(v, dtype=np.float64).copy() for k, v in st.items()}
                      for st in state]
        self.dt_prev = float(dt_prev)
