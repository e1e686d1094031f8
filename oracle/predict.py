"""State prediction by the upwind finite-difference scheme (Section "State prediction",
eq:hflow_propagation_top/low, eq:dhflow_propagation_low, eq:invdepth_propagation_low,
eq:img_propagation_low; Section "Numerical prediction", eq:hflow_propagation_discrete,
eq:oflow_numeric, eq:numerical_stability).

One frame is integrated with N steps of length dt = 1/N (time unit = one frame).  Each
step is a column (beta_1) half-step followed by a row (beta_2) half-step:

  column:  u_p = b1_p . (P_p w_p) / dmu_p                         (eq:oflow_numeric)
           u_hat_p = dominant neighbour of u_{i,j-1}, u_{i,j+1}
           s_p = <eta_p, w_p>
           f <- f - dt [ u_hat D_1(f; u_hat) + sigma f s ]      for f in the fields,
  row:     the same along i with v = b2 . (P w*) / dmu and s from the half-stepped w*.

D is the upwind difference: backward (f_p - f_prev) if the dominant flow is positive,
forward (f_next - f_p) otherwise.  Neighbours are clamped at the image border.  The
transported image has no source term.  Readings (dominant rule, sigma, clamping of
u_hat to [-N, N]) are in readings.py.

Top level: fields {w, rho} transported by w.  Lower levels: {w, dw, rho, Y} all
transported by the level's reconstructed flow w, with dw and rho also carrying the
source term with <eta, w> (w of the same level: the printed eq:invdepth_propagation_low
has w^H in the transport term, read as w^h).

Inertial source terms (optional).  The paper drops the terms -Omega x w + a_w of
eq:hflow_conservation (eq:assumption), where a_w = -rho a - Omega x (w + Omega x eta) is the
field acceleration of Section "Structure Flow".  (The printed a_w has +rho a; differentiating
w = -Omega x eta - rho v with dv/dt = -Omega x v + a, eq:camvel_dot, gives -rho a, and the
accelerating-plane pin fails with the printed sign.)  The derivation takes Omega constant
(eq:totaldev_camangvel); when it changes, differentiating -Omega x eta adds -dOmega/dt x eta,
which is kept too when the angular acceleration is given.  With the camera's angular velocity
Omega, angular acceleration dOmega and linear acceleration a (in the filter's time unit:
rad/frame, rad/frame^2, 1/frame^2), each step ends with an explicit step of length dt of
    dw/dt  = -2 Omega x w - Omega x (Omega x eta) - dOmega x eta - rho a   (w, every level)
    ddw/dt = -2 Omega x dw                                               (dw, lower levels)
The increment dw = w_h - up(w_{h+1}) takes the part that is linear in the field: the terms
that do not depend on it cancel between a level and its parent up to the difference of
their inverse depths.  rho and Y have no inertial terms (eq:invdepth_conservation,
eq:image_conservation).
"""
from __future__ import annotations

import numpy as np

from .models import _clamped


def flow_u(grid, w):
    Pw = np.einsum("rcab,rcb->rca", grid.P, w)
    return np.sum(grid.b1 * Pw, axis=-1) / grid.dmu


def flow_v(grid, w):
    Pw = np.einsum("rcab,rcb->rca", grid.P, w)
    return np.sum(grid.b2 * Pw, axis=-1) / grid.dmu


def dominant(prev: np.ndarray, nxt: np.ndarray, literal: bool) -> np.ndarray:
    """Dominant optical flow from the two neighbours along the pass's axis."""
    larger_next = np.abs(nxt) > np.abs(prev)
    if literal:
        return np.where(larger_next, prev, nxt)
    return np.where(larger_next, nxt, prev)


def _shift(a, axis, step):
    return _clamped(a, step, 0) if axis == 0 else _clamped(a, 0, step)


def half_step(grid, fields: dict, axis: int, N: int, readings, sourced: dict) -> dict:
    """One half-step along `axis` (1 = columns / beta_1, 0 = rows / beta_2)."""
    w = fields["w"]
    dt = 1.0 / N
    u = flow_u(grid, w) if axis == 1 else flow_v(grid, w)
    uhat = dominant(_shift(u, axis, -1), _shift(u, axis, +1), readings.dominant_literal)
    if readings.cfl_clamp:
        uhat = np.clip(uhat, -float(N), float(N))
    s = np.sum(grid.eta * w, axis=-1)
    out = {}
    for name, f in fields.items():
        uh = uhat if f.ndim == 2 else uhat[..., None]
        ss = s if f.ndim == 2 else s[..., None]
        D = np.where(uh > 0, f - _shift(f, axis, -1), _shift(f, axis, +1) - f)
        sigma = readings.sigma if sourced[name] else 0.0
        out[name] = f - dt * (uh * D + sigma * f * ss)
    return out


def inertial_step(grid, fields: dict, dt: float, imu) -> dict:
    """An explicit step of length dt of the inertial source terms; imu = (Omega, dOmega, a) as
    3-vectors in rad/frame, rad/frame^2 and 1/frame^2."""
    om = np.asarray(imu[0], dtype=np.float64)
    dom = np.asarray(imu[1], dtype=np.float64)
    acc = np.asarray(imu[2], dtype=np.float64)
    out = dict(fields)
    w = fields["w"]
    centripetal = np.cross(om, np.cross(om, grid.eta))
    out["w"] = w + dt * (-2.0 * np.cross(om, w) - centripetal - np.cross(dom, grid.eta)
                         - fields["rho"][..., None] * acc)
    if "dw" in fields:
        out["dw"] = fields["dw"] + dt * (-2.0 * np.cross(om, fields["dw"]))
    return out


def predict(grid, fields: dict, N: int, readings, imu=None) -> dict:
    """Integrate the fields over one frame; `fields` must contain the transporting 'w'.
    imu: None (the paper's eq:assumption) or (Omega, dOmega, a) in rad/frame, rad/frame^2 and
    1/frame^2.
    Returns the predicted fields (the k+ state)."""
    sourced = {"w": True, "dw": True, "rho": True, "Y": False}
    f = {k: v.copy() for k, v in fields.items()}
    for _ in range(N):
        f = half_step(grid, f, 1, N, readings, sourced)
        f = half_step(grid, f, 0, N, readings, sourced)
        if imu is not None:
            f = inertial_step(grid, f, 1.0 / N, imu)
    return f
