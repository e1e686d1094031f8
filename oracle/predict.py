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


def predict(grid, fields: dict, N: int, readings) -> dict:
    """Integrate the fields over one frame; `fields` must contain the transporting 'w'.
    Returns the predicted fields (the k+ state)."""
    sourced = {"w": True, "dw": True, "rho": True, "Y": False}
    f = {k: v.copy() for k, v in fields.items()}
    for _ in range(N):
        f = half_step(grid, f, 1, N, readings, sourced)
        f = half_step(grid, f, 0, N, readings, sourced)
    return f
