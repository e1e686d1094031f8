"""Mapping a camera's image and inverse depth onto the filter's grid of directions (Section
"Experimental Validation": the timed path maps the image and depth measurements onto the
Spherepix grid before the filter runs; Section "Spherical image data structure").

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The source is a pinhole camera (fx, fy, cx, cy; rows x cols).  Grid direction eta projects to
the source pixel coordinates
    u = fx eta_x / eta_z + cx,   v = fy eta_y / eta_z + cy        (eta_z > 0),
and the grid's values are interpolated there (the paper does not say how; reading R24):
  * brightness: bilinear, the source clamped to its edge (directions outside the image take
    the nearest edge values);
  * inverse depth (NaN = missing): bilinear over the valid neighbours only (their weights
    renormalised), NaN when the valid neighbours carry less than half of the weight (so that a
    direction on a missing pixel stays missing whatever the rounding of its coordinates) or
    the direction falls outside the image (by more than 1e-3 px, so that the image's own edge
    pixels stay inside whatever the rounding) or behind the camera (eta_z <= 0).
"""
from __future__ import annotations

import numpy as np


def source_coords(eta: np.ndarray, fx: float, fy: float, cx: float, cy: float):
    """(u, v, ahead) per grid direction."""
    ez = eta[..., 2]
    ahead = ez > 0
    safe = np.where(ahead, ez, 1.0)
    return fx * eta[..., 0] / safe + cx, fy * eta[..., 1] / safe + cy, ahead


def map_frame(Y: np.ndarray, rho: np.ndarray, eta: np.ndarray, fx: float, fy: float,
              cx: float, cy: float):
    """Y, rho on the source camera (rows x cols) -> on the grid eta (R x C x 3)."""
    rows, cols = Y.shape
    u, v, ahead = source_coords(eta, fx, fy, cx, cy)
    tol = 1e-3
    inside = ahead & (u >= -tol) & (u <= cols - 1 + tol) & (v >= -tol) & (v <= rows - 1 + tol)
    uc = np.clip(np.where(ahead, u, 0.0), 0, cols - 1)
    vc = np.clip(np.where(ahead, v, 0.0), 0, rows - 1)
    j0 = np.minimum(np.floor(uc).astype(int), cols - 1)
    i0 = np.minimum(np.floor(vc).astype(int), rows - 1)
    j1 = np.minimum(j0 + 1, cols - 1)
    i1 = np.minimum(i0 + 1, rows - 1)
    fu, fv = uc - j0, vc - i0
    corners = ((i0, j0, (1 - fv) * (1 - fu)), (i0, j1, (1 - fv) * fu),
               (i1, j0, fv * (1 - fu)), (i1, j1, fv * fu))
    Yg = sum(w * Y[i, j] for i, j, w in corners)
    num = np.zeros(eta.shape[:2])
    den = np.zeros(eta.shape[:2])
    for i, j, w in corners:
        r = rho[i, j]
        ok = ~np.isnan(r)
        num += np.where(ok, w * np.where(ok, r, 0.0), 0.0)
        den += np.where(ok, w, 0.0)
    ok = inside & (den >= 0.5)
    rg = np.where(ok, num / np.where(ok, den, 1.0), np.nan)
    return Yg, rg
