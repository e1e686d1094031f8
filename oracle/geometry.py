"""Spherical grid geometry (Section "Spherical image data structure", eq:tmatrix,
eq:tspace_projection, eq:beta_to_mu).

For every pixel p = (i, j) of a level:
  * eta_p      unit direction on the sphere,
  * P_p        = I - eta eta^T, the projector onto the tangent space (eq:tmatrix),
  * b1_p, b2_p orthonormal tangent basis: b1 along the projection of the next column's
               direction eta_{i,j+1}, b2 = eta x b1 oriented toward the next row,
  * dmu_p      = |P_p eta_{i,j+1}|, the tangent-plane distance to the next column.
B = [b1 b2] is a 3x2 matrix with orthonormal columns; 2-D tangent coordinates map to
3-D by B (.) and back by B^T (.).  In the last column the previous column is used
(its projection points the other way, so it is negated); in the last row the
orientation of b2 is checked against the previous row.

The pinhole grid of level h samples the level-1 grid at every 2^(h-1)-th pixel,
eta^h_{ij} = eta^1_{2^(h-1) i, 2^(h-1) j}, which is the pinhole with fx, fy, cx, cy
divided by 2^(h-1).  A general grid of unit directions (a Spherepix patch, an equiangular or
fisheye camera) is given as its finest level, and the coarser levels sample it the same way.
"""
from __future__ import annotations

import numpy as np


def level_shape(rows: int, cols: int, level: int):
    r, c = rows, cols
    for _ in range(level - 1):
        r, c = (r + 1) // 2, (c + 1) // 2
    return r, c


def level_intrinsics(fx, fy, cx, cy, level: int):
    s = 2.0 ** (level - 1)
    return fx / s, fy / s, cx / s, cy / s


def pinhole_eta(rows: int, cols: int, fx: float, fy: float, cx: float, cy: float) -> np.ndarray:
    """Unit directions (rows, cols, 3): normalize(((j - cx)/fx, (i - cy)/fy, 1))."""
    j = np.arange(cols, dtype=np.float64)[None, :]
    i = np.arange(rows, dtype=np.float64)[:, None]
    r = np.zeros((rows, cols, 3))
    r[..., 0] = (j - cx) / fx
    r[..., 1] = (i - cy) / fy
    r[..., 2] = 1.0
    return r / np.sqrt(np.sum(r * r, axis=-1, keepdims=True))


def projector(eta: np.ndarray) -> np.ndarray:
    """P = I - eta eta^T per pixel, (..., 3, 3)."""
    return np.eye(3) - eta[..., :, None] * eta[..., None, :]


def tangent_frame(eta: np.ndarray):
    """b1, b2 (rows, cols, 3) and dmu (rows, cols) for a grid of unit directions."""
    rows, cols, _ = eta.shape
    if cols < 2:
        raise ValueError("the tangent basis needs at least two columns")
    P = projector(eta)
    # neighbour in the next column; the last column uses the previous one, negated
    nxt = np.concatenate([eta[:, 1:], eta[:, -2:-1]], axis=1)
    sign = np.ones((rows, cols))
    sign[:, -1] = -1.0
    q = np.einsum("rcab,rcb->rca", P, nxt)
    dmu = np.sqrt(np.sum(q * q, axis=-1))
    b1 = sign[..., None] * q / dmu[..., None]
    c = np.cross(eta, b1)
    c /= np.sqrt(np.sum(c * c, axis=-1, keepdims=True))
    # orient b2 toward the next row (the last row: away from the previous row)
    if rows >= 2:
        below = np.concatenate([eta[1:], eta[-2:-1]], axis=0)
        s = np.sum(c * below, axis=-1)
        s[-1] = -s[-1]
        c = np.where((s < 0)[..., None], -c, c)
    return b1, c, dmu


def subsample(eta1: np.ndarray, level: int) -> np.ndarray:
    """Level h of a grid given at the finest level: every 2^(h-1)-th direction."""
    s = 2 ** (level - 1)
    return np.ascontiguousarray(eta1[::s, ::s])


class Grid:
    """Geometry of one pyramid level: the pinhole grid of the intrinsics, or, with eta1 (the
    finest level's unit directions, (rows, cols, 3)), that grid sampled for the level (the
    intrinsics then only give the nominal focal length of the weights, readings.gammas)."""

    def __init__(self, rows, cols, fx, fy, cx, cy, level, eta1=None):
        self.level = level
        self.rows, self.cols = level_shape(rows, cols, level)
        self.fx, self.fy, self.cx, self.cy = level_intrinsics(fx, fy, cx, cy, level)
        if eta1 is None:
            self.eta = pinhole_eta(self.rows, self.cols, self.fx, self.fy, self.cx, self.cy)
        else:
            eta1 = np.asarray(eta1, dtype=np.float64)
            if eta1.shape != (rows, cols, 3):
                raise ValueError("eta must be (rows, cols, 3)")
            self.eta = subsample(eta1, level)
            assert self.eta.shape == (self.rows, self.cols, 3)
        self.P = projector(self.eta)
        self.b1, self.b2, self.dmu = tangent_frame(self.eta)
        # B as (rows, cols, 3, 2) with columns b1, b2
        self.B = np.stack([self.b1, self.b2], axis=-1)
