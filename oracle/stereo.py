"""Inverse depth from a rectified stereo pair (the paper's future work, Section "Conclusions and
Future Work": express the depth measurements in terms of image disparity of a coupled stereo
pair so that the update runs on image data only).  Not in the paper; this is the design the
library implements, written plainly.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Geometry.  The left camera is the filter's pinhole camera (fx, fy, cx, cy); the right camera
has the same intrinsics and orientation, its centre `baseline` metres along the left camera's
x axis.  A point at inverse range rho along the left direction eta (Section "Structure Flow",
eq:inv_depth) has depth Z = eta_z / rho and appears in the right image on the same row,
d = fx baseline / Z = kappa rho pixels to the left, kappa = fx baseline / eta_z
(= fx baseline sqrt(x^2 + y^2 + 1), x = (j - cx)/fx, y = (i - cy)/fy).  Brightness constancy
across the pair: Y_R(i, j - d) = Y_L(i, j).

Per pixel (i, j):
  1. block matching: the integer d in [0, D] minimising the sum of absolute differences
     |Y_R(i+a, j+c-d) - Y_L(i+a, j+c)| over the 5x5 window (a, c in -2..2, rows and columns
     clamped to the image), the smallest d on ties.  The sums are taken in float32, over a
     then c, so that the same decisions come out of any float32 implementation that adds in
     that order (the GPU's).
  2. refinement: n Gauss-Newton steps on the window's squared residuals r = Y_R(i+a, j+c-d) -
     Y_L(i+a, j+c), Y_R interpolated linearly along the row (its slope g between the two
     neighbouring samples): d <- d + sum(g r) / (sum(g^2) + eps), kept in [0, D + 1].
  3. the measurement rho = d / kappa, missing (NaN) where the window has too little texture
     along the row (sum g^2 < texture), where the match is poor (mean |r| > residual) after
     the refinement, or where the point leaves the right image (j - d < 0).
"""
from __future__ import annotations

import numpy as np

WIN = 2          # window radius (5x5)


def kappa(rows: int, cols: int, fx: float, fy: float, cx: float, cy: float, baseline: float):
    """Disparity per unit inverse range, (rows, cols)."""
    j = np.arange(cols, dtype=np.float64)[None, :]
    i = np.arange(rows, dtype=np.float64)[:, None]
    x = (j - cx) / fx
    y = (i - cy) / fy
    return fx * baseline * np.sqrt(x * x + y * y + 1.0)


def block_match(YL: np.ndarray, YR: np.ndarray, dmax: int) -> np.ndarray:
    """Integer disparity per pixel (step 1), float32 sums in the stated order."""
    YL = np.asarray(YL, dtype=np.float32)
    YR = np.asarray(YR, dtype=np.float32)
    R, C = YL.shape
    ii = np.arange(R)[:, None]
    jj = np.arange(C)[None, :]
    best = np.full((R, C), np.inf, dtype=np.float32)
    dbest = np.zeros((R, C), dtype=np.int64)
    for d in range(dmax + 1):
        s = np.zeros((R, C), dtype=np.float32)
        for a in range(-WIN, WIN + 1):
            ri = np.clip(ii + a, 0, R - 1)
            for c in range(-WIN, WIN + 1):
                cl = np.clip(jj + c, 0, C - 1)
                cr = np.clip(jj + c - d, 0, C - 1)
                s = s + np.abs(YR[ri, cr] - YL[ri, cl])
        better = s < best
        best = np.where(better, s, best)
        dbest = np.where(better, d, dbest)
    return dbest


def _window_terms(YL, YR, d):
    """sum(g^2), sum(g r), mean |r| over the window at (fractional) disparity d."""
    R, C = YL.shape
    ii = np.arange(R)[:, None]
    jj = np.arange(C)[None, :]
    A = np.zeros((R, C))
    B = np.zeros((R, C))
    E = np.zeros((R, C))
    for a in range(-WIN, WIN + 1):
        ri = np.clip(ii + a, 0, R - 1)
        for c in range(-WIN, WIN + 1):
            xs = np.clip(jj + c - d, 0.0, C - 1.0)
            j0 = np.minimum(np.floor(xs).astype(np.int64), C - 1)
            j1 = np.minimum(j0 + 1, C - 1)
            t = xs - j0
            yr = (1.0 - t) * YR[ri, j0] + t * YR[ri, j1]
            g = YR[ri, j1] - YR[ri, j0]
            r = yr - YL[ri, np.clip(jj + c, 0, C - 1)]
            A += g * g
            B += g * r
            E += np.abs(r)
    return A, B, E / (2 * WIN + 1) ** 2


def disparity(YL, YR, dmax: int, iters: int = 3, eps: float = 1e-6):
    """Refined disparity (steps 1-2) and the final window terms."""
    YL = np.asarray(YL, dtype=np.float64)
    YR = np.asarray(YR, dtype=np.float64)
    d = block_match(YL, YR, dmax).astype(np.float64)
    for _ in range(iters):
        A, B, _ = _window_terms(YL, YR, d)
        d = np.clip(d + B / (A + eps), 0.0, dmax + 1.0)
    A, _, E = _window_terms(YL, YR, d)
    return d, A, E


def stereo_rho(YL, YR, fx, fy, cx, cy, baseline, dmax, iters=3, texture=2.5e-3,
               residual=0.05):
    """The inverse-depth measurement of the left image from the pair (step 3)."""
    R, C = np.asarray(YL).shape
    d, A, E = disparity(YL, YR, dmax, iters)
    jj = np.arange(C)[None, :]
    ok = (A >= texture) & (E <= residual) & (jj - d >= 0.0)
    return np.where(ok, d / kappa(R, C, fx, fy, cx, cy, baseline), np.nan)
