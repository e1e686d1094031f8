"""Brightness and inverse-depth model extraction.

Brightness (Section "Brightness parameters extraction", eq:img_model, eq:img_gradient).
For each pixel p the linear model Y_q ~ Yhat_p + dY1 (q_j - p_j) + dY2 (q_i - p_i) is fit
over the 5x5 window around p with Gaussian weights G(q - p) = g(q_i - p_i) g(q_j - p_j),
g = [1, 4, 6, 4, 1]/16.  Reading: the offset is (q - p) so that (dY1, dY2) is the gradient
toward increasing column/row (the printed (p - q) would give its negative).  The image is
clamp-padded at its borders.  For these weights sum G = 1, sum G d = 0, sum G d^2 = 1 and
all cross sums vanish, so the weighted normal matrix is the identity and the fit is

    Yhat = sum_q G Y_q,   dY1 = sum_q G (q_j - p_j) Y_q,   dY2 = sum_q G (q_i - p_i) Y_q,

which is what `brightness_model` computes, term by term.  The 3-D gradient is
grad_Y = dmu (b1 dY1 + b2 dY2) (eq:img_gradient, with B mapping 2-D to 3-D).

Inverse depth (Section "Inverse depth parameters extraction", eq:dominant_b1/b2,
Table diff_operators, eq:inv_depth_gradient).  Along each axis the one-sided difference
of smaller magnitude is used, the forward one on a tie.  Neighbours are clamped at the
image border (so the outward difference is 0).  NaN marks a missing measurement: a
difference that involves one cannot be used and the other one is taken; if neither can be
used the component is 0.  rhohat_p is the raw measurement.
"""
from __future__ import annotations

import numpy as np

G1D = np.array([1.0, 4.0, 6.0, 4.0, 1.0]) / 16.0
OFFSETS = (-2, -1, 0, 1, 2)


def _clamped(a: np.ndarray, di: int, dj: int) -> np.ndarray:
    """a[clamp(i + di), clamp(j + dj)] for every (i, j)."""
    rows, cols = a.shape[:2]
    ii = np.clip(np.arange(rows) + di, 0, rows - 1)
    jj = np.clip(np.arange(cols) + dj, 0, cols - 1)
    return a[ii][:, jj]


def brightness_model(Y: np.ndarray):
    """(Yhat, dY1, dY2), each (rows, cols): constant term and 2-D gradient along the
    column (j) and row (i) axes."""
    Yhat = np.zeros_like(Y)
    d1 = np.zeros_like(Y)
    d2 = np.zeros_like(Y)
    for a, ga in zip(OFFSETS, G1D):          # a = q_i - p_i
        for b, gb in zip(OFFSETS, G1D):      # b = q_j - p_j
            Yq = _clamped(Y, a, b)
            G = ga * gb
            Yhat += G * Yq
            d1 += G * b * Yq
            d2 += G * a * Yq
    return Yhat, d1, d2


def to_tangent(dmu, b1, b2, d1, d2):
    """3-D tangent vector dmu (b1 d1 + b2 d2), (rows, cols, 3)."""
    return dmu[..., None] * (b1 * d1[..., None] + b2 * d2[..., None])


def _min_abs(dp: np.ndarray, dm: np.ndarray) -> np.ndarray:
    choose_fwd = np.abs(dp) <= np.abs(dm)
    out = np.where(choose_fwd, dp, dm)
    out = np.where(np.isnan(dp), dm, out)
    out = np.where(np.isnan(dm), dp, out)
    out = np.where(np.isnan(dp) & np.isnan(dm), 0.0, out)
    return out


def depth_model(rho: np.ndarray):
    """(rhohat, drho1, drho2): raw inverse depth and its occlusion-aware 2-D gradient."""
    fwd1 = _clamped(rho, 0, 1) - rho         # delta+ along beta_1 (columns)
    bwd1 = rho - _clamped(rho, 0, -1)        # delta- along beta_1
    fwd2 = _clamped(rho, 1, 0) - rho         # delta+ along beta_2 (rows)
    bwd2 = rho - _clamped(rho, -1, 0)
    d1 = _min_abs(fwd1, bwd1)
    d2 = _min_abs(fwd2, bwd2)
    missing = np.isnan(rho)
    d1 = np.where(missing, 0.0, d1)
    d2 = np.where(missing, 0.0, d2)
    return rho.copy(), d1, d2
