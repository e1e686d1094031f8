"""Image pyramid and flow reconstruction (Section "Filter Architecture",
eq:hflow_reconstruction).

The paper builds an H-level pyramid (h = 1 finest) but does not say how.  Reading:
level h+1 is the 5x5 Gaussian blur (g = [1, 4, 6, 4, 1]/16 in each axis, clamped
borders) of level h sampled at (2i, 2j); sizes halve rounding up.  Inverse depth is
blurred over the valid (non-NaN) samples only and normalised by their total weight;
a pixel with no valid sample stays missing (NaN).

Reconstruction (eq:hflow_reconstruction), applied for h = H-1, ..., 1:
w_h = up(w_{h+1}) + dw_h, where up() samples w_{h+1} bilinearly at (i/2, j/2) with
clamped borders.  Structure flow is an angular rate, so it is not rescaled between
levels (unlike optical flow in pixels).
"""
from __future__ import annotations

import numpy as np

from .models import G1D, OFFSETS, _clamped


def downsample(Y: np.ndarray) -> np.ndarray:
    acc = np.zeros_like(Y)
    for a, ga in zip(OFFSETS, G1D):
        for b, gb in zip(OFFSETS, G1D):
            acc += ga * gb * _clamped(Y, a, b)
    return acc[::2, ::2].copy()


def downsample_valid(rho: np.ndarray) -> np.ndarray:
    valid = ~np.isnan(rho)
    r0 = np.where(valid, rho, 0.0)
    num = np.zeros_like(r0)
    den = np.zeros_like(r0)
    for a, ga in zip(OFFSETS, G1D):
        for b, gb in zip(OFFSETS, G1D):
            num += ga * gb * _clamped(r0, a, b)
            den += ga * gb * _clamped(valid.astype(np.float64), a, b)
    with np.errstate(invalid="ignore", divide="ignore"):
        out = np.where(den > 0, num / np.where(den > 0, den, 1.0), np.nan)
    return out[::2, ::2].copy()


def upsample(W: np.ndarray, rows: int, cols: int) -> np.ndarray:
    """Bilinear sample of the coarse field W at (i/2, j/2) for a (rows, cols) grid."""
    R, C = W.shape[:2]
    i = np.arange(rows)
    j = np.arange(cols)
    i0, j0 = i // 2, j // 2
    i1, j1 = np.minimum(i0 + 1, R - 1), np.minimum(j0 + 1, C - 1)
    fi = (0.5 * (i % 2))[:, None]
    fj = (0.5 * (j % 2))[None, :]
    if W.ndim == 3:
        fi, fj = fi[..., None], fj[..., None]
    return ((1 - fi) * (1 - fj) * W[i0][:, j0] + (1 - fi) * fj * W[i0][:, j1]
            + fi * (1 - fj) * W[i1][:, j0] + fi * fj * W[i1][:, j1])
