"""Error metrics (Section "Ground truth evaluation", eq:RMSE_vel and the angular error).

Endpoint error per pixel |w_a - w_b| / dmu with w in rad/frame, i.e. in pixels; the
paper's "average RMSE" is its mean over the image.  The angular error's printed
normalisation sqrt(1 + w) is read as sqrt(1 + |w|^2), evaluated on w / dmu.
"""
from __future__ import annotations

import numpy as np


def epe_field(wa: np.ndarray, wb: np.ndarray, dmu: np.ndarray) -> np.ndarray:
    return np.sqrt(np.sum((np.asarray(wa, np.float64) - np.asarray(wb, np.float64)) ** 2,
                          axis=-1)) / dmu


def epe_stats(wa, wb, dmu) -> dict:
    e = epe_field(wa, wb, dmu)
    return {"mean": float(e.mean()), "p99": float(np.percentile(e, 99)),
            "max": float(e.max())}


def aae_deg(w_gt: np.ndarray, w: np.ndarray, dmu: np.ndarray) -> float:
    a = w_gt / dmu[..., None]
    b = w / dmu[..., None]
    num = 1.0 + np.sum(a * b, axis=-1)
    den = np.sqrt(1.0 + np.sum(a * a, axis=-1)) * np.sqrt(1.0 + np.sum(b * b, axis=-1))
    return float(np.degrees(np.arccos(np.clip(num / den, -1.0, 1.0))).mean())
