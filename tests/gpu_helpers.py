"""Shared helpers of the GPU parity tests: run the HIP library and the oracle on the same
seeded inputs and compare them."""
from __future__ import annotations

import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(a, dtype="float32"):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a, dtype=dtype), device="cuda")


def rounded(a, storage):
    """The values the GPU sees, promoted back to float64 for the oracle."""
    dt = np.float16 if storage == 1 else np.float32
    return np.asarray(a).astype(dt).astype(np.float64)


def gpu_flow_frame(f):
    """GPU w in rad/frame as (rows, cols, 3) float64."""
    from paper_2406_18031_amd import sflow
    return f.flow(sflow.SF_FLOW_W_FRAME).cpu().numpy().transpose(1, 2, 0).astype(np.float64)


def epe_px(wa, wb, dmu):
    e = np.sqrt(np.sum((wa - wb) ** 2, axis=-1)) / dmu
    return {"mean": float(e.mean()), "p99": float(np.percentile(e, 99)), "max": float(e.max())}


def make_pair(R, C, H, mf, smooth, cam, alpha=None, storage=0, read_flags=0):
    from oracle import Filter as OFilter, Readings
    from paper_2406_18031_amd import sflow
    alpha = alpha or sflow.DEFAULT_ALPHA
    rd = Readings(dominant_literal=bool(read_flags & 1), source_literal=bool(read_flags & 2),
                  cfl_clamp=not (read_flags & 4))
    o = OFilter(R, C, H, mf, smooth, *cam, alpha=alpha, readings=rd)
    g = sflow.Filter(R, C, H, mf, smooth, *cam, alpha=alpha, storage=storage,
                     read_flags=read_flags)
    return o, g
