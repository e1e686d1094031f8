"""Named synthetic workloads: input recipe plus the filter settings they are run with.

Each entry gives a builder for a seeded Sequence and the filter parameters (levels,
maximum expected flow in pixels, smoothing passes per level, finest first).  Sizes,
rates and flow magnitudes follow the paper's own experiments (512 x 512 spherical
images at 300 Hz with flow up to 8 px; a 1024-wide driving setup) with seeded
ray-cast scenes standing in for the paper's rendered city and stereo recordings.
"""
from __future__ import annotations

import numpy as np

from .scenes import box_sequence, driving_sequence, sinusoid_plane_sequence


def _smooth(levels):
    # two passes at the finest level, four at every coarser level
    return [2] + [4] * (levels - 1)


WORKLOADS = {
    # 64 x 64, one level, 20 frames, dt = 1: sinusoid-textured tilted plane,
    # rho in [0.2, 1], constant translation, flow <= 1 px
    "plane64": dict(
        build=lambda device="cpu": sinusoid_plane_sequence(64, 64, 20, seed=1, dt=1.0),
        levels=1, max_flow_px=1.0, smooth=[2], frames=20),
    # 512 x 512, three levels, 100 frames at 300 Hz: eight seeded boxes/planes,
    # constant linear velocity plus sinusoidal rotation, flow up to 8 px, 1 % depth noise
    "boxes512": dict(
        build=lambda device="cpu": box_sequence(512, 512, 100, seed=2, dt=1.0 / 300.0,
                                                max_flow_px=8.0, device=device),
        levels=3, max_flow_px=8.0, smooth=_smooth(3), frames=100),
    # 2048 x 1024, four levels, flow up to 16 px, 200 frames at 200 Hz, ground plane +
    # 30 boxes, forward motion at 15 m/s, 2 % depth noise, open sky (rho = 0)
    "driving2048x1024": dict(
        build=lambda device="cpu": driving_sequence(1024, 2048, 200, seed=4, device=device),
        levels=4, max_flow_px=16.0, smooth=_smooth(4), frames=200),
}


def workload(name: str):
    return WORKLOADS[name]


# The shapes of the paper's runtime tables (Section "Experimental Validation", Tables
# runtime_pyramid_1, runtime_pyramid_2, runtime_pyramid_2_1024): image size, levels, smoothing
# passes per level (finest first) and the maximum flows the rows are quoted at.  Seeded box
# scenes at 300 Hz (1024 x 1024 at the ZED's 1024-wide resolution) stand in for the paper's
# rendered city and stereo recordings; the motion is scaled to each row's maximum flow.
PAPER_SWEEP = (
    dict(table="runtime_pyramid_1", size=512, levels=1, smooth=[2], flows=(1.0, 2.0, 4.0)),
    dict(table="runtime_pyramid_2", size=512, levels=2, smooth=[2, 4], flows=(1.0, 2.0, 4.0, 8.0)),
    dict(table="runtime_pyramid_2_1024", size=1024, levels=2, smooth=[2, 4],
         flows=(1.0, 2.0, 4.0, 8.0)),
)


def sweep_sequence(size: int, max_flow_px: float, n_frames: int, device="cpu"):
    return box_sequence(size, size, n_frames, seed=5, dt=1.0 / 300.0, max_flow_px=max_flow_px,
                        device=device)


_MIX_SIZES = (256, 512, 1024)


def stream_mix(n_streams: int = 64, seed: int = 3, n_frames: int = 100, device="cpu"):
    """Batched workload: n_streams independent box scenes of mixed square sizes drawn
    from {256, 512, 1024}; 3 levels (4 for 1024), max flow 4/8/16 px; scene seeds
    1000 + i.  Returns a list of dicts with the builder and filter settings."""
    rng = np.random.default_rng(seed)
    sizes = rng.choice(_MIX_SIZES, n_streams)
    out = []
    for i, s in enumerate(sizes):
        s = int(s)
        levels = 4 if s == 1024 else 3
        mf = {256: 4.0, 512: 8.0, 1024: 16.0}[s]
        out.append(dict(
            size=s, levels=levels, max_flow_px=mf, smooth=_smooth(levels),
            build=(lambda s=s, mf=mf, i=i: box_sequence(s, s, n_frames, seed=1000 + i,
                                                        dt=1.0 / 300.0, max_flow_px=mf,
                                                        device=device))))
    return out
