"""Seeded synthetic inputs for the structure-flow filter.

This package renders brightness images Y, inverse-depth maps rho and ground-truth
structure flow for moving pinhole cameras in simple seeded scenes.  It holds the
scene, camera-motion and ray-casting code only: none of the filter's arithmetic
lives here, so both the CPU oracle and the GPU path may consume what it produces.
"""
from .scenes import (Camera, Trajectory, Sequence, SinusoidPlaneScene,  # noqa: F401
                     BoxScene, render_sequence)
from .workloads import WORKLOADS, workload, stream_mix  # noqa: F401
