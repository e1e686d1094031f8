"""FP64 CPU oracle of the structure-flow predictor-update filter.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the tests, the smoke
check and the CPU-baseline leg of the benchmark may import it; the product path
never does.  It shares no code with the HIP library.

It follows Adarve & Mahony, "Real-time Structure Flow" (arXiv 2406.18031):
  * geometry.py  - spherical grid, tangent bases and pixel spacing
                   (Section "Spherical image data structure")
  * models.py    - brightness model (eq:img_model, eq:img_gradient) and inverse-depth
                   model (eq:dominant_b1, eq:dominant_b2, eq:inv_depth_gradient)
  * predict.py   - numerical prediction (Section "Numerical prediction",
                   eq:hflow_propagation_discrete, eq:oflow_numeric, eq:numerical_stability)
  * update.py    - least-squares update (eq:cost_top, eq:cost_bottom, eq:LS_update),
                   smoothing, inverse-depth update (eq:cost_invdepth)
  * pyramid.py   - image pyramid and flow reconstruction (eq:hflow_reconstruction)
  * filter.py    - the per-frame filter (Section "Filter Architecture")
  * literal.py   - an independent per-pixel loop version for tiny images (pin)
  * metrics.py   - endpoint error (eq:RMSE_vel), angular error, tangent/normal flow

Readings of points where the paper is silent or garbled are listed in readings.py.
"""
from .readings import Readings, DEFAULT_ALPHA  # noqa: F401
from .filter import Filter, LevelGeometry  # noqa: F401
