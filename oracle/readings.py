"""Readings of the points the paper leaves silent, ambiguous or garbled.

Each field records one choice; the GPU library takes the same choices (its
configuration flags mirror dominant_literal, source_literal and cfl_clamp).

* dominant_literal (Section "Numerical prediction", dominant optical flow): the text
  calls the dominant flow the *largest* neighbouring component, while the printed
  case split picks u_{j-1} when |u_{j+1}| > |u_{j-1}|, i.e. the smaller one.  Default
  False = the text: u_hat = u_{j+1} if |u_{j+1}| > |u_{j-1}| else u_{j-1}.  True = the
  printed case split.  (With the printed split a moving edge is never transported.)
* source_literal (column/row half-steps of the same section): the printed half-steps
  apply the source term f<eta, w> with the full step in *both* passes, which doubles
  the source of eq:hflow_propagation_discrete.  Default False = half of it in each
  pass (sigma = 1/2); True = sigma = 1.
* cfl_clamp (eq:numerical_stability): the scheme is stable when dt*|u_hat| <= 1.
  Default True = clamp u_hat, v_hat to [-N, N]; False = no clamp.
* N per level: N_h = max(1, ceil(max_flow_px / 2^(h-1))), dt = 1/N_h.
* gammas (eq:cost_top and eq:cost_invdepth give no values): gamma_1 = alpha_1/dmu0^2,
  gamma_2 = alpha_2/dmu0^2, gamma_3 = alpha_3, gamma_4 = alpha_4, gamma_5 = alpha_5 with
  dmu0 = 1/sqrt(fx_h^2 + 1), the tangent-plane pixel spacing on the optical axis of
  level h.  The data terms carry dmu^2, so without the 1/dmu0^2 they would vanish.
"""
from __future__ import annotations

import dataclasses
import math

# alpha_1..alpha_5 defaults (image, depth, temporal prior, depth measurement, depth prior)
DEFAULT_ALPHA = (300.0, 1.0e3, 1.0, 1.0, 1.0)


@dataclasses.dataclass(frozen=True)
class Readings:
    dominant_literal: bool = False
    source_literal: bool = False
    cfl_clamp: bool = True

    @property
    def sigma(self) -> float:
        return 1.0 if self.source_literal else 0.5


def iterations(max_flow_px: float, level: int) -> int:
    """N_h for level h (1 = finest)."""
    return max(1, int(math.ceil(max_flow_px / 2.0 ** (level - 1))))


def gammas(alpha, fx_level: float):
    dmu0 = 1.0 / math.sqrt(fx_level * fx_level + 1.0)
    a1, a2, a3, a4, a5 = alpha
    return (a1 / dmu0 ** 2, a2 / dmu0 ** 2, a3, a4, a5)
