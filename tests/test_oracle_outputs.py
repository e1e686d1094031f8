"""Pins for the oracle's output kinds and error metrics (Section "Ground truth evaluation":
eq:tangent_flow, eq:normal_flow, eq:RMSE_vel and the angular error).

The flow outputs are checked on states built from closed forms, so a transposed basis, a
missing projector, a dropped 1/dmu or a wrong component order fails one of them; the
angular error against hand-computed angles.
"""
import math

import numpy as np
import pytest

from oracle import Filter
from oracle.metrics import aae_deg, epe_field, epe_stats


def _filter_with_w(w, R=9, C=11, fx=30.0, fy=27.0, cx=5.0, cy=4.0, rho=None):
    f = Filter(R, C, 1, 1.0, [2], fx, fy, cx, cy)
    g = f.grids[0]
    st = {"w": w(g), "rho": np.full((R, C), 0.5) if rho is None else rho,
          "Y": np.zeros((R, C))}
    f.set_state([st], 0.25)
    return f, g


def test_tangent_and_normal_split_a_flow_built_from_the_frame():
    """w = dmu (u b1 + v b2 + n eta) per pixel gives tangent (u, v) and normal n."""
    rng = np.random.default_rng(11)
    u, v, n = (rng.normal(size=(9, 11)) for _ in range(3))
    f, g = _filter_with_w(lambda g: g.dmu[..., None] * (u[..., None] * g.b1 + v[..., None] * g.b2
                                                         + n[..., None] * g.eta))
    t = f.flow("tangent_px")
    assert t.shape == (9, 11, 2)
    np.testing.assert_allclose(t[..., 0], u, atol=1e-12)
    np.testing.assert_allclose(t[..., 1], v, atol=1e-12)
    np.testing.assert_allclose(f.flow("normal_px"), n, atol=1e-12)


def test_pure_b1_and_pure_eta_flows():
    """Flow along b1 alone is all first tangent component; flow along eta alone is all
    normal component (the projector removes it from the tangent flow)."""
    f, g = _filter_with_w(lambda g: 0.7 * g.dmu[..., None] * g.b1)
    t = f.flow("tangent_px")
    np.testing.assert_allclose(t[..., 0], 0.7, atol=1e-12)
    np.testing.assert_allclose(t[..., 1], 0.0, atol=1e-12)
    np.testing.assert_allclose(f.flow("normal_px"), 0.0, atol=1e-12)
    f, g = _filter_with_w(lambda g: 0.3 * g.eta)
    np.testing.assert_allclose(f.flow("tangent_px"), 0.0, atol=1e-12)
    np.testing.assert_allclose(f.flow("normal_px"), 0.3 / g.dmu, atol=1e-12)


def test_principal_pixel_hand_values():
    """At the principal pixel eta = (0, 0, 1), b1 = x, b2 = y and dmu = 1/sqrt(fx^2 + 1)
    (the next column's ray (1/fx, 0, 1) normalised, projected).  A static point at inverse
    depth rho seen by a camera translating with velocity v has w = -rho v
    (eq:homogeneous_flow), so the tangent flow is -rho (vx, vy) sqrt(fx^2 + 1) and the normal
    flow -rho vz sqrt(fx^2 + 1) pixels per frame; the rad/s output is w / dt."""
    fx, rho, vel = 30.0, 0.4, np.array([0.02, -0.05, 0.03])
    f, g = _filter_with_w(lambda g: np.broadcast_to(-rho * vel, (9, 11, 3)).copy(),
                          fx=fx, cx=5.0, cy=4.0)
    s = math.sqrt(fx * fx + 1.0)
    t = f.flow("tangent_px")[4, 5]
    np.testing.assert_allclose(t, [-rho * vel[0] * s, -rho * vel[1] * s], rtol=1e-12)
    np.testing.assert_allclose(f.flow("normal_px")[4, 5], -rho * vel[2] * s, rtol=1e-12)
    np.testing.assert_allclose(f.flow("w_rad_s")[4, 5], -rho * vel / 0.25, rtol=1e-12)


def test_rho_output_is_the_state():
    rho = np.linspace(0.1, 0.9, 99).reshape(9, 11)
    f, _ = _filter_with_w(lambda g: np.zeros((9, 11, 3)), rho=rho)
    np.testing.assert_array_equal(f.flow("rho"), rho)


@pytest.mark.parametrize("a,b,deg", [
    ((1.0, 0.0, 0.0), (1.0, 0.0, 0.0), 0.0),
    ((1.0, 0.0, 0.0), (0.0, 0.0, 0.0), 45.0),     # (1,0,0,1).(0,0,0,1) = 1 over sqrt(2)
    ((1.0, 0.0, 0.0), (0.0, 1.0, 0.0), 60.0),     # 1 / (sqrt 2 sqrt 2) = cos 60
    ((1.0, 0.0, 0.0), (-1.0, 0.0, 0.0), 90.0),    # 1 - 1 = 0
    ((0.0, 0.0, 0.0), (0.0, 0.0, math.sqrt(3.0)), 60.0),   # 1 / 2
])
def test_aae_hand_values(a, b, deg):
    """Angle between (a, 1) and (b, 1) in 4-D, a and b in pixels (w / dmu).  The tolerance
    is arccos's conditioning at 0 degrees: a cosine rounded by 1 ulp below 1 is an angle of
    sqrt(2 * 2^-53) rad, about 1e-6 degrees."""
    dmu = np.full((2, 3), 0.01)
    wa = np.broadcast_to(np.array(a) * 0.01, (2, 3, 3))
    wb = np.broadcast_to(np.array(b) * 0.01, (2, 3, 3))
    assert abs(aae_deg(wa, wb, dmu) - deg) < 1e-5
    assert abs(aae_deg(wb, wa, dmu) - deg) < 1e-5


def test_aae_is_a_mean_over_pixels():
    dmu = np.ones((1, 2))
    wa = np.array([[[1.0, 0, 0], [1.0, 0, 0]]])
    wb = np.array([[[1.0, 0, 0], [-1.0, 0, 0]]])
    assert abs(aae_deg(wa, wb, dmu) - 45.0) < 1e-5


def test_epe_hand_values():
    """|wa - wb| / dmu per pixel: a 3-4-5 triangle over dmu = 0.5 is 10 px."""
    dmu = np.array([[0.5, 1.0]])
    wa = np.array([[[3.0, 4.0, 0.0], [0.0, 0.0, 2.0]]])
    wb = np.zeros_like(wa)
    np.testing.assert_allclose(epe_field(wa, wb, dmu), [[10.0, 2.0]])
    s = epe_stats(wa, wb, dmu)
    assert s["mean"] == 6.0 and s["max"] == 10.0
