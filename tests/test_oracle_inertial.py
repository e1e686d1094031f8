"""Pins for the oracle's inertial source terms: the terms of eq:hflow_conservation that the
paper drops by eq:assumption (-Omega x w + a_w, Section "State prediction"), kept when the
camera's angular velocity and linear acceleration are given.

The pins are exact solutions of the kinematics of Section "Structure Flow" (eq:camvel_dot,
eq:totaldev_ppos, eq:homogeneous_flow), built here from rigid motion, not from the PDE: a
camera rotating inside a sphere (a stationary field), and a textured plane seen by a camera
that rotates, translates and accelerates.  Predicting one frame from the exact fields must
land near the exact fields one frame later with the terms, and miss by the size of the
dropped terms without them."""
import numpy as np
import pytest

from oracle import Filter, geometry, predict
from oracle.literal import LiteralFilter
from oracle.metrics import epe_field
from oracle.readings import Readings


def _skew(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def _rotation(w):
    """exp([w]x) by Rodrigues' formula."""
    th = float(np.linalg.norm(w))
    K = _skew(w)
    if th < 1e-15:
        return np.eye(3) + K
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * K @ K


def _plane_fields(g, n0, d0, V, A, om, t):
    """Exact fields at time t (frames) of the static plane n0 . x = d0 (world frame, which is
    the camera frame at t = 0) for a camera with constant body angular velocity om, position
    V t + A t^2 / 2 and so velocity V + A t in the world: the camera-to-world rotation is
    exp(t [om]x), a ray eta meets the plane at range d / (n . eta) with n the plane normal in
    the camera frame and d the camera's distance to the plane, and the structure flow of a
    static point is -om x eta - rho v with v the camera's velocity in its own frame."""
    Rt = _rotation(om * t)
    c = V * t + 0.5 * A * t * t
    n = Rt.T @ n0
    d = d0 - n0 @ c
    rho = (g.eta @ n) / d
    v = Rt.T @ (V + A * t)
    w = -np.cross(om, g.eta) - rho[..., None] * v
    return w, rho


def _grid(R):
    return geometry.Grid(R, R, R, R, (R - 1) / 2, (R - 1) / 2, 1)


def test_pure_rotation_inside_a_sphere_is_stationary():
    """A camera rotating at the centre of a sphere sees w = -Omega x eta and a constant rho at
    all times.  With the inertial terms the prediction keeps that field (up to the upwind
    scheme's discretisation error); without them it drifts by -Omega x (Omega x eta) per
    frame."""
    R = 48
    g = _grid(R)
    om = np.array([0.01, -0.015, 0.02])       # rad/frame: about a pixel per frame
    w0 = -np.cross(om, g.eta)
    rho = np.full((R, R), 0.2)
    inner = (slice(4, -4), slice(4, -4))
    drift = np.abs(np.cross(om, np.cross(om, g.eta)))[inner].max()
    for N in (2, 4, 8):
        kept = predict.predict(g, {"w": w0, "rho": rho}, N, Readings(),
                               (om, np.zeros(3), np.zeros(3)))
        plain = predict.predict(g, {"w": w0, "rho": rho}, N, Readings())
        assert np.abs(kept["w"] - w0)[inner].max() < 0.1 * drift
        moved = (plain["w"] - w0)[inner]
        want = -np.cross(om, np.cross(om, g.eta))[inner]
        assert np.abs(moved).max() > 0.8 * drift
        assert np.abs(moved - want).max() < 0.25 * drift


@pytest.mark.parametrize("case", ["accelerating", "rotating", "both"])
def test_plane_under_rotation_and_acceleration(case):
    """One frame of prediction from the exact plane fields against the exact fields one frame
    later, relative to the change over that frame: within a few per cent with the inertial
    terms, off by the order of the change itself without them.  The accelerating case fixes
    the sign of the acceleration term (the printed field acceleration has +rho a; with that
    sign the error doubles instead of vanishing)."""
    n0 = np.array([0.1, -0.3, 1.0])
    n0 /= np.linalg.norm(n0)
    V = {"accelerating": np.array([0.002, 0.001, 0.01])}.get(case, np.array([0.004, 0.002, 0.03]))
    A = np.zeros(3) if case == "rotating" else np.array([0.0005, -0.0003, 0.004])
    om = np.zeros(3) if case == "accelerating" else np.array([0.01, 0.02, -0.005])
    bound = {"accelerating": 0.01, "rotating": 0.15, "both": 0.05}[case]
    R = 48
    g = _grid(R)
    w0, r0 = _plane_fields(g, n0, 2.0, V, A, om, 0.0)
    w1, r1 = _plane_fields(g, n0, 2.0, V, A, om, 1.0)
    # the acceleration in the camera frame at mid-interval (it turns with the camera)
    imu = (om, np.zeros(3), _rotation(0.5 * om).T @ A)
    inner = (slice(4, -4), slice(4, -4))
    change = np.abs(w1 - w0)[inner].max()
    for N in (2, 4, 8):
        kept = predict.predict(g, {"w": w0, "rho": r0}, N, Readings(), imu)
        plain = predict.predict(g, {"w": w0, "rho": r0}, N, Readings())
        assert np.abs(kept["w"] - w1)[inner].max() < bound * change
        assert np.abs(plain["w"] - w1)[inner].max() > 0.9 * change
        flipped = predict.predict(g, {"w": w0, "rho": r0}, N, Readings(), (om, imu[1], -imu[2]))
        if case == "accelerating":
            assert np.abs(flipped["w"] - w1)[inner].max() > 1.5 * change


def test_angular_acceleration_about_a_fixed_axis():
    """A camera whose angular velocity grows along a fixed axis, Omega(t) = (w0 + al t) n, so
    that its attitude is exp((w0 t + al t^2 / 2) [n]x) exactly, in front of a plane while it
    translates.  The structure flow -Omega(t) x eta - rho v changes with Omega itself: with the
    angular acceleration the prediction lands near the exact fields one frame later, with
    Omega alone (the paper's constant-rate kinematics, eq:totaldev_camangvel) it misses by the
    -dOmega x eta of the frame."""
    n0 = np.array([0.1, -0.3, 1.0])
    n0 /= np.linalg.norm(n0)
    V = np.array([0.004, 0.002, 0.03])
    axis = np.array([0.3, 1.0, -0.2])
    axis /= np.linalg.norm(axis)
    w0, al = 0.01, 0.006                      # rad/frame, rad/frame^2
    R = 48
    g = _grid(R)

    def fields(t):
        Rt = _rotation(axis * (w0 * t + 0.5 * al * t * t))
        n = Rt.T @ n0
        rho = (g.eta @ n) / (2.0 - n0 @ (V * t))
        om = axis * (w0 + al * t)
        return -np.cross(om, g.eta) - rho[..., None] * (Rt.T @ V), rho

    wa, ra = fields(0.0)
    wb, _ = fields(1.0)
    om_mid = axis * (w0 + 0.5 * al)
    inner = (slice(4, -4), slice(4, -4))
    change = np.abs(wb - wa)[inner].max()
    with_dom = predict.predict(g, {"w": wa, "rho": ra}, 8, Readings(),
                               (om_mid, axis * al, np.zeros(3)))
    without = predict.predict(g, {"w": wa, "rho": ra}, 8, Readings(),
                              (om_mid, np.zeros(3), np.zeros(3)))
    e_with = np.abs(with_dom["w"] - wb)[inner].max()
    e_without = np.abs(without["w"] - wb)[inner].max()
    assert e_with < 0.15 * change
    assert e_without > 3.0 * e_with


def test_zero_rates_give_the_plain_prediction():
    rng = np.random.default_rng(3)
    g = _grid(16)
    fields = {"w": 1e-3 * rng.standard_normal((16, 16, 3)),
              "dw": 1e-4 * rng.standard_normal((16, 16, 3)),
              "rho": 0.2 + rng.random((16, 16)), "Y": rng.random((16, 16))}
    a = predict.predict(g, fields, 3, Readings(), (np.zeros(3), np.zeros(3), np.zeros(3)))
    b = predict.predict(g, fields, 3, Readings())
    for k in fields:
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("R,C,H,mf,sm", [(8, 8, 1, 2.0, [2]), (8, 8, 3, 4.0, [1, 2, 2])])
def test_vectorised_equals_per_pixel_literal_with_inertial_terms(R, C, H, mf, sm):
    """The per-pixel loop version (cross products by components, the double cross product by
    the vector triple product identity) agrees with the vectorised oracle."""
    rng = np.random.default_rng(R + 10 * H)
    cam = (R * 1.1, R * 1.1, (C - 1) / 2 + 0.3, (R - 1) / 2 - 0.2)
    a = Filter(R, C, H, mf, sm, *cam)
    b = LiteralFilter(R, C, H, mf, sm, *cam)
    om = np.array([3.0, -2.0, 5.0])           # rad/s, with dt = 0.01: 0.03-0.05 rad/frame
    dom = np.array([-20.0, 35.0, 10.0])       # rad/s^2
    acc = np.array([40.0, 10.0, -30.0])       # m/s^2
    for k in range(4):
        Y = rng.random((R, C))
        rho = 0.2 + rng.random((R, C))
        rho[rng.random((R, C)) < 0.1] = np.nan
        a.push(Y, rho, 0.01, omega=om, acc=acc, omega_dot=dom)
        b.push(Y, rho, 0.01, omega=om, acc=acc, omega_dot=dom)
        np.testing.assert_allclose(a.flow("w_frame"), b.flow("w_frame"), atol=1e-12)
        for h in range(H):
            np.testing.assert_allclose(a.state[h]["rho"], b.state[h]["rho"], atol=1e-12)


def test_inertial_terms_lower_the_error_under_rotation():
    """A box scene whose image motion is mostly from camera rotation (80 %): the filter with
    the inertial terms (the renderer's angular velocity and its rate of change at
    mid-interval; the inertial velocity is constant, so the acceleration is zero) ends closer
    to the true flow."""
    from synth.scenes import box_sequence, render_sequence
    seq = box_sequence(96, 96, 16, seed=5, max_flow_px=4.0, rot_share=0.8)
    Y, rho, W = render_sequence(seq)
    c = seq.camera
    err = {}
    for use in (False, True):
        f = Filter(96, 96, 2, 4.0, [2, 4], c.fx, c.fy, c.cx, c.cy)
        e = []
        for k in range(seq.n_frames):
            if use and k > 0:
                om, dom, acc = seq.imu(k)
                f.push(Y[k], rho[k], seq.dt, omega=om, omega_dot=dom, acc=acc)
            else:
                f.push(Y[k], rho[k], seq.dt)
            if k >= 6:
                e.append(epe_field(f.flow("w_frame"), W[k] * seq.dt, f.grids[0].dmu).mean())
        err[use] = float(np.mean(e))
    assert err[True] < 0.95 * err[False], err
