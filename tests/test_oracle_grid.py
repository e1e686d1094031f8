"""Pins for the oracle on general grids of unit directions (Section "Spherical image data
structure": the filter is written for any grid of directions on the sphere with its tangent
bases and spacing, the pinhole being one case)."""
import numpy as np
import pytest

from oracle import Filter, geometry, predict
from oracle.literal import LiteralFilter
from oracle.readings import Readings
from synth.scenes import equiangular_rays


def test_pinhole_grid_given_as_directions_equals_the_intrinsics():
    """The pinhole's own rays passed as a general grid give the same geometry at every level
    (coarser levels sample the finest grid) and the same filter results."""
    R, C, H = 37, 29, 3
    cam = (40.0, 38.0, 13.7, 18.2)
    eta1 = geometry.pinhole_eta(R, C, *cam)
    a = Filter(R, C, H, 4.0, [2, 2, 2], *cam)
    b = Filter(R, C, H, 4.0, [2, 2, 2], *cam, eta=eta1)
    for ga, gb in zip(a.grids, b.grids):
        for k in ("eta", "b1", "b2", "dmu"):
            np.testing.assert_allclose(getattr(ga, k), getattr(gb, k), atol=1e-14)
    rng = np.random.default_rng(5)
    for _ in range(3):
        Y, rho = rng.random((R, C)), 0.2 + rng.random((R, C))
        a.push(Y, rho, 0.01)
        b.push(Y, rho, 0.01)
    np.testing.assert_allclose(a.flow("w_frame"), b.flow("w_frame"), atol=1e-14)


def test_equiangular_basis_and_spacing():
    """On a longitude-latitude grid the spacing to the next column is the chord angle
    sin(angle between neighbours), the same along a row of constant latitude, and b1 lies in
    the plane spanned by the two neighbouring directions."""
    R, C = 21, 31
    eta = equiangular_rays(R, C, 120.0)
    g = geometry.Grid(R, C, 20.0, 20.0, 15.0, 10.0, 1, eta)
    cosang = np.sum(eta[:, :-1] * eta[:, 1:], axis=-1)
    np.testing.assert_allclose(g.dmu[:, :-1], np.sqrt(1 - cosang ** 2), rtol=1e-12)
    np.testing.assert_allclose(g.dmu[:, :-1], np.broadcast_to(g.dmu[:, :1], (R, C - 1)),
                               rtol=1e-12)   # constant along rows
    normal = np.cross(eta[:, :-1], eta[:, 1:])
    np.testing.assert_allclose(np.sum(normal * g.b1[:, :-1], axis=-1), 0.0, atol=1e-14)
    np.testing.assert_allclose(np.sum(g.b1 * g.b2, axis=-1), 0.0, atol=1e-14)


def _rotation(w):
    th = float(np.linalg.norm(w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    return np.eye(3) + np.sin(th) / th * K + (1.0 - np.cos(th)) / th ** 2 * K @ K


def _texture(e):
    return np.sin(9 * e[..., 0] + 2 * e[..., 1]) * np.cos(7 * e[..., 1] - 3 * e[..., 0])


@pytest.mark.parametrize("om", [(0.0, 0.03, 0.0), (0.02, -0.015, 0.01)])
def test_texture_transport_under_rotation_on_an_equiangular_grid(om):
    """A camera rotating with Omega (rad/frame) in a static textured world: the image seen
    along eta at time t is the texture at exp(t [Omega]x) eta, and the structure flow is
    -Omega x eta (with the inertial terms it is stationary).  Transporting the image one frame
    on the grid's own bases and spacings lands within a fifth of the frame's change of the
    exact image; the same fields transported with the pinhole geometry of the same nominal
    resolution, or on the mirrored grid, do not."""
    om = np.asarray(om)
    R = 64
    eta = equiangular_rays(R, R, 100.0)
    Y0 = _texture(eta)
    Y1 = _texture(eta @ _rotation(om).T)
    fields = {"w": -np.cross(om, eta), "dw": np.zeros((R, R, 3)), "rho": np.full((R, R), 0.2),
              "Y": Y0}
    inner = (slice(8, -8), slice(8, -8))
    change = np.abs(Y1 - Y0)[inner].max()

    def err(grid):
        out = predict.predict(grid, fields, 4, Readings(), (om, np.zeros(3), np.zeros(3)))
        return np.abs(out["Y"] - Y1)[inner].max() / change

    c = (R - 1) / 2
    assert err(geometry.Grid(R, R, R, R, c, c, 1, eta)) < 0.25
    assert err(geometry.Grid(R, R, 35.0, 35.0, c, c, 1)) > 0.3
    assert err(geometry.Grid(R, R, R, R, c, c, 1, np.ascontiguousarray(eta[:, ::-1]))) > 1.0


def test_analytic_plane_prediction_on_an_equiangular_grid():
    """The exact plane fields (rho = n.eta / d(t), w = -rho v) on a 100-degree equiangular
    grid: one frame of prediction lands within a fifth of the frame's change of the exact
    fields one frame later, for every number of steps."""
    n = np.array([0.1, -0.3, 1.0])
    n /= np.linalg.norm(n)
    v = np.array([0.004, 0.002, 0.03])
    d0 = 2.0
    R = 48
    eta = equiangular_rays(R, R, 100.0)
    g = geometry.Grid(R, R, R, R, (R - 1) / 2, (R - 1) / 2, 1, eta)
    r0, r1 = (eta @ n) / d0, (eta @ n) / (d0 - n @ v)
    w0, w1 = -r0[..., None] * v, -r1[..., None] * v
    inner = (slice(4, -4), slice(4, -4))
    for N in (1, 2, 4, 8):
        out = predict.predict(g, {"w": w0, "rho": r0}, N, Readings())
        assert np.abs(out["w"] - w1)[inner].max() < 0.2 * np.abs(w1 - w0)[inner].max()
        assert np.abs(out["rho"] - r1)[inner].max() < 0.2 * np.abs(r1 - r0)[inner].max()


@pytest.mark.parametrize("R,C,H", [(8, 8, 1), (8, 8, 3), (9, 7, 2)])
def test_vectorised_equals_per_pixel_literal_on_an_equiangular_grid(R, C, H):
    rng = np.random.default_rng(R * 10 + H)
    eta = equiangular_rays(R, C, 110.0)
    cam = (4.0, 4.0, (C - 1) / 2, (R - 1) / 2)
    a = Filter(R, C, H, 2.0 * H, [2] * H, *cam, eta=eta)
    b = LiteralFilter(R, C, H, 2.0 * H, [2] * H, *cam, eta=eta)
    for k in range(4):
        Y = rng.random((R, C))
        rho = 0.2 + rng.random((R, C))
        rho[rng.random((R, C)) < 0.1] = np.nan
        a.push(Y, rho, 0.01)
        b.push(Y, rho, 0.01)
        np.testing.assert_allclose(a.flow("w_frame"), b.flow("w_frame"), atol=1e-12)
        for h in range(H):
            np.testing.assert_allclose(a.state[h]["rho"], b.state[h]["rho"], atol=1e-12)


def test_static_scene_on_an_equiangular_grid_gives_zero_flow():
    R, C = 24, 32
    eta = equiangular_rays(R, C, 120.0)
    rng = np.random.default_rng(9)
    Y, rho = rng.random((R, C)), 0.2 + rng.random((R, C))
    f = Filter(R, C, 2, 3.0, [2, 2], 15.0, 15.0, 15.5, 11.5, eta=eta)
    for _ in range(4):
        f.push(Y, rho, 0.01)
        assert np.all(f.flow("w_frame") == 0.0)
