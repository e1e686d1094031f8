"""Pins for the oracle's spherical-grid geometry (Section "Spherical image data structure")."""
import numpy as np
import pytest

from oracle import geometry


CAMS = [(64, 64, 64.0, 64.0, 31.5, 31.5), (37, 53, 40.0, 35.0, 20.3, 17.9),
        (8, 8, 9.0, 9.0, 3.5, 3.5)]


@pytest.mark.parametrize("cam", CAMS)
def test_basis_orthonormal_and_tangent(cam):
    R, C, fx, fy, cx, cy = cam
    eta = geometry.pinhole_eta(R, C, fx, fy, cx, cy)
    b1, b2, dmu = geometry.tangent_frame(eta)
    np.testing.assert_allclose(np.linalg.norm(eta, axis=-1), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(b1, axis=-1), 1.0, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(b2, axis=-1), 1.0, atol=1e-13)
    assert np.abs(np.sum(b1 * b2, -1)).max() < 1e-13
    assert np.abs(np.sum(b1 * eta, -1)).max() < 1e-13
    assert np.abs(np.sum(b2 * eta, -1)).max() < 1e-13
    assert (dmu > 0).all()


@pytest.mark.parametrize("cam", CAMS)
def test_pinhole_closed_form(cam):
    """For a pinhole grid, P_eta eta_{i,j+1} is parallel to P_eta e_x (the next column's ray
    differs from eta's by e_x/fx before normalisation), so b1 = normalize(e_x - eta eta_x)
    and dmu = sqrt(1 - eta_x^2) / (fx |r_{i,j+1}|) with r the unnormalised ray; the last
    column uses r_{i,j-1} and the same b1.  b2 = eta x b1 points toward +y."""
    R, C, fx, fy, cx, cy = cam
    eta = geometry.pinhole_eta(R, C, fx, fy, cx, cy)
    b1, b2, dmu = geometry.tangent_frame(eta)
    ex = np.array([1.0, 0.0, 0.0])
    q = ex - eta * eta[..., :1]
    b1_ref = q / np.linalg.norm(q, axis=-1, keepdims=True)
    np.testing.assert_allclose(b1, b1_ref, atol=1e-12)
    jn = np.arange(C) + 1.0
    jn[-1] = C - 2.0
    x = (jn[None, :] - cx) / fx
    y = (np.arange(R)[:, None] - cy) / fy
    rn = np.sqrt(x * x + y * y + 1.0)
    dmu_ref = np.sqrt(1.0 - eta[..., 0] ** 2) / (fx * rn)
    np.testing.assert_allclose(dmu, dmu_ref, rtol=1e-10)
    b2_ref = np.cross(eta, b1_ref)
    np.testing.assert_allclose(b2, b2_ref, atol=1e-12)
    assert (b2[..., 1] > 0).all()


def test_levels_subsample_the_finest_grid():
    R, C, fx, fy, cx, cy = 37, 53, 40.0, 35.0, 20.3, 17.9
    g1 = geometry.Grid(R, C, fx, fy, cx, cy, 1)
    for h in (2, 3, 4):
        gh = geometry.Grid(R, C, fx, fy, cx, cy, h)
        s = 2 ** (h - 1)
        assert (gh.rows, gh.cols) == (-(-R // s), -(-C // s))
        np.testing.assert_allclose(gh.eta, g1.eta[::s, ::s], atol=1e-15)


def test_needs_two_columns():
    eta = geometry.pinhole_eta(4, 1, 4.0, 4.0, 0.0, 1.5)
    with pytest.raises(ValueError):
        geometry.tangent_frame(eta)
