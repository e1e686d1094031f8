"""Pins for the oracle's mapping of a camera's image and inverse depth onto a grid of
directions (oracle/mapping.py)."""
import numpy as np

from oracle import geometry, mapping
from synth.scenes import equiangular_rays


def test_the_cameras_own_rays_map_identically():
    rng = np.random.default_rng(1)
    R, C = 23, 31
    cam = (30.0, 28.0, 14.6, 11.2)
    Y = rng.random((R, C))
    rho = 0.2 + rng.random((R, C))
    rho[rng.random((R, C)) < 0.2] = np.nan
    Yg, rg = mapping.map_frame(Y, rho, geometry.pinhole_eta(R, C, *cam), *cam)
    np.testing.assert_allclose(Yg, Y, atol=1e-12)
    np.testing.assert_array_equal(np.isnan(rg), np.isnan(rho))
    np.testing.assert_allclose(rg[~np.isnan(rho)], rho[~np.isnan(rho)], atol=1e-12)


def test_affine_images_are_reproduced_inside():
    """Bilinear interpolation is exact for an image affine in the source pixel coordinates."""
    R, C = 40, 50
    cam = (45.0, 45.0, 24.5, 19.5)
    j, i = np.meshgrid(np.arange(C), np.arange(R))
    Y = 0.3 + 0.01 * j - 0.02 * i
    rho = 0.5 + 0.003 * j + 0.001 * i
    eta = equiangular_rays(30, 30, 60.0)
    u, v, ahead = mapping.source_coords(eta, *cam)
    inside = ahead & (u >= -1e-3) & (u <= C - 1 + 1e-3) & (v >= -1e-3) & (v <= R - 1 + 1e-3)
    assert inside.mean() > 0.5
    Yg, rg = mapping.map_frame(Y, rho, eta, *cam)
    np.testing.assert_allclose(Yg[inside], (0.3 + 0.01 * u - 0.02 * v)[inside], atol=1e-12)
    np.testing.assert_allclose(rg[inside], (0.5 + 0.003 * u + 0.001 * v)[inside], atol=1e-12)
    assert np.all(np.isnan(rg[~inside]))
    # outside the image the brightness is the nearest edge value
    edge = (~inside) & ahead
    uc, vc = np.clip(u, 0, C - 1), np.clip(v, 0, R - 1)
    np.testing.assert_allclose(Yg[edge], (0.3 + 0.01 * uc - 0.02 * vc)[edge], atol=1e-12)


def test_missing_depth_uses_the_valid_neighbours():
    Y = np.zeros((2, 2))
    rho = np.array([[0.2, np.nan], [0.4, 0.6]])
    # one direction at source pixel (u, v) = (0.25, 0.5): weights 0.375, 0.125, 0.375, 0.125
    cam = (10.0, 10.0, 0.0, 0.0)
    eta = np.array([[[0.025, 0.05, 1.0]]])
    eta /= np.linalg.norm(eta)
    _, rg = mapping.map_frame(Y, rho, eta, *cam)
    want = (0.375 * 0.2 + 0.375 * 0.4 + 0.125 * 0.6) / (0.375 + 0.375 + 0.125)
    np.testing.assert_allclose(rg[0, 0], want, rtol=1e-12)
    rho2 = np.array([[np.nan, np.nan], [np.nan, 0.6]])
    eta0 = np.array([[[0.0, 0.0, 1.0]]])          # exactly on pixel (0, 0)
    _, rg2 = mapping.map_frame(Y, rho2, eta0, *cam)
    assert np.isnan(rg2[0, 0])


def test_rendered_scene_mapped_onto_a_grid_matches_rendering_on_it():
    """A box scene rendered by a 480x480 pinhole camera and mapped onto a coarser, narrower
    equiangular grid agrees with the same scene rendered directly on the grid, up to the
    interpolation error (texture and depth are smooth away from edges): the median absolute
    differences are small against the images' own spread; the source mapped transposed is
    not."""
    from synth.scenes import GridCamera, box_sequence
    seq = box_sequence(480, 480, 2, seed=9, max_flow_px=4.0, hfov_deg=90.0)
    c = seq.camera
    f_pin = seq.frame(0)
    eta = equiangular_rays(96, 96, 70.0)
    seq.camera = GridCamera(96, 96, c.fx, c.fy, c.cx, c.cy, eta=eta)
    seq._eta = {}
    f_grid = seq.frame(0)
    Yg, rg = mapping.map_frame(f_pin.Y.numpy(), f_pin.rho_true.numpy(), eta, c.fx, c.fy, c.cx,
                               c.cy)
    dY = np.abs(Yg - f_grid.Y.numpy())
    dr = np.abs(rg - f_grid.rho_true.numpy())
    assert np.median(dY) < 0.05 * np.std(f_grid.Y.numpy())
    Yw, _ = mapping.map_frame(f_pin.Y.numpy().T.copy(), f_pin.rho_true.numpy().T.copy(), eta,
                              c.fx, c.fy, c.cx, c.cy)
    assert np.median(np.abs(Yw - f_grid.Y.numpy())) > 0.5 * np.std(f_grid.Y.numpy())
    assert np.nanmedian(dr) < 0.01 * np.nanmedian(f_grid.rho_true.numpy())
    assert np.isnan(rg).mean() == 0.0        # the narrower grid lies inside the camera's view
