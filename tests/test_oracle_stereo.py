"""Pins for the oracle's inverse depth from a rectified stereo pair (oracle/stereo.py)."""
import numpy as np

from oracle import stereo


def _texture(R, C, shift=0.0, seed=0):
    """A smooth random texture sampled at columns j + shift (several sinusoids)."""
    rng = np.random.default_rng(seed)
    j = np.arange(C, dtype=np.float64)[None, :] + shift
    i = np.arange(R, dtype=np.float64)[:, None]
    out = np.zeros((R, C))
    for _ in range(8):
        fj, fi = rng.uniform(0.05, 0.2), rng.uniform(0.02, 0.15)
        out += rng.uniform(0.2, 1.0) * np.sin(2 * np.pi * (fj * j + fi * i) + rng.uniform(0, 6))
    return 0.5 + 0.08 * out


def test_integer_shift_is_found_exactly():
    """Y_R(i, j) = Y_L(i, j + d0): block matching finds d0 with zero cost and the refinement
    keeps it, where the window stays inside both images."""
    rng = np.random.default_rng(2)
    R, C, d0 = 30, 60, 5
    big = rng.random((R, C + d0))
    YL = big[:, :C]
    YR = big[:, d0:C + d0]
    d = stereo.block_match(YL, YR, 12)
    inner = (slice(2, -2), slice(d0 + 2, -2))
    assert np.all(d[inner] == d0)
    dr, _, E = stereo.disparity(YL, YR, 12)
    np.testing.assert_allclose(dr[inner], d0, atol=1e-9)
    assert np.all(E[inner] < 1e-12)


def test_fractional_shift_converges():
    """A smooth texture shifted by a fraction of a pixel: the refinement lands within 0.02 px."""
    R, C = 30, 80
    for d0 in (3.4, 6.75):
        YL = _texture(R, C, 0.0, seed=3)
        YR = _texture(R, C, d0, seed=3)       # Y_R(j) = texture(j + d0) = Y_L(j + d0)
        d, A, _ = stereo.disparity(YL, YR, 12)
        inner = (slice(3, -3), slice(12, -3))
        assert np.median(np.abs(d[inner] - d0)) < 0.02
        assert np.percentile(np.abs(d[inner] - d0), 95) < 0.1


def test_plane_at_known_depth():
    """A fronto-parallel textured plane at depth Z, rendered into both cameras: the measured
    inverse range equals eta_z / Z (to a per cent in the median)."""
    from synth.scenes import Camera, SinusoidPlaneScene, Sequence, Trajectory
    R, C, f, Z, b = 48, 64, 60.0, 4.0, 0.2
    cam = Camera(R, C, f, f, (C - 1) / 2, (R - 1) / 2)
    scene = SinusoidPlaneScene(np.array([0.0, 0.0, 1.0]), Z, 8, np.random.default_rng(4))
    seq = Sequence(cam, scene, Trajectory(V=np.zeros(3)), 1.0, 1)
    fr = seq.frame(0)
    YL, rho_true = fr.Y.numpy(), fr.rho_true.numpy()
    YR = seq.right_image(0, b).numpy()
    rho = stereo.stereo_rho(YL, YR, f, f, cam.cx, cam.cy, b, 12)
    ok = ~np.isnan(rho)
    assert ok.mean() > 0.7
    rel = np.abs(rho[ok] - rho_true[ok]) / rho_true[ok]
    assert np.median(rel) < 0.01


def test_textureless_image_gives_no_measurement():
    YL = np.full((20, 30), 0.4)
    rho = stereo.stereo_rho(YL, YL.copy(), 30.0, 30.0, 14.5, 9.5, 0.1, 8)
    assert np.all(np.isnan(rho))


def test_rendered_box_scene():
    """The 256x256 box scene seen by a stereo pair (baseline 0.2 m; disparities 0.5-5 px):
    nearly every pixel gets a measurement, and its disparity (kappa rho) is within a fraction
    of a pixel of the true one (the far enclosure's texture is finer than a pixel, which bounds
    the sub-pixel accuracy); with the right image taken from the wrong side almost none is."""
    from synth.scenes import box_sequence
    S, b = 256, 0.2
    seq = box_sequence(S, S, 1, seed=6, max_flow_px=8.0)
    c = seq.camera
    fr = seq.frame(0)
    YL, rt = fr.Y.numpy(), fr.rho_true.numpy()
    k = stereo.kappa(S, S, c.fx, c.fy, c.cx, c.cy, b)
    dmax = int(np.ceil((k * rt).max() * 1.2)) + 2
    res = {}
    for side in (b, -b):
        rho = stereo.stereo_rho(YL, seq.right_image(0, side).numpy(), c.fx, c.fy, c.cx, c.cy, b,
                                dmax)
        ok = ~np.isnan(rho)
        err = np.abs(k[ok] * (rho[ok] - rt[ok]))
        res[side] = (ok.mean(), np.median(err), np.mean(err < 0.5))
    assert res[b][0] > 0.8 and res[b][1] < 0.2 and res[b][2] > 0.75, res
    assert res[-b][2] < 0.1, res
