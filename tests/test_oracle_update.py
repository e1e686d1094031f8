"""Pins for the oracle's update (eq:LS_update, smoothing, eq:cost_invdepth) and for the
pyramid and reconstruction (eq:hflow_reconstruction)."""
import numpy as np

from oracle import geometry, pyramid, update


def _rand_terms(rng, n=50):
    g = geometry.Grid(5, 10, 8.0, 8.0, 4.5, 2.0, 1)
    gradY = rng.standard_normal((5, 10, 3)) * 0.1
    gradR = rng.standard_normal((5, 10, 3)) * 0.01
    Ynew, Yprev = rng.random((5, 10)), rng.random((5, 10))
    rnew = 0.2 + rng.random((5, 10))
    rnew[0, :3] = np.nan
    rprev = 0.2 + rng.random((5, 10))
    return g, update.ls_terms(g, gradY, Ynew, Yprev, gradR, rnew, rprev)


def test_solution_minimises_the_cost():
    """The solution is a stationary point of the quadratic cost: its gradient vanishes, and
    small perturbations only increase the cost."""
    rng = np.random.default_rng(0)
    g, (aY, cY, ar, cr, valid) = _rand_terms(rng)
    x0 = rng.standard_normal((5, 10, 3)) * 0.01
    g1, g2, g3 = 7.0, 3.0, 0.5
    x = update.ls_solve(aY, cY, ar, cr, valid, x0, g1, g2, g3)
    g2p = np.where(valid, g2, 0.0)

    def cost(z):
        eY = np.sum(aY * z, -1) + cY
        er = np.sum(ar * z, -1) + cr
        return g1 * eY ** 2 + g2p * er ** 2 + g3 * np.sum((z - x0) ** 2, -1)

    eY = np.sum(aY * x, -1) + cY
    er = np.sum(ar * x, -1) + cr
    grad = 2 * (g1 * eY[..., None] * aY + (g2p * er)[..., None] * ar + g3 * (x - x0))
    assert np.abs(grad).max() < 1e-12
    c0 = cost(x)
    for _ in range(5):
        dz = rng.standard_normal(x.shape) * 1e-4
        assert (cost(x + dz) >= c0 - 1e-18).all()


def test_no_data_returns_the_prior():
    rng = np.random.default_rng(1)
    g, terms = _rand_terms(rng)
    x0 = rng.standard_normal((5, 10, 3))
    x = update.ls_solve(*terms, x0, 0.0, 0.0, 2.0)
    np.testing.assert_array_equal(x, x0)


def test_single_data_term_matches_sherman_morrison():
    """With only the image term the system is g3 I + g1 a a^T, whose inverse gives
    x = x0 - a (a.x0 + c) / (|a|^2 + g3/g1); as g3 -> 0 this is the minimum-norm
    correction of x0 along a."""
    rng = np.random.default_rng(2)
    g, (aY, cY, ar, cr, valid) = _rand_terms(rng)
    x0 = rng.standard_normal((5, 10, 3)) * 0.01
    for g3 in (0.3, 1e-4):
        x = update.ls_solve(aY, cY, ar, cr, valid, x0, 1.0, 0.0, g3)
        ref = x0 - aY * ((np.sum(aY * x0, -1) + cY) / (np.sum(aY * aY, -1) + g3))[..., None]
        np.testing.assert_allclose(x, ref, rtol=1e-9, atol=1e-13)


def test_missing_depth_drops_the_depth_term():
    rng = np.random.default_rng(3)
    g, (aY, cY, ar, cr, valid) = _rand_terms(rng)
    x0 = rng.standard_normal((5, 10, 3)) * 0.01
    with_d = update.ls_solve(aY, cY, ar, cr, valid, x0, 1.0, 5.0, 0.3)
    without = update.ls_solve(aY, cY, ar, cr, valid, x0, 1.0, 0.0, 0.3)
    np.testing.assert_array_equal(with_d[~valid], without[~valid])
    assert np.abs(with_d[valid] - without[valid]).max() > 0


def test_box_filter_preserves_constants_and_linear_fields():
    x = np.full((9, 11, 3), 0.7)
    np.testing.assert_allclose(update.smooth(x, 3), 0.7, atol=1e-15)
    i, j = np.mgrid[0:9, 0:11].astype(float)
    lin = np.stack([i, j, i + 2 * j], -1)
    out = update.box5(lin)
    np.testing.assert_allclose(out[2:-2, 2:-2], lin[2:-2, 2:-2], atol=1e-13)


def test_rho_update_weights():
    rn = np.array([[1.0, np.nan]])
    rp = np.array([[3.0, 5.0]])
    out = update.rho_update(rn, rp, 1.0, 3.0)
    np.testing.assert_allclose(out, [[(1 + 9) / 4.0, 5.0]])


def test_pyramid_downsample():
    i, j = np.mgrid[0:13, 0:10].astype(float)
    Y = 0.1 + 0.02 * i - 0.03 * j
    D = pyramid.downsample(Y)
    assert D.shape == (7, 5)
    np.testing.assert_allclose(D[1:-1, 1:-1], Y[::2, ::2][1:-1, 1:-1], atol=1e-14)
    # validity-normalised blur: all-valid equals the plain blur, an all-missing window is missing
    np.testing.assert_allclose(pyramid.downsample_valid(Y), D, atol=1e-15)
    rho = np.full((8, 8), 0.5)
    rho[:5, :5] = np.nan
    R = pyramid.downsample_valid(rho)
    assert np.isnan(R[0, 0]) and np.isnan(R[1, 1])
    np.testing.assert_allclose(R[~np.isnan(R)], 0.5, atol=1e-15)


def test_upsample_bilinear():
    I, J = np.mgrid[0:6, 0:5].astype(float)
    W = np.stack([1 + 2 * I - J, I * 0 + 3, 0.5 * J], -1)
    up = pyramid.upsample(W, 11, 9)
    i, j = np.mgrid[0:11, 0:9].astype(float)
    ref = np.stack([1 + i - 0.5 * j, i * 0 + 3, 0.25 * j], -1)
    np.testing.assert_allclose(up, ref, atol=1e-14)
    # clamped at the far border of an even-sized fine grid
    up2 = pyramid.upsample(W, 12, 10)
    np.testing.assert_allclose(up2[11, 9], W[5, 4], atol=1e-14)
