"""Pins for the brightness model (eq:img_model, eq:img_gradient) and the inverse-depth
model (eq:dominant_b1/b2, Table diff_operators) of the oracle."""
import json
import os

import numpy as np
import pytest

from oracle import models
from oracle.literal import _image_model

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gaussian_window_normal_matrix_is_identity():
    """With G = g g^T, g = [1,4,6,4,1]/16 (as printed under eq:img_model), the weighted
    normal matrix of the basis [1, q_j - p_j, q_i - p_i] over the 5x5 window is I."""
    fx = json.load(open(os.path.join(GOLDEN, "image_model_weights.json")))
    g = np.array(fx["g_numerators"], float) / fx["g_denominator"]
    d = np.arange(-2, 3, dtype=float)
    G = np.outer(g, g)
    basis = [np.ones((5, 5)), np.tile(d, (5, 1)), np.tile(d[:, None], (1, 5))]
    M = np.array([[np.sum(G * a * b) for b in basis] for a in basis])
    np.testing.assert_array_equal(M, np.eye(3))
    np.testing.assert_array_equal(g, models.G1D)


def test_brightness_model_equals_brute_force_weighted_ls():
    rng = np.random.default_rng(3)
    Y = rng.random((8, 9))
    Yhat, d1, d2 = models.brightness_model(Y)
    for i in range(8):
        for j in range(9):
            c, g1, g2 = _image_model(Y, i, j)
            assert abs(c - Yhat[i, j]) < 1e-12
            assert abs(g1 - d1[i, j]) < 1e-12
            assert abs(g2 - d2[i, j]) < 1e-12


def test_linear_and_quadratic_images():
    i, j = np.mgrid[0:12, 0:13].astype(float)
    Y = 0.3 + 0.05 * j - 0.02 * i
    Yhat, d1, d2 = models.brightness_model(Y)
    inner = (slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(Yhat[inner], Y[inner], atol=1e-14)
    np.testing.assert_allclose(d1[inner], 0.05, atol=1e-14)
    np.testing.assert_allclose(d2[inner], -0.02, atol=1e-14)
    # Y = j^2: Yhat = j^2 + sum G b^2 = j^2 + 1, gradient 2j (third moment vanishes)
    Yq = j ** 2
    Yhat, d1, d2 = models.brightness_model(Yq)
    np.testing.assert_allclose(Yhat[inner], Yq[inner] + 1.0, atol=1e-12)
    np.testing.assert_allclose(d1[inner], 2 * j[inner], atol=1e-12)
    np.testing.assert_allclose(d2[inner], 0.0, atol=1e-12)


def test_gradient_sign_points_uphill():
    """Reading of eq:img_model: the model offset is q - p, so brighter to the right gives a
    positive column component."""
    Y = np.tile(np.linspace(0, 1, 10), (6, 1))
    _, d1, d2 = models.brightness_model(Y)
    assert (d1[:, 2:-2] > 0).all()


def test_depth_model_hand_cases():
    cases = json.load(open(os.path.join(GOLDEN, "depth_model_cases.json")))["cases"]
    for case in cases:
        row = np.array([np.nan if v is None else v for v in case["row"]], float)
        rho = np.tile(row, (3, 1))
        _, d1, d2 = models.depth_model(rho)
        np.testing.assert_allclose(d1[1], case["d1"], atol=1e-15, err_msg=case["name"])
        np.testing.assert_allclose(d2[1], 0.0, atol=0)
        # the transposed image gives the same values along rows
        _, t1, t2 = models.depth_model(rho.T.copy())
        np.testing.assert_allclose(t2[:, 1], case["d1"], atol=1e-15, err_msg=case["name"])
