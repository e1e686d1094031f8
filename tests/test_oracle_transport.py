"""Pins for the oracle's numerical prediction (Section "Numerical prediction")."""
import numpy as np
import pytest

from oracle import geometry, predict
from oracle.readings import Readings


def _grid(R=6, C=40, f=40.0):
    return geometry.Grid(R, C, f, f, (C - 1) / 2.0, (R - 1) / 2.0, 1)


def _tangent_w(g, u_px):
    """A tangent flow field with column optical flow u_px (pixels per frame) everywhere."""
    return (u_px * g.dmu)[..., None] * g.b1


def test_constant_image_is_preserved_exactly():
    g = _grid()
    rng = np.random.default_rng(0)
    w = 0.05 * rng.standard_normal((g.rows, g.cols, 3))
    Y = np.full((g.rows, g.cols), 0.375)
    out = predict.predict(g, {"w": w, "dw": np.zeros_like(w), "rho": np.ones_like(Y), "Y": Y},
                          4, Readings())
    assert np.array_equal(out["Y"], Y)


def test_integer_cfl_shift_is_exact():
    """With |u_hat| dt = 1 the upwind step is an exact one-pixel translation: a field that
    only varies along the columns moves N pixels in one frame (row passes see D = 0)."""
    g = _grid()
    N = 4
    # u = 1.5 N everywhere, clamped to N: every column step moves exactly one pixel
    w = _tangent_w(g, np.full((g.rows, g.cols), 1.5 * N))
    prof = np.random.default_rng(1).random(g.cols)
    Y = np.tile(prof, (g.rows, 1))
    out = predict.predict(g, {"w": w, "Y": Y, "dw": np.zeros_like(w), "rho": np.zeros_like(Y)},
                          N, Readings())
    np.testing.assert_allclose(out["Y"][:, N:], Y[:, :-N], atol=1e-15)
    np.testing.assert_allclose(out["Y"][:, :N], prof[0], atol=1e-15)   # inflow border held


def _box_shift(readings, u=5.0, N=5):
    g = _grid(R=4, C=60, f=60.0)
    mask = np.zeros((g.rows, g.cols))
    mask[:, 15:25] = 1.0
    w = _tangent_w(g, u * mask)
    Y = 0.2 + 0.6 * mask
    out = predict.predict(g, {"w": w, "Y": Y, "dw": np.zeros_like(w), "rho": np.zeros_like(Y)},
                          N, readings)
    prof = out["Y"][1] - 0.2
    return float(np.sum(prof * np.arange(g.cols)) / np.sum(prof)) - 19.5


def test_dominant_flow_reading_carries_moving_edges():
    """Reading of the dominant optical flow: the text's 'largest component' transports a
    moving box by its velocity; the printed case split never moves it."""
    assert abs(_box_shift(Readings()) - 5.0) < 0.5
    assert abs(_box_shift(Readings(dominant_literal=True))) < 1e-12


def test_max_principle_with_cfl_clamp():
    """With the clamp, each pass is a convex combination of a value and one neighbour, so the
    unsourced image stays within its initial range whatever the flow."""
    g = _grid(R=12, C=12, f=12.0)
    rng = np.random.default_rng(2)
    w = 3.0 * rng.standard_normal((12, 12, 3))
    Y = rng.random((12, 12))
    out = predict.predict(g, {"w": w, "Y": Y, "dw": np.zeros_like(w), "rho": np.zeros_like(Y)},
                          2, Readings())
    assert out["Y"].min() >= Y.min() - 1e-15 and out["Y"].max() <= Y.max() + 1e-15
    nc = predict.predict(g, {"w": w, "Y": Y, "dw": np.zeros_like(w), "rho": np.zeros_like(Y)},
                         2, Readings(cfl_clamp=False))
    assert nc["Y"].max() > Y.max() + 0.1 or nc["Y"].min() < Y.min() - 0.1


def _plane_fields(g, n, v, d):
    """Exact structure flow and inverse depth of the plane n.x = d seen by a camera moving with
    velocity v (no rotation): rho = n.eta / d, w = -rho v (eq:homogeneous_flow)."""
    rho = (g.eta @ n) / d
    return -rho[..., None] * v, rho


@pytest.mark.parametrize("sigma_literal", [False, True])
def test_analytic_plane_prediction_converges(sigma_literal):
    """The plane flow with d(t) = d0 - (n.v) t solves the source-free structure-flow and
    inverse-depth PDEs exactly.  Predicting one frame from the exact fields must approach the
    exact fields at t + 1 as N grows (first order), and the half-source reading must be the
    accurate one."""
    n = np.array([0.1, -0.3, 1.0])
    n /= np.linalg.norm(n)
    v = np.array([0.004, 0.002, 0.03])       # m per frame, mostly forward
    d0 = 2.0
    errs = []
    for R, N in ((48, 1), (48, 2), (48, 4), (48, 8)):
        g = geometry.Grid(R, R, R, R, (R - 1) / 2, (R - 1) / 2, 1)
        w0, r0 = _plane_fields(g, n, v, d0)
        w1, r1 = _plane_fields(g, n, v, d0 - n @ v)
        out = predict.predict(g, {"w": w0, "rho": r0}, N, Readings(source_literal=sigma_literal))
        inner = (slice(4, -4), slice(4, -4))
        ew = np.abs(out["w"] - w1)[inner].max() / np.abs(w1 - w0)[inner].max()
        er = np.abs(out["rho"] - r1)[inner].max() / np.abs(r1 - r0)[inner].max()
        errs.append((ew, er))
    errs = np.array(errs)
    if sigma_literal:
        # doubled source: the change over one frame is off by about 100 %
        assert errs[-1, 0] > 0.5
    else:
        assert errs[-1, 0] < 0.2 and errs[-1, 1] < 0.2
        assert errs[-1, 0] <= errs[0, 0] + 1e-12
